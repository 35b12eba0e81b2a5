// Concurrency probe: an HBM-streaming kernel (9 reads + 2 writes per word) and an
// FP64 VALU-bound kernel, run back to back on one stream vs on two streams.
// All buffers hold W words; every index < W.
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdlib>

#define CK(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) { printf("HIP error %s at %d\n", hipGetErrorString(e_), __LINE__); exit(1); } } while (0)
constexpr int kT = 256;
struct Ptrs { const uint64_t *in[9]; uint64_t *out[2]; };

__global__ __launch_bounds__(kT) void hbm_k(Ptrs p, size_t W)
{
    size_t k = (size_t)blockIdx.x * kT + threadIdx.x;
    if (k >= W) return;
    uint64_t r[9];
#pragma unroll
    for (int s = 0; s < 9; s++) r[s] = p.in[s][k];
    uint64_t a0 = 0, a1 = 0;
#pragma unroll
    for (int s = 0; s < 9; s += 3) { a0 += r[s] * r[s + 1]; a1 += r[s] * r[s + 2]; }
    p.out[0][k] = a0;
    p.out[1][k] = a1;
}

__global__ __launch_bounds__(kT) void valu_k(double *o, size_t W, int iters)
{
    size_t k = (size_t)blockIdx.x * kT + threadIdx.x;
    if (k >= W) return;
    double x[8];
#pragma unroll
    for (int j = 0; j < 8; j++) x[j] = (double)(k + j) * 1e-9;
    for (int i = 0; i < iters; i++)
#pragma unroll
        for (int j = 0; j < 8; j++) x[j] = fma(x[j], 0.999999, 1e-7);
    double s = 0;
#pragma unroll
    for (int j = 0; j < 8; j++) s += x[j];
    o[k] = s;
}

int main()
{
    const size_t W = (size_t)8 << 20;  // 64 MiB per stream buffer
    uint64_t *buf[11];
    for (auto &q : buf) { CK(hipMalloc(&q, W * 8)); CK(hipMemset(q, 1, W * 8)); }
    double *vo;
    const size_t WV = (size_t)1 << 20;
    CK(hipMalloc(&vo, WV * 8));
    Ptrs p;
    for (int s = 0; s < 9; s++) p.in[s] = buf[s];
    p.out[0] = buf[9], p.out[1] = buf[10];
    hipStream_t s1, s2;
    CK(hipStreamCreateWithFlags(&s1, hipStreamNonBlocking));
    CK(hipStreamCreateWithFlags(&s2, hipStreamNonBlocking));
    hipEvent_t e0, e1, ej;
    CK(hipEventCreate(&e0)); CK(hipEventCreate(&e1)); CK(hipEventCreateWithFlags(&ej, hipEventDisableTiming));
    const unsigned gh = (unsigned)((W + kT - 1) / kT), gv = (unsigned)((WV + kT - 1) / kT);
    int iters = 400;
    auto timed = [&](int mode) {  // 0 hbm only, 1 valu only, 2 sequential, 3 two streams
        CK(hipDeviceSynchronize());
        CK(hipEventRecord(e0, s1));
        for (int r = 0; r < 10; r++) {
            if (mode == 0 || mode == 2) hbm_k<<<gh, kT, 0, s1>>>(p, W);
            if (mode == 1 || mode == 2) valu_k<<<gv, kT, 0, s1>>>(vo, WV, iters);
            if (mode == 3) {
                CK(hipEventRecord(ej, s1));
                CK(hipStreamWaitEvent(s2, ej, 0));
                valu_k<<<gv, kT, 0, s2>>>(vo, WV, iters);
                hbm_k<<<gh, kT, 0, s1>>>(p, W);
                CK(hipEventRecord(ej, s2));
                CK(hipStreamWaitEvent(s1, ej, 0));
            }
        }
        CK(hipEventRecord(e1, s1));
        CK(hipEventSynchronize(e1));
        float ms;
        CK(hipEventElapsedTime(&ms, e0, e1));
        return 1e3 * ms / 10;
    };
    for (int m = 0; m < 4; m++) timed(m);
    // size the VALU kernel to about the HBM kernel's time
    const float th = timed(0);
    float tv = timed(1);
    iters = (int)(iters * th / tv);
    printf("hbm %.1f us  valu %.1f us  sequential %.1f us  two streams %.1f us\n", timed(0), timed(1), timed(2),
           timed(3));
    printf("hbm %.1f us  valu %.1f us  sequential %.1f us  two streams %.1f us\n", timed(0), timed(1), timed(2),
           timed(3));
    return 0;
}
