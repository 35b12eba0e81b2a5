// HBM streaming probe: kernels shaped like the key inner product
// (9 input streams, 2 output streams per output word pair) with 8-byte vs 16-byte
// lane accesses, plus a plain copy.  All buffers hold W words; every index < W.
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdlib>
#include <vector>

#define CK(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) { printf("HIP error %s at %d\n", hipGetErrorString(e_), __LINE__); exit(1); } } while (0)

constexpr int kT = 256;

__global__ __launch_bounds__(kT) void copy2(const uint64_t *a, uint64_t *o, size_t W)
{
    size_t k = (size_t)blockIdx.x * kT + threadIdx.x;
    if (k < W) o[k] = a[k] + 1;
}

__global__ __launch_bounds__(kT) void copy4(const ulonglong2 *a, ulonglong2 *o, size_t W2)
{
    size_t k = (size_t)blockIdx.x * kT + threadIdx.x;
    if (k < W2) { ulonglong2 v = a[k]; v.x += 1; v.y += 1; o[k] = v; }
}

// 9 streams in (in[s] + k), 2 out, W words per stream
struct Ptrs { const uint64_t *in[9]; uint64_t *out[2]; };

__global__ __launch_bounds__(kT) void ip9_2(Ptrs p, size_t W)
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

__global__ __launch_bounds__(kT) void ip9_4(Ptrs p, size_t W2)
{
    size_t k = (size_t)blockIdx.x * kT + threadIdx.x;
    if (k >= W2) return;
    ulonglong2 r[9];
#pragma unroll
    for (int s = 0; s < 9; s++) r[s] = ((const ulonglong2 *)p.in[s])[k];
    ulonglong2 a0 = {0, 0}, a1 = {0, 0};
#pragma unroll
    for (int s = 0; s < 9; s += 3) {
        a0.x += r[s].x * r[s + 1].x; a1.x += r[s].x * r[s + 2].x;
        a0.y += r[s].y * r[s + 1].y; a1.y += r[s].y * r[s + 2].y;
    }
    ((ulonglong2 *)p.out[0])[k] = a0;
    ((ulonglong2 *)p.out[1])[k] = a1;
}

template <typename F>
float time_it(F f, int reps)
{
    hipEvent_t a, b;
    CK(hipEventCreate(&a)); CK(hipEventCreate(&b));
    f();
    CK(hipDeviceSynchronize());
    CK(hipEventRecord(a));
    for (int r = 0; r < reps; r++) f();
    CK(hipEventRecord(b));
    CK(hipEventSynchronize(b));
    float ms;
    CK(hipEventElapsedTime(&ms, a, b));
    return ms / reps;
}

int main()
{
    const size_t W = (size_t)16 << 20;  // 128 MiB per stream (beyond the last-level cache)
    std::vector<uint64_t *> buf(11);
    for (auto &q : buf) { CK(hipMalloc(&q, W * 8)); CK(hipMemset(q, 1, W * 8)); }
    Ptrs p;
    for (int s = 0; s < 9; s++) p.in[s] = buf[s];
    p.out[0] = buf[9]; p.out[1] = buf[10];
    const int reps = 50;
    const unsigned g2 = (unsigned)((W + kT - 1) / kT), g4 = (unsigned)((W / 2 + kT - 1) / kT);
    float t;
    t = time_it([&] { copy2<<<g2, kT>>>(buf[0], buf[9], W); }, reps);
    printf("copy 8B lanes : %8.2f us  %7.1f GB/s\n", t * 1e3, 16.0 * W / t / 1e6);
    t = time_it([&] { copy4<<<g4, kT>>>((const ulonglong2 *)buf[0], (ulonglong2 *)buf[9], W / 2); }, reps);
    printf("copy 16B lanes: %8.2f us  %7.1f GB/s\n", t * 1e3, 16.0 * W / t / 1e6);
    t = time_it([&] { ip9_2<<<g2, kT>>>(p, W); }, reps);
    printf("ip 9r2w 8B    : %8.2f us  %7.1f GB/s\n", t * 1e3, 88.0 * W / t / 1e6);
    t = time_it([&] { ip9_4<<<g4, kT>>>(p, W / 2); }, reps);
    printf("ip 9r2w 16B   : %8.2f us  %7.1f GB/s\n", t * 1e3, 88.0 * W / t / 1e6);
    // staggered stream starts: stream s begins s * st words into its buffer; the
    // kernels read Wr = W - 11 * stmax words per stream, so every index stays < W
    const size_t stmax = 1 << 16, Wr = W - 11 * stmax;
    const size_t st_words[] = {0, 8, 32, 128, 256, 512, 1024, 4096, 8192, 65536};
    for (size_t st : st_words) {
        Ptrs q;
        for (int s = 0; s < 9; s++) q.in[s] = buf[s] + s * st;
        q.out[0] = buf[9] + 9 * st; q.out[1] = buf[10] + 10 * st;
        const unsigned gr = (unsigned)((Wr + kT - 1) / kT), gr4 = (unsigned)((Wr / 2 + kT - 1) / kT);
        t = time_it([&] { ip9_2<<<gr, kT>>>(q, Wr); }, reps);
        const float t4 = time_it([&] { ip9_4<<<gr4, kT>>>(q, Wr / 2); }, reps);
        printf("stagger %6zu B: 8B %7.1f GB/s   16B %7.1f GB/s\n", st * 8, 88.0 * Wr / t / 1e6, 88.0 * Wr / t4 / 1e6);
    }
    CK(hipGetLastError());
    for (auto q : buf) CK(hipFree(q));
    return 0;
}
