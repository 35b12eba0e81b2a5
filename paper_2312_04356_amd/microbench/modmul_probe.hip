// Micro-benchmark behind the arithmetic choice: HBM copy bandwidth, and the
// throughput of an exact FP64-FMA modular product versus a 64-bit Shoup product
// built from 32-bit integer multiplies, on gfx950 (q < 2^50, 8 independent chains
// per thread; a sample of results is checked against unsigned __int128 % on the host).
// Build: hipcc --offload-arch=gfx950 -O3 -Xclang -target-feature -Xclang -packed-fp32-ops \
//        -o modmul_probe modmul_probe.hip
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdint>
#include <cmath>
#include <vector>
#define CK(x) do{hipError_t e=(x); if(e!=hipSuccess){printf("HIP error %s at %d\n",hipGetErrorString(e),__LINE__); return 1;}}while(0)

__global__ void copy_k(const ulonglong2* __restrict__ a, ulonglong2* __restrict__ b, size_t n){
  size_t i = blockIdx.x*(size_t)blockDim.x+threadIdx.x; size_t st=(size_t)gridDim.x*blockDim.x;
  for(; i<n; i+=st) b[i]=a[i];
}
__device__ __forceinline__ double mm_f64(double a, double b, double q, double qi){
  double h=a*b; double l=fma(a,b,-h); double c=rint(h*qi); double r=fma(-c,q,h)+l; return r<0.0? r+q : r;
}
__device__ __forceinline__ uint64_t mm_shoup(uint64_t b, uint64_t w, uint64_t wp, uint64_t q){
  uint64_t c=__umul64hi(b,wp); uint64_t r=w*b-c*q; return r>=q? r-q : r;
}
template<int CH>
__global__ void f64_k(const uint64_t* in, uint64_t* out, double q, double qi, double w, int iters){
  size_t t=blockIdx.x*(size_t)blockDim.x+threadIdx.x;
  double x[CH];
  #pragma unroll
  for(int c=0;c<CH;c++){ x[c]=(double)(in[t*CH+c] & ((1ull<<49)-1)); }
  for(int k=0;k<iters;k++){
    #pragma unroll
    for(int c=0;c<CH;c++) x[c]=mm_f64(x[c],w,q,qi);
  }
  #pragma unroll
  for(int c=0;c<CH;c++) out[t*CH+c]=(uint64_t)x[c];
}
template<int CH>
__global__ void shoup_k(const uint64_t* in, uint64_t* out, uint64_t q, uint64_t w, uint64_t wp, int iters){
  size_t t=blockIdx.x*(size_t)blockDim.x+threadIdx.x;
  uint64_t x[CH];
  #pragma unroll
  for(int c=0;c<CH;c++){ x[c]=in[t*CH+c] & ((1ull<<49)-1); }
  for(int k=0;k<iters;k++){
    #pragma unroll
    for(int c=0;c<CH;c++) x[c]=mm_shoup(x[c],w,wp,q);
  }
  #pragma unroll
  for(int c=0;c<CH;c++) out[t*CH+c]=x[c];
}
static uint64_t mulmod_host(uint64_t a, uint64_t b, uint64_t q){ return (uint64_t)((unsigned __int128)a*b%q); }
int main(){
  hipDeviceProp_t p; CK(hipGetDeviceProperties(&p,0));
  printf("device %s CUs %d clock %d kHz l2 %d\n", p.gcnArchName, p.multiProcessorCount, p.clockRate, p.l2CacheSize);
  size_t nbytes = (size_t)2<<30; size_t n = nbytes/16;
  ulonglong2 *a,*b; CK(hipMalloc(&a,nbytes)); CK(hipMalloc(&b,nbytes));
  CK(hipMemset(a,1,nbytes)); CK(hipMemset(b,0,nbytes));
  hipEvent_t e0,e1; CK(hipEventCreate(&e0)); CK(hipEventCreate(&e1));
  for(int rep=0;rep<3;rep++){
    CK(hipEventRecord(e0)); copy_k<<<256*8*4,256>>>(a,b,n); CK(hipEventRecord(e1)); CK(hipEventSynchronize(e1));
    float ms; CK(hipEventElapsedTime(&ms,e0,e1)); printf("copy 2GiB: %.3f ms  %.1f GB/s (r+w)\n", ms, 2.0*nbytes/ms/1e6);
  }
  CK(hipFree(a)); CK(hipFree(b));
  // modmul throughput
  const int CH=8; const int threads=256; const int blocks=256*16; const int iters=2048;
  size_t tot=(size_t)threads*blocks*CH;
  uint64_t *in,*out; CK(hipMalloc(&in,tot*8)); CK(hipMalloc(&out,tot*8));
  std::vector<uint64_t> h(tot); uint64_t s=0x1234567;
  for(size_t i=0;i<tot;i++){ s^=s<<13; s^=s>>7; s^=s<<17; h[i]=s; }
  CK(hipMemcpy(in,h.data(),tot*8,hipMemcpyHostToDevice));
  uint64_t q = 1125899906826241ull; // a prime < 2^50 of the form k*2^17+1? (checked below only as modulus)
  uint64_t w = 987654321987654ull % q;
  uint64_t wp = (uint64_t)(((unsigned __int128)w<<64)/q);
  double qd=(double)q, qi=1.0/qd, wd=(double)w;
  for(int rep=0;rep<2;rep++){
    CK(hipEventRecord(e0)); f64_k<CH><<<blocks,threads>>>(in,out,qd,qi,wd,iters); CK(hipEventRecord(e1)); CK(hipEventSynchronize(e1));
    float ms; CK(hipEventElapsedTime(&ms,e0,e1)); printf("f64 modmul: %.3f ms  %.3f T modmul/s\n", ms, (double)tot*iters/ms/1e9);
  }
  std::vector<uint64_t> o1(tot); CK(hipMemcpy(o1.data(),out,tot*8,hipMemcpyDeviceToHost));
  for(int rep=0;rep<2;rep++){
    CK(hipEventRecord(e0)); shoup_k<CH><<<blocks,threads>>>(in,out,q,w,wp,iters); CK(hipEventRecord(e1)); CK(hipEventSynchronize(e1));
    float ms; CK(hipEventElapsedTime(&ms,e0,e1)); printf("u64 shoup modmul: %.3f ms  %.3f T modmul/s\n", ms, (double)tot*iters/ms/1e9);
  }
  std::vector<uint64_t> o2(tot); CK(hipMemcpy(o2.data(),out,tot*8,hipMemcpyDeviceToHost));
  // verify a few entries on host
  int bad1=0,bad2=0;
  for(size_t i=0;i<tot;i+=tot/64){ uint64_t x=h[i]&((1ull<<49)-1); x%=q; for(int k=0;k<iters;k++) x=mulmod_host(x,w,q); if(x!=o1[i]) bad1++; if(x!=o2[i]) bad2++; }
  printf("check f64 bad=%d shoup bad=%d (of 64)\n",bad1,bad2);
  return 0;
}
