// Negacyclic NTT over RNS limbs for N >= 4096 (gfx950).
//
// Same transform as the LDS-staged generic kernels (forward Cooley-Tukey stages
// m = 1..N/2 with psi^rev(m+i), inverse Gentleman-Sande with psi^-rev(h+i) and
// N^-1), organised for registers:
//   * N = N1 * 4096.  The first log2(N1) stages couple words with equal index
//     mod 4096: one thread owns a whole column of N1 words (coalesced loads at
//     stride 4096, twiddles uniform across the wavefront) - no LDS at all.
//   * The last 12 stages stay inside a 4096-word tile: 256 threads own 16 words
//     each and run 3 rounds of 4 radix-2 stages in registers; between rounds the
//     tile goes through LDS once (padded by one word every 16 to avoid bank
//     conflicts).  Global loads and stores are fully coalesced.
// A round covering strides t0, t0/2, t0/4, t0/8 gives thread (lo, hi) the words
// x_k = lo + (t0/8) k + 2 t0 hi, k < 16; at stride t0/2^s the pair (k, k + 8>>s)
// belongs to butterfly block hi 2^s + (k >> (4-s)) of the tile.
#include <algorithm>

#include "internal.h"

namespace nj {

constexpr int kT = 4096;
constexpr int kNT = 256;

__device__ __forceinline__ int pad16(int x) { return x + (x >> 4); }

// Forward rounds are lazy: a round takes canonical words, runs its 4 stages without
// correction and reduces once at the end.  With t < 2^50 the lazy product of a word
// below B t in magnitude lies within (1/2 + 3B/8) t (the quotient estimate is off by
// at most 1/2 + 3 ulp-relative errors of a value below B 2^50), so the bound grows
// 1 -> 1.875 -> 3.08 -> 4.73 -> 7.01 over 4 stages: every intermediate is an integer
// below 2^53, computed exactly.

// one round of 4 forward stages on 16 registers (strides t0 .. t0/8 within the tile)
__device__ __forceinline__ void ct_round(double v[16], int t0, int hi, int tile, int logN1, const double *W, int N,
                                         Mod m)
{
#pragma unroll
    for (int s = 0; s < 4; s++) {
        const int t = t0 >> s;               // tile stride
        const int mm = N / (2 * t);          // global stage
        const int base = mm + tile * (mm >> logN1) + (hi << s);
        const int step = 8 >> s;
#pragma unroll
        for (int k = 0; k < 16; k++) {
            if (k & step) continue;
            const double w = W[base + (k >> (4 - s))];
            const double U = v[k], V = mul_lazy(v[k + step], w, m);
            v[k] = U + V;
            v[k + step] = U - V;
        }
    }
#pragma unroll
    for (int k = 0; k < 16; k++) v[k] = reduce(v[k], m);
}

// one round of 4 inverse stages (strides t0/8 .. t0)
__device__ __forceinline__ void gs_round(double v[16], int t0, int hi, int tile, int logN1, const double *W, int N,
                                         Mod m)
{
#pragma unroll
    for (int s = 3; s >= 0; s--) {
        const int t = t0 >> s;
        const int hh = N / (2 * t);
        const int base = hh + tile * (hh >> logN1) + (hi << s);
        const int step = 8 >> s;
#pragma unroll
        for (int k = 0; k < 16; k++) {
            if (k & step) continue;
            const double w = W[base + (k >> (4 - s))];
            const double U = v[k], V = v[k + step];
            v[k] = corr(U + V, m);
            v[k + step] = corr(mul_lazy(U - V, w, m), m);  // U - V in (-t, t)
        }
    }
}

// The 15 twiddles of one round (tile strides t0 .. t0/8) of butterfly block hi: stage
// s's 2^s words at tw[2^s - 1 + i], W[mm + tile (mm >> logN1) + (hi << s) + i] with
// mm = N / (2 (t0 >> s)).  The forward and the inverse table are indexed alike.
__device__ __forceinline__ void round_tw(double tw[15], int t0, int hi, int tile, int logN1, const double *W, int N)
{
#pragma unroll
    for (int st = 0; st < 4; st++) {
        const int mm = N / (2 * (t0 >> st));
        const int base = mm + tile * (mm >> logN1) + (hi << st);
#pragma unroll
        for (int i = 0; i < (1 << st); i++) tw[(1 << st) - 1 + i] = W[base + i];
    }
}

// ct_round / gs_round with the round's twiddles given (round_tw)
__device__ __forceinline__ void ct_round_tw(double v[16], const double tw[15], Mod m)
{
#pragma unroll
    for (int st = 0; st < 4; st++) {
        const int step = 8 >> st;
#pragma unroll
        for (int k = 0; k < 16; k++) {
            if (k & step) continue;
            const double U = v[k], V = mul_lazy(v[k + step], tw[(1 << st) - 1 + (k >> (4 - st))], m);
            v[k] = U + V;
            v[k + step] = U - V;
        }
    }
#pragma unroll
    for (int k = 0; k < 16; k++) v[k] = reduce(v[k], m);
}

__device__ __forceinline__ void gs_round_tw(double v[16], const double tw[15], Mod m)
{
#pragma unroll
    for (int st = 3; st >= 0; st--) {
        const int step = 8 >> st;
#pragma unroll
        for (int k = 0; k < 16; k++) {
            if (k & step) continue;
            const double U = v[k], V = v[k + step];
            v[k] = corr(U + V, m);
            v[k + step] = corr(mul_lazy(U - V, tw[(1 << st) - 1 + (k >> (4 - st))], m), m);  // U - V in (-t, t)
        }
    }
}

// The last 12 forward stages of one 4096-word tile: v holds words tid + 256 k on
// entry; on return the transformed tile is in s (word x at pad16(x)), after a barrier.
// Each round's twiddles are requested before the barrier that precedes the round (the
// registers of v are free there), so their latency overlaps the barrier wait.
__device__ __forceinline__ void tile_forward(double v[16], double *s, int tid, int tile, int logN1, const double *W,
                                             int N, Mod m)
{
    double tw[15];
    // round 0: strides 2048..256, thread tid owns x = tid + 256 k
    round_tw(tw, 2048, 0, tile, logN1, W, N);
    ct_round_tw(v, tw, m);
#pragma unroll
    for (int k = 0; k < 16; k++) s[pad16(tid + 256 * k)] = v[k];
    // round 1: strides 128..16, (lo, hi) = (tid & 15, tid >> 4): x = lo + 16 k + 256 hi
    const int lo = tid & 15, hi = tid >> 4;
    round_tw(tw, 128, hi, tile, logN1, W, N);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; k++) v[k] = s[pad16(lo + 16 * k + 256 * hi)];
    ct_round_tw(v, tw, m);
#pragma unroll
    for (int k = 0; k < 16; k++) s[pad16(lo + 16 * k + 256 * hi)] = v[k];
    // round 2: strides 8..1, thread owns x = 16 tid + k
    round_tw(tw, 8, tid, tile, logN1, W, N);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; k++) v[k] = s[pad16(16 * tid + k)];
    ct_round_tw(v, tw, m);
#pragma unroll
    for (int k = 0; k < 16; k++) s[pad16(16 * tid + k)] = v[k];
    __syncthreads();
}

// The first 12 inverse stages of one 4096-word tile (inverse twiddles W): v holds
// words tid + 256 k on entry and on return; s must be free on entry (callers that used
// it before put a barrier first).  Twiddles requested ahead as in tile_forward.
__device__ __forceinline__ void tile_inverse(double v[16], double *s, int tid, int tile, int logN1, const double *W,
                                             int N, Mod m)
{
    double tw[15];
    round_tw(tw, 8, tid, tile, logN1, W, N);
#pragma unroll
    for (int k = 0; k < 16; k++) s[pad16(tid + 256 * k)] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; k++) v[k] = s[pad16(16 * tid + k)];
    gs_round_tw(v, tw, m);
#pragma unroll
    for (int k = 0; k < 16; k++) s[pad16(16 * tid + k)] = v[k];
    const int lo = tid & 15, hi = tid >> 4;
    round_tw(tw, 128, hi, tile, logN1, W, N);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; k++) v[k] = s[pad16(lo + 16 * k + 256 * hi)];
    gs_round_tw(v, tw, m);
#pragma unroll
    for (int k = 0; k < 16; k++) s[pad16(lo + 16 * k + 256 * hi)] = v[k];
    round_tw(tw, 2048, 0, tile, logN1, W, N);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; k++) v[k] = s[pad16(tid + 256 * k)];
    gs_round_tw(v, tw, m);
}

// tile_forward and tile_inverse with each round's twiddles loaded where they are used
// (fewer live registers, for kernels held to 128 VGPRs)
__device__ __forceinline__ void tile_forward_lean(double v[16], double *s, int tid, int tile, int logN1, const double *W,
                                             int N, Mod m)
{
    // round 0: strides 2048..256, thread tid owns x = tid + 256 k
    ct_round(v, 2048, 0, tile, logN1, W, N, m);
#pragma unroll
    for (int k = 0; k < 16; k++) s[pad16(tid + 256 * k)] = v[k];
    __syncthreads();
    // round 1: strides 128..16, (lo, hi) = (tid & 15, tid >> 4): x = lo + 16 k + 256 hi
    {
        const int lo = tid & 15, hi = tid >> 4;
#pragma unroll
        for (int k = 0; k < 16; k++) v[k] = s[pad16(lo + 16 * k + 256 * hi)];
        ct_round(v, 128, hi, tile, logN1, W, N, m);
#pragma unroll
        for (int k = 0; k < 16; k++) s[pad16(lo + 16 * k + 256 * hi)] = v[k];
    }
    __syncthreads();
    // round 2: strides 8..1, thread owns x = 16 tid + k
#pragma unroll
    for (int k = 0; k < 16; k++) v[k] = s[pad16(16 * tid + k)];
    ct_round(v, 8, tid, tile, logN1, W, N, m);
#pragma unroll
    for (int k = 0; k < 16; k++) s[pad16(16 * tid + k)] = v[k];
    __syncthreads();
}

__device__ __forceinline__ void tile_inverse_lean(double v[16], double *s, int tid, int tile, int logN1, const double *W,
                                             int N, Mod m)
{
#pragma unroll
    for (int k = 0; k < 16; k++) s[pad16(tid + 256 * k)] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; k++) v[k] = s[pad16(16 * tid + k)];
    gs_round(v, 8, tid, tile, logN1, W, N, m);
#pragma unroll
    for (int k = 0; k < 16; k++) s[pad16(16 * tid + k)] = v[k];
    __syncthreads();
    {
        const int lo = tid & 15, hi = tid >> 4;
#pragma unroll
        for (int k = 0; k < 16; k++) v[k] = s[pad16(lo + 16 * k + 256 * hi)];
        gs_round(v, 128, hi, tile, logN1, W, N, m);
#pragma unroll
        for (int k = 0; k < 16; k++) s[pad16(lo + 16 * k + 256 * hi)] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; k++) v[k] = s[pad16(tid + 256 * k)];
    gs_round(v, 2048, 0, tile, logN1, W, N, m);
}

// The twiddles of one tile's forward pass (last 12 stages), for blocks that transform
// many limbs of the same prime and tile: staged in LDS once, so that the transform
// issues no vector memory operation and loads already in flight are never waited for
// in it.  Round 0, stage s: entry i of 2^s at kTwR1 + kTwR2 + 2^s - 1 + i (every lane
// reads the same word).  Round 1, stage s: entry (hi, i) of 16 2^s at 16 (2^s - 1) +
// hi 2^s + i (16 lanes per word).  Round 2, stage s: entry (tid, i) of 256 2^s at kTwR1
// + 256 (2^s - 1) + 256 i + tid (consecutive lanes, consecutive words).
constexpr int kTwR1 = 240, kTwR2 = 3840, kTwR0 = 15, kTwAll = kTwR1 + kTwR2 + kTwR0;

__device__ __forceinline__ void stage_tile_twiddles(double *tws, const double *W, int tile, int logN1, int N, int tid)
{
    constexpr int kPer = (kTwAll + kNT - 1) / kNT;
    double w[kPer];
#pragma unroll
    for (int q = 0; q < kPer; q++) {  // all loads in flight before the first store
        const int e = min(tid + kNT * q, kTwAll - 1);
        int t0, st, ent;
        if (e < kTwR1) {
            st = e < 16 ? 0 : e < 48 ? 1 : e < 112 ? 2 : 3;
            ent = e - 16 * ((1 << st) - 1);
            t0 = 128;
        } else if (e < kTwR1 + kTwR2) {
            const int f = e - kTwR1;
            st = f < 256 ? 0 : f < 768 ? 1 : f < 1792 ? 2 : 3;
            const int g = f - 256 * ((1 << st) - 1);
            ent = (g & 255) * (1 << st) + (g >> 8);
            t0 = 8;
        } else {
            const int f = e - kTwR1 - kTwR2;
            st = f < 1 ? 0 : f < 3 ? 1 : f < 7 ? 2 : 3;
            ent = f - ((1 << st) - 1);
            t0 = 2048;
        }
        const int mm = N / (2 * (t0 >> st));
        w[q] = W[mm + tile * (mm >> logN1) + ent];
    }
#pragma unroll
    for (int q = 0; q < kPer; q++)
        if (tid + kNT * q < kTwAll) tws[tid + kNT * q] = w[q];
}

// ct_round of round R (0: hi = 0, 1: hi = tid >> 4, 2: hi = tid) with the twiddles
// staged by stage_tile_twiddles
template <int R>
__device__ __forceinline__ void ct_round_lds(double v[16], const double *tws, int hi, Mod m)
{
#pragma unroll
    for (int st = 0; st < 4; st++) {
        const int step = 8 >> st;
#pragma unroll
        for (int k = 0; k < 16; k++) {
            if (k & step) continue;
            const int i = k >> (4 - st);
            const double w = R == 0   ? tws[kTwR1 + kTwR2 + (1 << st) - 1 + i]
                             : R == 1 ? tws[16 * ((1 << st) - 1) + (hi << st) + i]
                                      : tws[kTwR1 + 256 * ((1 << st) - 1) + 256 * i + hi];
            const double U = v[k], V = mul_lazy(v[k + step], w, m);
            v[k] = U + V;
            v[k + step] = U - V;
        }
    }
#pragma unroll
    for (int k = 0; k < 16; k++) v[k] = reduce(v[k], m);
}

// tile_forward with the twiddles staged by stage_tile_twiddles
__device__ __forceinline__ void tile_forward_lds(double v[16], double *s, const double *tws, int tid, Mod m)
{
    ct_round_lds<0>(v, tws, 0, m);
#pragma unroll
    for (int k = 0; k < 16; k++) s[pad16(tid + 256 * k)] = v[k];
    __syncthreads();
    {
        const int lo = tid & 15, hi = tid >> 4;
#pragma unroll
        for (int k = 0; k < 16; k++) v[k] = s[pad16(lo + 16 * k + 256 * hi)];
        ct_round_lds<1>(v, tws, hi, m);
#pragma unroll
        for (int k = 0; k < 16; k++) s[pad16(lo + 16 * k + 256 * hi)] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; k++) v[k] = s[pad16(16 * tid + k)];
    ct_round_lds<2>(v, tws, tid, m);
#pragma unroll
    for (int k = 0; k < 16; k++) s[pad16(16 * tid + k)] = v[k];
    __syncthreads();
}

// rows pass: last 12 stages on 4096-word tiles.  grid (N/4096, limbs)
template <bool INV>
__global__ __launch_bounds__(kNT) void k_ntt_tile(uint64_t *data, const uint64_t *src, LimbTab lt, const double *tw,
                                                  const PrimeInfo *info, int logN)
{
    __shared__ double s[kT + kT / 16];
    const int N = 1 << logN, logN1 = logN - 12;
    const int limb = blockIdx.y, pidx = lt.pidx[limb], tile = blockIdx.x, tid = threadIdx.x;
    const PrimeInfo pi = info[pidx];
    const Mod m = pi.m;
    const size_t off = (size_t)lt.off[limb] * N + (size_t)tile * kT;
    const uint64_t *in = src ? src + (size_t)lt.soff[limb] * N + (size_t)tile * kT : data + off;
    uint64_t *out = data + off;
    const double *W = tw + (size_t)pidx * N;
    double v[16];
    if (!INV) {
#pragma unroll
        for (int k = 0; k < 16; k++) v[k] = u2d(in[tid + 256 * k]);
        tile_forward(v, s, tid, tile, logN1, W, N, m);
#pragma unroll
        for (int k = 0; k < 16; k++) out[tid + 256 * k] = d2u(s[pad16(tid + 256 * k)]);
    } else {
#pragma unroll
        for (int k = 0; k < 16; k++) v[k] = u2d(in[tid + 256 * k]);
        tile_inverse(v, s, tid, tile, logN1, W, N, m);
        if (logN1 == 0) {
#pragma unroll
            for (int k = 0; k < 16; k++) v[k] = mul_canon(v[k], pi.ninv, m);
        }
#pragma unroll
        for (int k = 0; k < 16; k++) out[tid + 256 * k] = d2u(v[k]);
    }
}

// Special-prime rows of a key inner product (a0: first half, a1: second, words
// tid + 256 k of one tile) through the first 12 stages of ModDown's inverse transform
// (W: inverse twiddles of that prime), stored at out (first half) and out + half_off
// (second half).  Begins with a barrier, so s may still be in use on entry.
__device__ __forceinline__ void store_p_rows(double a0[16], double a1[16], double *s, uint64_t *out, size_t half_off,
                                             size_t w0, int tid, int tile, int logN1, const double *W, int N, Mod m)
{
    __syncthreads();
    tile_inverse(a0, s, tid, tile, logN1, W, N, m);
#pragma unroll
    for (int k = 0; k < 16; k++) out[w0 + 256 * k] = d2u(a0[k]);
    __syncthreads();
    tile_inverse(a1, s, tid, tile, logN1, W, N, m);
#pragma unroll
    for (int k = 0; k < 16; k++) out[half_off + w0 + 256 * k] = d2u(a1[k]);
}

// x words of step q = z ND + j of a key inner product (job z, digit j) at words
// w0 + 256 k: the job's own limb through X -> X^g, or the extended digit ([ND][ne][N])
// as it came out of its column pass.  Buffer loads: one 32-bit offset register per
// stream, the 256-word steps in the scalar offset.
template <int ND>
__device__ __forceinline__ void ip_load_x(const KeyJobs &kj, const IpRow &r, int q, uint32_t w0, int logN, uint32_t N,
                                          uint64_t *xn)
{
    const int z = q / ND, j = q - z * ND;
    if (j == r.own) {
        const auto d = buf_rsrc(kj.d[z] + r.t * N, 8u * N);
        const uint32_t g = kj.g[z];
#pragma unroll
        for (int k = 0; k < 16; k++) {
            xn[k] = buf_ld(d, 8u * (uint32_t)galois_src2((int)(w0 + 256u * k), g, logN), 0);  // g = 1: identity
        }
    } else {
        const auto e = buf_rsrc(kj.ext[z], 8u * (uint32_t)(ND * r.ne) * N);
        const uint32_t vo = 8u * ((uint32_t)(j * r.ne + r.t) * N + w0);
#pragma unroll
        for (int k = 0; k < 16; k++) xn[k] = buf_ld(e, vo, 2048u * k);
    }
}

// Key inner products fused with the forward tile pass of the extended digits (N >=
// 8192).  The key switch is of tau_g(d_z), g = kj.g[z]: at output limb t, digit j of
// job z is either the job's own limb d_z[t] read through X -> X^g (evaluation form) or
// the converted limb ext_z[j][t] of tau_g(d_z), which arrives with only its column
// pass applied: the block finishes that tile's transform in LDS and
// multiplies it by the key words at once, so extended digits are never stored in
// evaluation form.  Grid (jobs, N/4096, l+1+alpha-skip): grid row 0 is limb 0, row r > 0
// limb r + skip (skip = l - 1: only Q limbs 0 and l and the special primes, what a
// rescale followed by a drop to level 0 reads).  SUM: u = (accumulate ? u : 0) +
// the sum over all jobs (one block per tile); else job z = blockIdx.x has its own u_z
// = u_base + z 2 ne N (plus its previous value when accumulate): jobs vary fastest, so
// jobs sharing one key read each key tile close together in time.  After each job the
// running sums take at most ND <= 4 lazy terms on a reduced value.
// Latency: a block works through its (job, digit) steps one after another with two
// blocks per CU (256 registers per lane), so the words of the next step are requested
// before this step's transform, and the transform reads its twiddles from LDS (staged
// once per block) rather than memory: no wait in it holds up those loads.
template <int ND, bool SUM>
__global__ __launch_bounds__(kNT, 2) void k_ntt_ip(KeyJobs kj, int n_jobs, uint64_t *u_base, int accumulate, int level,
                                                int L, int alpha, int nq, const double *tw, const PrimeInfo *info,
                                                int logN, uint64_t *pout, const double *itw, int skip)
{
    __shared__ double s[kT + kT / 16];
    __shared__ double tws[kTwAll];
    const int N = 1 << logN, logN1 = logN - 12;
    const int t = blockIdx.z == 0 ? 0 : (int)blockIdx.z + skip, tile = blockIdx.y, tid = threadIdx.x;
    const int pidx = t <= level ? t : nq + (t - level - 1);
    const Mod m = info[pidx].m;
    const double *W = tw + (size_t)pidx * N;
    const IpRow r = ip_row(t, level, L, alpha);
    const size_t w0 = (size_t)tile * kT + tid;
    const int z0 = SUM ? 0 : (int)blockIdx.x, z1 = SUM ? n_jobs : z0 + 1;
    uint64_t *u = u_base + (SUM ? 0 : (size_t)z0 * 2 * r.ne * N);
    const size_t o0 = r.t * N + w0, o1 = (r.ne + r.t) * N + w0;
    // steps q = z ND + j run in order; the words of step q + 1 are requested before step
    // q's transform, so their latency hides behind it
    const int q0 = z0 * ND, q1 = z1 * ND;
    uint64_t xn[16];
    ip_load_x<ND>(kj, r, q0, (uint32_t)w0, logN, (uint32_t)N, xn);
    stage_tile_twiddles(tws, W, tile, logN1, N, tid);
    double a0[16], a1[16];
    if (accumulate) {
#pragma unroll
        for (int k = 0; k < 16; k++) a0[k] = u2d(u[o0 + 256 * k]), a1[k] = u2d(u[o1 + 256 * k]);
    } else {
#pragma unroll
        for (int k = 0; k < 16; k++) a0[k] = 0.0, a1[k] = 0.0;
    }
    __syncthreads();  // staged twiddles visible
#pragma unroll 1
    for (int q = q0; q < q1; q++) {
        const int z = q / ND, j = q - z * ND;
        const bool own = j == r.own;
        double x[16];
#pragma unroll
        for (int k = 0; k < 16; k++) x[k] = u2d(xn[k]);
        if (q + 1 < q1) ip_load_x<ND>(kj, r, q + 1, (uint32_t)w0, logN, (uint32_t)N, xn);
        if (!own) {
            __syncthreads();  // the previous step's words have been read out of s
            tile_forward_lds(x, s, tws, tid, m);
        } else {
            // words every thread reads back itself (its own positions), as the
            // transformed tile's are; no other thread touches them before the next barrier
#pragma unroll
            for (int k = 0; k < 16; k++) s[pad16(tid + 256 * k)] = x[k];
        }
        // key [ND][2][nk][N]: words of row kl of digit j, b half then a half
        const auto key = buf_rsrc(kj.key[z], 8u * (uint32_t)(2 * ND * r.nk) * (uint32_t)N);
        const uint32_t vb = 8u * ((uint32_t)(j * 2 * r.nk + r.kl) * (uint32_t)N + (uint32_t)w0),
                       va = vb + 8u * (uint32_t)(r.nk * N);
#pragma unroll
        for (int k = 0; k < 16; k++) {
            const double xv = s[pad16(tid + 256 * k)];
            a0[k] += mul_lazy(xv, u2d(buf_ld(key, vb, 2048u * k)), m);
            a1[k] += mul_lazy(xv, u2d(buf_ld(key, va, 2048u * k)), m);
        }
        if (j == ND - 1) {
#pragma unroll
            for (int k = 0; k < 16; k++) a0[k] = reduce(a0[k], m), a1[k] = reduce(a1[k], m);
        }
    }
    if (pout && t > level) {  // special-prime rows: on to ModDown's inverse transform
        store_p_rows(a0, a1, s, pout + ((size_t)2 * z0 * alpha + (t - level - 1)) * N, (size_t)alpha * N, w0, tid,
                     tile, logN1, itw + (size_t)pidx * N, N, m);
        return;
    }
#pragma unroll
    for (int k = 0; k < 16; k++) {
        u[o0 + 256 * k] = d2u(a0[k]);
        u[o1 + 256 * k] = d2u(a1[k]);
    }
}

// Special-prime rows of the key inner products of n_jobs jobs whose digits are already
// extended and in evaluation form (job z: [ND][ne][N] at kj.ext[z], read through
// X -> X^g, g = kj.g[z]; a special prime is in no digit, so no own limb): each block
// sums one tile of one half's products over the digits and sends it through the first
// 12 stages of ModDown's inverse transform into row (2 z + p) alpha + a of pout, as
// launch_ntt_ip does with its special-prime rows.  The products never go to memory in
// evaluation form.  Grid (2 jobs, N/4096, alpha): blockIdx.x = 2 z + p, so the two
// halves of one tile, which read the same digit words, are dispatched together.
template <int ND>
__global__ __launch_bounds__(kNT, 4) void k_key_ip_ptile(KeyJobs kj, int level, int L, int alpha, int nq,
                                                         const PrimeInfo *info, int logN, uint64_t *pout,
                                                         const double *itw)
{
    __shared__ double s[kT + kT / 16];
    const int N = 1 << logN, logN1 = logN - 12;
    const int z = blockIdx.x >> 1, p = blockIdx.x & 1, tile = blockIdx.y, a = blockIdx.z, tid = threadIdx.x;
    const int t = level + 1 + a, pidx = nq + a;
    const Mod m = info[pidx].m;
    const IpRow r = ip_row(t, level, L, alpha);
    const uint32_t g = kj.g[z], w0 = (uint32_t)tile * kT + tid;
    const auto e = buf_rsrc(kj.ext[z], 8u * (uint32_t)(ND * r.ne) * (uint32_t)N);
    const auto key = buf_rsrc(kj.key[z], 8u * (uint32_t)(2 * ND * r.nk) * (uint32_t)N);
    uint32_t src[16];
#pragma unroll
    for (int k = 0; k < 16; k++) src[k] = 8u * (uint32_t)galois_src2((int)(w0 + 256u * k), g, logN);
    double acc[16];
#pragma unroll
    for (int k = 0; k < 16; k++) acc[k] = 0.0;
#pragma unroll
    for (int j = 0; j < ND; j++) {
        const uint32_t xo = 8u * (uint32_t)((j * r.ne + r.t) * N),
                       vk = 8u * ((uint32_t)((j * 2 + p) * r.nk + r.kl) * (uint32_t)N + w0);
#pragma unroll
        for (int k = 0; k < 16; k++)
            acc[k] += mul_lazy(u2d(buf_ld(e, src[k], xo)), u2d(buf_ld(key, vk, 2048u * k)), m);
    }
#pragma unroll
    for (int k = 0; k < 16; k++) acc[k] = reduce(acc[k], m);
    tile_inverse(acc, s, tid, tile, logN1, itw + (size_t)pidx * N, N, m);
    uint64_t *out = pout + ((size_t)(2 * z + p) * alpha + a) * N + w0;
#pragma unroll
    for (int k = 0; k < 16; k++) out[256 * k] = d2u(acc[k]);
}

// Inverse tile pass whose input limbs are read through X -> X^g (the automorphism of a
// key switch folded into ModUp's inverse transform): limb lt[b] is of job off / L1,
// read from src + soff N at the words the Galois element gt.g[job] moves to each
// position.  grid (N/4096, limbs).
__global__ __launch_bounds__(kNT) void k_ntt_tile_gal(uint64_t *data, const uint64_t *src, LimbTab lt, GalTab gt,
                                                      int L1, const double *tw, const PrimeInfo *info, int logN)
{
    __shared__ double s[kT + kT / 16];
    const int N = 1 << logN, logN1 = logN - 12;
    const int limb = blockIdx.y, pidx = lt.pidx[limb], tile = blockIdx.x, tid = threadIdx.x;
    const Mod m = info[pidx].m;
    const uint32_t g = gt.g[lt.off[limb] / L1];
    const uint64_t *in = src + (size_t)lt.soff[limb] * N;
    const size_t w0 = (size_t)tile * kT + tid;
    double v[16];
#pragma unroll
    for (int k = 0; k < 16; k++) {
        const int w = (int)w0 + 256 * k;
        v[k] = u2d(in[g == 1u ? w : galois_src2(w, g, logN)]);
    }
    tile_inverse(v, s, tid, tile, logN1, tw + (size_t)pidx * N, N, m);
    uint64_t *out = data + (size_t)lt.off[limb] * N + w0;
#pragma unroll
    for (int k = 0; k < 16; k++) out[256 * k] = d2u(v[k]);
}

// The first log2(N1) forward stages on one column of N1 canonical words (lazy, one
// reduction at the end: at most 4 stages).
template <int N1>
__device__ __forceinline__ void col_forward(double v[N1], const double *W, Mod m)
{
#pragma unroll
    for (int mm = 1; mm < N1; mm <<= 1) {
        const int tr = N1 / (2 * mm);
#pragma unroll
        for (int r = 0; r < N1; r++) {
            if (r & tr) continue;
            const double w = W[mm + r / (2 * tr)];
            const double U = v[r], V = mul_lazy(v[r + tr], w, m);
            v[r] = U + V;
            v[r + tr] = U - V;
        }
    }
#pragma unroll
    for (int r = 0; r < N1; r++) v[r] = reduce(v[r], m);
}

// columns pass: first log2(N1) stages, one column of N1 words per thread.  grid (4096/256, limbs).
// The inverse ends with the factor N^-1, or scale[pidx] when a scale table is given
// (N^-1 times a basis conversion's input factor, so the conversion need not apply it).
// DBL: the results are stored as FP64 values (bit patterns of exact integers in [0, t))
// for the fused basis conversion, which then skips the integer -> FP64 step.
template <int N1, bool INV, bool DBL = false>
__global__ __launch_bounds__(kNT) void k_ntt_col(uint64_t *data, const uint64_t *src, LimbTab lt, const double *tw,
                                                 const PrimeInfo *info, int logN, const double *scale)
{
    const int N = 1 << logN;
    const int limb = blockIdx.y, pidx = lt.pidx[limb];
    const PrimeInfo pi = info[pidx];
    const Mod m = pi.m;
    const uint32_t cb = 8u * (blockIdx.x * kNT + threadIdx.x);
    uint64_t *outp = data + (size_t)lt.off[limb] * N;
    const auto in = buf_rsrc(src ? src + (size_t)lt.soff[limb] * N : outp, 8u * N);
    const auto out = buf_rsrc(outp, 8u * N);
    const double *W = tw + (size_t)pidx * N;
    double v[N1];
#pragma unroll
    for (int r = 0; r < N1; r++) v[r] = u2d(buf_ld(in, cb, 8u * r * kT));
    if (!INV) {
        col_forward<N1>(v, W, m);
    } else {
#pragma unroll
        for (int h = N1 / 2; h >= 1; h >>= 1) {
            const int tr = N1 / (2 * h);
#pragma unroll
            for (int r = 0; r < N1; r++) {
                if (r & tr) continue;
                const double w = W[h + r / (2 * tr)];
                const double U = v[r], V = v[r + tr];
                v[r] = corr(U + V, m);
                v[r + tr] = corr(mul_lazy(U - V, w, m), m);
            }
        }
        const double sc = scale ? scale[pidx] : pi.ninv;
#pragma unroll
        for (int r = 0; r < N1; r++) v[r] = mul_canon(v[r], sc, m);
    }
#pragma unroll
    for (int r = 0; r < N1; r++)
        buf_st(out, cb, 8u * r * kT, DBL ? (uint64_t)__double_as_longlong(v[r]) : d2u(v[r]));
}

// Basis conversion fused with the first log2(N1) forward stages of its outputs (the
// column pass).  Inputs are coefficient-form limbs already multiplied by
// (D/q_a)^-1 (folded into their inverse transform's N^-1) and stored by that transform
// as FP64 values (launch_intt_scaled, launch_intt_cols_scaled), so each output word is
// y_t = sum_a x_a (D/q_a) mod t; the converted limbs are never stored before their
// column pass.  Thread = one column (N1 words at stride 4096) of OUT consecutive
// targets of (job, digit) blockIdx.z = job * nd + digit; grid (4096/256,
// ceil(n_out/OUT), jobs nd).  Input slots past the digit size re-read its last limb
// with a zero factor; targets past n_out repeat the last one and are not stored.
constexpr int kBcOut = 2;  // targets per thread

template <int MMAX, int N1>
__global__ __launch_bounds__(kNT) void k_bconv_col(BconvShared sh, BconvPtrs jp, const double *tw,
                                                   const PrimeInfo *info, int logN)
{
    const int N = 1 << logN;
    const int job = blockIdx.z / sh.nd, j = blockIdx.z % sh.nd;
    const int c = blockIdx.x * kNT + threadIdx.x;
    const int n_out = sh.n_out[j], m = sh.m[j], o0 = blockIdx.y * kBcOut;
    if (o0 >= n_out) return;
    const auto in = buf_rsrc(jp.in[job] + (size_t)sh.in_off0[j] * N, (uint32_t)m * N * 8u);
    const uint32_t cb = 8u * c;
    const double *hat = sh.hat[j];
    int o[kBcOut];
    Mod mo[kBcOut];
#pragma unroll
    for (int q = 0; q < kBcOut; q++) {
        o[q] = o0 + q < n_out ? o0 + q : n_out - 1;
        mo[q] = info[sh.out_pidx[j][o[q]]].m;
    }
    double acc[kBcOut][N1];
#pragma unroll
    for (int q = 0; q < kBcOut; q++)
#pragma unroll
        for (int r = 0; r < N1; r++) acc[q][r] = 0.0;
#pragma unroll 2
    for (int a = 0; a < MMAX; a++) {  // two input limbs' loads in flight at a time
        const int aa = a < m ? a : m - 1;
        double h[kBcOut];
#pragma unroll
        for (int q = 0; q < kBcOut; q++) h[q] = a < m ? hat[aa * n_out + o[q]] : 0.0;
        uint64_t x[N1];
#pragma unroll
        for (int r = 0; r < N1; r++) x[r] = buf_ld(in, cb, 8u * ((uint32_t)aa * N + r * kT));
#pragma unroll
        for (int r = 0; r < N1; r++) {
            const double xv = __longlong_as_double((long long)x[r]);  // stored as FP64 by the inverse transform
#pragma unroll
            for (int q = 0; q < kBcOut; q++) acc[q][r] += mul_lazy(xv, h[q], mo[q]);
        }
        if (a % 7 == 6 && a + 1 < MMAX) {  // at most 7 lazy terms on a reduced sum
#pragma unroll
            for (int q = 0; q < kBcOut; q++)
#pragma unroll
                for (int r = 0; r < N1; r++) acc[q][r] = reduce(acc[q][r], mo[q]);
        }
    }
#pragma unroll
    for (int q = 0; q < kBcOut; q++) {
#pragma unroll
        for (int r = 0; r < N1; r++) acc[q][r] = reduce(acc[q][r], mo[q]);
        const int pq = sh.out_pidx[j][o[q]];
        col_forward<N1>(acc[q], tw + (size_t)pq * N, mo[q]);
        if (o0 + q < n_out) {
            const auto out = buf_rsrc(jp.out[job] + (size_t)sh.out_off[j][o[q]] * N, 8u * N);
#pragma unroll
            for (int r = 0; r < N1; r++) buf_st(out, cb, 8u * r * kT, d2u(acc[q][r]));
        }
    }
}

// ModDown of K key switches, finished inside the forward transform's tile pass.  The
// converted limbs conv [K][2][l+1][N] (coefficient form, column pass already applied)
// are transformed tile by tile and, instead of being stored, combined at once:
// out_z[p][i] = (u_z[p][i] - NTT(conv_z[p][i])) P^-1 (+ c0 of job z read through
// X -> X^g_add[z] for p = 0) (+ the previous out_z when acc; job 0 reads it from acc0
// instead when given), with u_z at u_base + z 2 ne N.  With last_out (one job), the
// blocks of the last limb also run the first 12 stages of its inverse transform on
// the words they wrote and store them at last_out + p N, ready for a rescale.
// grid (N/4096, 2 K (l+1)): limb w = (2 z + p)(l+1) + i.
template <bool CONJ>
__global__ __launch_bounds__(kNT, 4) void k_ntt_tile_md(const uint64_t *conv, const uint64_t *u_base, MdJobs mj, int acc,
                                                     int level, int ne, const double *pinv, const double *tw,
                                                     const PrimeInfo *info, int logN, const uint64_t *acc0,
                                                     uint64_t *last_out, const double *itw, MdConj cj, int skip)
{
    __shared__ double s[kT + kT / 16];
    const int N = 1 << logN, logN1 = logN - 12, L1 = level + 1, L1e = L1 - skip;
    const int w = blockIdx.y, h = w / L1e, ie = w - h * L1e, i = ie == 0 ? 0 : ie + skip, z = h >> 1, p = h & 1;
    const int tile = blockIdx.x, tid = threadIdx.x;
    const Mod m = info[i].m;
    const double *W = tw + (size_t)i * N;
    const size_t t0 = (size_t)tile * kT;
    const uint64_t *in = conv + ((size_t)h * L1 + i) * N + t0;
    double v[16];
#pragma unroll
    for (int k = 0; k < 16; k++) v[k] = u2d(in[tid + 256 * k]);
    tile_forward_lean(v, s, tid, tile, logN1, W, N, m);
    const uint64_t *u = u_base + ((size_t)z * 2 * ne + (size_t)p * ne + i) * N + t0;
    const uint64_t *add = p == 0 ? mj.add[z] : nullptr;
    const uint32_t g = mj.g_add[z];
    uint64_t *out = mj.out[z] + ((size_t)p * L1 + i) * N + t0;
    const uint64_t *prev = acc0 && z == 0 ? acc0 + ((size_t)p * L1 + i) * N + t0 : out;
    const double pv = pinv[i];
#pragma unroll
    for (int k = 0; k < 16; k++) {
        const int x = tid + 256 * k;
        double t = mul_canon(sub_mod(u2d(u[x]), s[pad16(x)], m), pv, m);
        if (add) {
            const int kk = (int)t0 + x;
            t = add_mod(t, u2d(add[(size_t)i * N + (g <= 1u ? kk : galois_src2(kk, g, logN))]), m);
        }
        if (acc) t = add_mod(t, u2d(prev[x]), m);
        if (CONJ) {  // the real/imaginary split, as in k_conj_split
            const size_t o = ((size_t)p * L1 + i) * N + t0 + x;
            const double a = u2d(cj.x[o]);
            cj.re[o] = d2u(add_mod(a, t, m));
            double r = mul_canon(sub_mod(a, t, m), W[1], m);
            if ((brev_n((uint32_t)(t0 + x), logN) & 1u) == 0u) r = r == 0.0 ? 0.0 : m.t - r;
            cj.im[o] = d2u(r);
        } else {
            out[x] = d2u(t);
        }
    }
    if (last_out && i == level) {  // the rescale's inverse tile pass of this limb
#pragma unroll
        for (int k = 0; k < 16; k++) v[k] = u2d(out[tid + 256 * k]);  // this thread's own words
        __syncthreads();
        tile_inverse_lean(v, s, tid, tile, logN1, itw + (size_t)i * N, N, m);
#pragma unroll
        for (int k = 0; k < 16; k++) last_out[(size_t)p * N + t0 + tid + 256 * k] = d2u(v[k]);
    }
}

// ModDown combine of K key switches from extended evaluation-form digits, with their
// key inner products on the Q limbs computed in the same block (the plain combine of
// k_ntt_tile_md, no accumulation): job z's half p at limb i is the sum over digits j of
// x_j read through X -> X^g (the own limb of kj.d[z] for i's digit, else the extended
// digit j at kj.ext[z]) times the key words, then (that - the converted special-prime
// part, after its tile pass) P^-1 plus add.  The products never go to memory.  Grid
// (N/4096, 2 K (l+1)).
template <int ND>
__global__ __launch_bounds__(kNT, ND == 1 ? 3 : ND == 4 ? 2 : 4) void k_key_ip_md(const uint64_t *conv, KeyJobs kj, MdJobs mj, int level, int L,
                                                      int alpha, const double *pinv, const double *tw,
                                                      const PrimeInfo *info, int logN)
{
    __shared__ double s[kT + kT / 16];
    const int N = 1 << logN, logN1 = logN - 12, L1 = level + 1;
    const int w = blockIdx.y, h = w / L1, i = w - h * L1, z = h >> 1, p = h & 1;
    const int tile = blockIdx.x, tid = threadIdx.x;
    const Mod m = info[i].m;
    const size_t t0 = (size_t)tile * kT;
    const IpRow r = ip_row(i, level, L, alpha);
    const uint32_t g = kj.g[z], w0 = (uint32_t)t0 + tid;
    const auto e = buf_rsrc(kj.ext[z], 8u * (uint32_t)(ND * r.ne) * (uint32_t)N);
    const auto dd = buf_rsrc(kj.d[z] + (size_t)i * N, 8u * (uint32_t)N);
    const auto key = buf_rsrc(kj.key[z], 8u * (uint32_t)(2 * ND * r.nk) * (uint32_t)N);
    double a[16];
    {
        uint32_t src[16];
#pragma unroll
        for (int k = 0; k < 16; k++)
            src[k] = 8u * (g <= 1u ? w0 + 256u * k : (uint32_t)galois_src2((int)(w0 + 256u * k), g, logN));
#pragma unroll
        for (int k = 0; k < 16; k++) a[k] = 0.0;
#pragma unroll
        for (int j = 0; j < ND; j++) {
            const uint32_t vk = 8u * ((uint32_t)((j * 2 + p) * r.nk + r.kl) * (uint32_t)N + w0);
            if (j == r.own) {
#pragma unroll
                for (int k = 0; k < 16; k++)
                    a[k] += mul_lazy(u2d(buf_ld(dd, src[k], 0)), u2d(buf_ld(key, vk, 2048u * k)), m);
            } else {
                const uint32_t xo = 8u * (uint32_t)((j * r.ne + r.t) * N);
#pragma unroll
                for (int k = 0; k < 16; k++)
                    a[k] += mul_lazy(u2d(buf_ld(e, src[k], xo)), u2d(buf_ld(key, vk, 2048u * k)), m);
            }
        }
#pragma unroll
        for (int k = 0; k < 16; k++) a[k] = reduce(a[k], m);
    }
    const uint64_t *in = conv + ((size_t)h * L1 + i) * N + t0;
    double v[16];
#pragma unroll
    for (int k = 0; k < 16; k++) v[k] = u2d(in[tid + 256 * k]);
    tile_forward_lean(v, s, tid, tile, logN1, tw + (size_t)i * N, N, m);
    const uint64_t *add = p == 0 ? mj.add[z] : nullptr;
    const uint32_t ga = mj.g_add[z];
    uint64_t *out = mj.out[z] + ((size_t)p * L1 + i) * N + t0;
    const double pv = pinv[i];
#pragma unroll
    for (int k = 0; k < 16; k++) {
        const int x = tid + 256 * k;
        double t = mul_canon(sub_mod(a[k], s[pad16(x)], m), pv, m);
        if (add) {
            const int kk = (int)t0 + x;
            t = add_mod(t, u2d(add[(size_t)i * N + (ga <= 1u ? kk : galois_src2(kk, ga, logN))]), m);
        }
        out[x] = d2u(t);
    }
}

// Rescale by q_l, fused into the lifted limbs' transform (N >= 8192).  k_lift_col: the
// last limb of each polynomial (coefficient form, last [P][N]) lifted centred into
// target limb i, then the forward column pass; grid (4096/256, n_out, P).
template <int N1>
__global__ __launch_bounds__(kNT) void k_lift_col(const uint64_t *last, int src_pidx, int n_out, uint64_t *lifted,
                                                  const double *tw, const PrimeInfo *info, int logN)
{
    const int N = 1 << logN, i = blockIdx.y, z = blockIdx.z;
    const uint32_t cb = 8u * (blockIdx.x * kNT + threadIdx.x);
    const Mod ms = info[src_pidx].m, mt = info[i].m;
    const double half = info[src_pidx].half;
    const auto src = buf_rsrc(last + (size_t)z * N, 8u * N);
    double v[N1];
#pragma unroll
    for (int r = 0; r < N1; r++) {
        const double x = u2d(buf_ld(src, cb, 8u * r * kT));
        v[r] = reduce(x > half ? x - ms.t : x, mt);  // centred, |x| < t_l / 2 < 2^49
    }
    col_forward<N1>(v, tw + (size_t)i * N, mt);
    const auto dst = buf_rsrc(lifted + ((size_t)z * n_out + i) * N, 8u * N);
#pragma unroll
    for (int r = 0; r < N1; r++) buf_st(dst, cb, 8u * r * kT, d2u(v[r]));
}

// k_ntt_tile_rs: the lifted limbs' tile pass with the rescale combine as its epilogue,
// out[z][i] = (in[z][i] - NTT(lift)[z][i]) q_l^-1 mod q_i; grid (N/4096, P n_out).
__global__ __launch_bounds__(kNT) void k_ntt_tile_rs(const uint64_t *lifted, const uint64_t *in, uint64_t *out,
                                                     int level, int n_out, const double *qlinv, const double *qlinvq,
                                                     int nq, const double *tw, const PrimeInfo *info, int logN)
{
    __shared__ double s[kT + kT / 16];
    const int N = 1 << logN, logN1 = logN - 12;
    const int w = blockIdx.y, z = w / n_out, i = w - z * n_out;
    const int tile = blockIdx.x, tid = threadIdx.x;
    const Mod m = info[i].m;
    const size_t t0 = (size_t)tile * kT;
    const uint64_t *src = lifted + (size_t)w * N + t0;
    double v[16];
#pragma unroll
    for (int k = 0; k < 16; k++) v[k] = u2d(src[tid + 256 * k]);
    tile_forward(v, s, tid, tile, logN1, tw + (size_t)i * N, N, m);
    const uint64_t *a = in + ((size_t)z * (level + 1) + i) * N + t0;
    uint64_t *o = out + ((size_t)z * n_out + i) * N + t0;
    const double wl = qlinv[level * nq + i], wlq = qlinvq[level * nq + i];
#pragma unroll
    for (int k = 0; k < 16; k++) {
        const int x = tid + 256 * k;
        o[x] = d2u(mul_shoup(sub_mod(u2d(a[x]), s[pad16(x)], m), wl, wlq, m));
    }
}

template <bool INV, bool DBL = false>
static hipError_t launch_cols(const nj_ctx *c, int kind, double bytes, int N1, dim3 grid, hipStream_t s,
                              uint64_t *data, const uint64_t *src, const LimbTab &lt, const double *tw,
                              const PrimeInfo *info, int logN, const double *scale = nullptr)
{
    switch (N1) {
    case 2: return launch(c, kind, bytes, k_ntt_col<2, INV, DBL>, grid, dim3(kNT), s, data, src, lt, tw, info, logN, scale);
    case 4: return launch(c, kind, bytes, k_ntt_col<4, INV, DBL>, grid, dim3(kNT), s, data, src, lt, tw, info, logN, scale);
    case 8: return launch(c, kind, bytes, k_ntt_col<8, INV, DBL>, grid, dim3(kNT), s, data, src, lt, tw, info, logN, scale);
    default:
        return launch(c, kind, bytes, k_ntt_col<16, INV, DBL>, grid, dim3(kNT), s, data, src, lt, tw, info, logN, scale);
    }
}

// N >= 4096: forward = columns then tiles, inverse = tiles then columns.  src (optional)
// is read instead of data by the first pass (limb i at src + soff[i]*N).
hipError_t launch_ntt_fast(const nj_ctx *c, uint64_t *data, const uint64_t *src, const LimbTab &lt, bool inverse,
                           hipStream_t s)
{
    const int N = c->N, N1 = N / kT;
    const double *tw = inverse ? c->d_itw : c->d_tw;
    dim3 gt(N1, lt.n), gc(kT / kNT, lt.n);
    const double bytes = 16.0 * N * lt.n;  // each pass reads and writes every word once
    hipError_t e;
    if (!inverse) {
        if (N1 > 1) {
            e = launch_cols<false>(c, PROF_NTT_COL, bytes, N1, gc, s, data, src, lt, tw, c->d_info, c->log_n);
            if (e != hipSuccess) return e;
            src = nullptr;
        }
        return launch(c, PROF_NTT_TILE, bytes, k_ntt_tile<false>, gt, dim3(kNT), s, data, src, lt, tw, c->d_info,
                      c->log_n);
    }
    e = launch(c, PROF_NTT_TILE_INV, bytes, k_ntt_tile<true>, gt, dim3(kNT), s, data, src, lt, tw, c->d_info, c->log_n);
    if (e != hipSuccess || N1 == 1) return e;
    return launch_cols<true>(c, PROF_NTT_COL_INV, bytes, N1, gc, s, data, nullptr, lt, tw, c->d_info, c->log_n);
}

// Inverse transform whose final factor is scale[pidx] instead of N^-1 (N >= 8192),
// for the fused basis conversion: the results are stored as FP64 values.  With gt,
// the input limbs are read through X -> X^g of their job (off / L1).
hipError_t launch_intt_scaled(const nj_ctx *c, uint64_t *data, const uint64_t *src, const LimbTab &lt,
                              const double *scale, hipStream_t s, const GalTab *gt, int L1)
{
    const int N = c->N, N1 = N / kT;
    if (N1 < 2 || (gt && (!src || L1 < 1))) return hipErrorInvalidValue;
    if (lt.n == 0) return hipSuccess;
    const double bytes = 16.0 * N * lt.n;
    hipError_t e = gt ? launch(c, PROF_NTT_TILE_INV, bytes, k_ntt_tile_gal, dim3(N1, lt.n), dim3(kNT), s, data, src,
                               lt, *gt, L1, c->d_itw, c->d_info, c->log_n)
                      : launch(c, PROF_NTT_TILE_INV, bytes, k_ntt_tile<true>, dim3(N1, lt.n), dim3(kNT), s, data, src,
                               lt, c->d_itw, c->d_info, c->log_n);
    if (e != hipSuccess) return e;
    return launch_cols<true, true>(c, PROF_NTT_COL_INV, bytes, N1, dim3(kT / kNT, lt.n), s, data, nullptr, lt,
                                   c->d_itw, c->d_info, c->log_n, scale);
}

// Rescale of P packed level-l polynomials (P = 2 per ciphertext; limbs 0..n_out-1 of
// each kept), N >= 8192: inverse transform of the last limbs read in place (into
// last [P][N]), lift fused with the column pass (into lifted [P][n_out][N], which may be
// out: each tile block reads its own lifted words before writing them), tile pass
// fused with the combine.  in must not alias out.
hipError_t launch_rescale_fused(const nj_ctx *c, int level, const uint64_t *in, uint64_t *out, int n_out,
                                uint64_t *last, uint64_t *lifted, hipStream_t s, int n_polys, bool last_tiled)
{
    const int N = c->N, N1 = N / kT;
    if (N1 < 2 || n_out < 1 || n_out > level || n_polys < 1 || n_polys > NJ_MAX_LIMBS) return hipErrorInvalidValue;
    LimbTab lt;
    lt.n = n_polys;
    for (int p = 0; p < n_polys; p++) lt.pidx[p] = level, lt.off[p] = p, lt.soff[p] = p * (level + 1) + level;
    // last_tiled: the last limbs' inverse tile pass already ran (into last), the column pass follows
    hipError_t e = last_tiled ? launch_cols<true>(c, PROF_NTT_COL_INV, 16.0 * N * n_polys, N1, dim3(kT / kNT, n_polys), s,
                                                  last, nullptr, lt, c->d_itw, c->d_info, c->log_n)
                              : launch_ntt_fast(c, last, in, lt, true, s);
    if (e != hipSuccess) return e;
    const dim3 gl(kT / kNT, n_out, n_polys);
    const double bl = 8.0 * N * n_polys * (1 + n_out);
    switch (N1) {
    case 2: e = launch(c, PROF_OTHER, bl, k_lift_col<2>, gl, dim3(kNT), s, last, level, n_out, lifted, c->d_tw, c->d_info, c->log_n); break;
    case 4: e = launch(c, PROF_OTHER, bl, k_lift_col<4>, gl, dim3(kNT), s, last, level, n_out, lifted, c->d_tw, c->d_info, c->log_n); break;
    case 8: e = launch(c, PROF_OTHER, bl, k_lift_col<8>, gl, dim3(kNT), s, last, level, n_out, lifted, c->d_tw, c->d_info, c->log_n); break;
    default: e = launch(c, PROF_OTHER, bl, k_lift_col<16>, gl, dim3(kNT), s, last, level, n_out, lifted, c->d_tw, c->d_info, c->log_n);
    }
    if (e != hipSuccess) return e;
    return launch(c, PROF_OTHER, 8.0 * N * n_polys * n_out * 4.0, k_ntt_tile_rs, dim3(N1, n_polys * n_out), dim3(kNT),
                  s, lifted, in, out, level, n_out, c->d_qlinv, c->d_qlinvq, c->n_q, c->d_tw, c->d_info, c->log_n);
}

// Forward tile pass alone (the column pass already applied), N >= 8192.
hipError_t launch_ntt_tiles(const nj_ctx *c, uint64_t *data, const LimbTab &lt, hipStream_t s)
{
    const int N = c->N, N1 = N / kT;
    if (N1 < 2) return hipErrorInvalidValue;
    if (lt.n == 0) return hipSuccess;
    return launch(c, PROF_NTT_TILE, 16.0 * N * lt.n, k_ntt_tile<false>, dim3(N1, lt.n), dim3(kNT), s, data, nullptr,
                  lt, c->d_tw, c->d_info, c->log_n);
}

// Basis conversion of n_jobs (job, digit) pairs fused with the outputs' column pass
// (inputs pre-multiplied by (D/q_a)^-1), N >= 8192.
hipError_t launch_bconv_col(const nj_ctx *c, const BconvShared &sh, const BconvPtrs &jp, int n_jobs, hipStream_t s)
{
    const int N = c->N, N1 = N / kT;
    if (N1 < 2 || n_jobs == 0) return N1 < 2 ? hipErrorInvalidValue : hipSuccess;
    int max_out = 0, mmax = 0;
    double bytes = 0;
    for (int j = 0; j < sh.nd; j++) {
        max_out = std::max(max_out, sh.n_out[j]);
        mmax = std::max(mmax, sh.m[j]);
        bytes += 8.0 * N * (sh.m[j] + sh.n_out[j]) * n_jobs;
    }
    if (mmax > 8) return hipErrorInvalidValue;
    const dim3 grid(kT / kNT, (max_out + kBcOut - 1) / kBcOut, n_jobs * sh.nd);
#define NJ_BC(MM, NN)                                                                                               \
    if (mmax <= MM && N1 == NN)                                                                                    \
        return launch(c, PROF_BCONV, bytes, k_bconv_col<MM, NN>, grid, dim3(kNT), s, sh, jp, c->d_tw, c->d_info,   \
                      c->log_n);
    NJ_BC(2, 2) NJ_BC(2, 4) NJ_BC(2, 8) NJ_BC(2, 16)
    NJ_BC(4, 2) NJ_BC(4, 4) NJ_BC(4, 8) NJ_BC(4, 16)
    NJ_BC(8, 2) NJ_BC(8, 4) NJ_BC(8, 8) NJ_BC(8, 16)
#undef NJ_BC
    return hipErrorInvalidValue;
}

// ModDown combine of K jobs fused into the forward transform of their converted
// limbs (N >= 4096; cols_done: the column pass was already applied); same results
// as the transform followed by the combine.
hipError_t launch_ntt_moddown(const nj_ctx *c, int level, int K, uint64_t *conv, const uint64_t *u_base,
                              const MdJobs &mj, int acc, int cols_done, hipStream_t s, const uint64_t *acc0,
                              uint64_t *last_out, const MdConj *conj, int skip)
{
    const int N = c->N, N1 = N / kT, L1 = level + 1, n = 2 * K * (L1 - skip);
    if (N < kT || K < 1 || K > NJ_MAX_JOBS || ((last_out || conj) && K != 1) || (last_out && conj) || skip < 0 ||
        skip > std::max(0, level - 1) || (skip && (!cols_done || last_out || conj)))
        return hipErrorInvalidValue;
    MdConj cj{nullptr, nullptr, nullptr};
    if (conj) cj = *conj;
    if (N1 > 1 && !cols_done) {
        LimbTab lt;
        for (int b = 0; b < n; b += NJ_MAX_LIMBS) {
            lt.n = std::min(NJ_MAX_LIMBS, n - b);
            for (int j = 0; j < lt.n; j++) lt.pidx[j] = (b + j) % L1, lt.off[j] = b + j, lt.soff[j] = 0;
            hipError_t e = launch_cols<false>(c, PROF_NTT_COL, 16.0 * N * lt.n, N1, dim3(kT / kNT, lt.n), s, conv,
                                              nullptr, lt, c->d_tw, c->d_info, c->log_n);
            if (e != hipSuccess) return e;
        }
    }
    const double bytes = 8.0 * N * (n * 3.0 + K * (L1 - skip) + (acc ? n : 0));
    if (conj)
        return launch(c, PROF_NTT_MD, bytes, k_ntt_tile_md<true>, dim3(N1, n), dim3(kNT), s, conv, u_base, mj, acc,
                      level, L1 + c->alpha, c->d_pinv, c->d_tw, c->d_info, c->log_n, acc0, last_out, c->d_itw, cj, skip);
    return launch(c, PROF_NTT_MD, bytes, k_ntt_tile_md<false>, dim3(N1, n), dim3(kNT), s, conv, u_base, mj, acc, level,
                  L1 + c->alpha, c->d_pinv, c->d_tw, c->d_info, c->log_n, acc0, last_out, c->d_itw, cj, skip);
}

// The plain ModDown combine of K key switches (converted limbs column-passed) with their
// Q-limb key inner products computed inside it from extended evaluation-form digits
// (N >= 8192, 1..4 digits).
hipError_t launch_key_ip_moddown(const nj_ctx *c, int level, int K, const uint64_t *conv, const KeyJobs &kj,
                                 const MdJobs &mj, hipStream_t s)
{
    const int N = c->N, N1 = N / kT, L1 = level + 1, n = 2 * K * L1, nd = n_digits(c, level);
    if (N1 < 2 || K < 1 || K > NJ_MAX_JOBS || nd < 1 || nd > 4) return hipErrorInvalidValue;
    const double bytes = 8.0 * N * (n * (2.0 * nd + 2.0) + K * L1);
#define NJ_IPMD(ND)                                                                                                \
    case ND:                                                                                                       \
        return launch(c, PROF_KEYIP, bytes, k_key_ip_md<ND>, dim3(N1, n), dim3(kNT), s, conv, kj, mj, level, c->L, \
                      c->alpha, c->d_pinv, c->d_tw, c->d_info, c->log_n);
    switch (nd) {
        NJ_IPMD(1) NJ_IPMD(2) NJ_IPMD(3) NJ_IPMD(4)
    }
#undef NJ_IPMD
    return hipErrorInvalidValue;
}

// Key inner products of n_jobs jobs (digits of tau_g(d) column-passed only, own limbs
// read from d through X -> X^g) fused with the digits' tile pass; sum = 1: one output,
// summed over the jobs; accumulate: added to the output's previous value.
hipError_t launch_ntt_ip(const nj_ctx *c, int level, const KeyJobs &kj, int n_jobs, uint64_t *u, int sum,
                         int accumulate, hipStream_t s, uint64_t *pout, int skip)
{
    const int N = c->N, N1 = N / kT, nd = n_digits(c, level), ne = level + 1 + c->alpha;
    if (N1 < 2 || nd < 1 || nd > 4 || n_jobs < 1 || n_jobs > NJ_MAX_JOBS || skip < 0 || skip > std::max(0, level - 1))
        return hipErrorInvalidValue;
    const double bytes = 8.0 * N * (ne - skip) * (3.0 * nd * n_jobs + 2.0 * (sum ? 1 : n_jobs) * (1 + accumulate));
    const dim3 grid(sum ? 1 : n_jobs, N1, ne - skip);
#define NJ_IP(ND)                                                                                                   \
    case ND:                                                                                                        \
        return sum ? launch(c, PROF_KEYIP, bytes, k_ntt_ip<ND, true>, grid, dim3(kNT), s, kj, n_jobs, u, accumulate, \
                            level, c->L, c->alpha, c->n_q, c->d_tw, c->d_info, c->log_n, pout, c->d_itw, skip)     \
                   : launch(c, PROF_KEYIP, bytes, k_ntt_ip<ND, false>, grid, dim3(kNT), s, kj, n_jobs, u, accumulate, \
                            level, c->L, c->alpha, c->n_q, c->d_tw, c->d_info, c->log_n, pout, c->d_itw, skip);
    switch (nd) {
        NJ_IP(1) NJ_IP(2) NJ_IP(3) NJ_IP(4)
    }
#undef NJ_IP
    return hipErrorInvalidValue;
}

// Special-prime rows of n_jobs key inner products from extended evaluation-form digits,
// through the first 12 stages of ModDown's inverse transform into pout (N >= 8192,
// 1..4 digits, alpha <= 8).
hipError_t launch_key_ip_ptile(const nj_ctx *c, int level, const KeyJobs &kj, int n_jobs, uint64_t *pout,
                               hipStream_t s)
{
    const int N = c->N, N1 = N / kT, nd = n_digits(c, level);
    if (N1 < 2 || nd < 1 || nd > 4 || c->alpha > 8 || n_jobs < 1 || n_jobs > NJ_MAX_JOBS || !pout)
        return hipErrorInvalidValue;
    const double bytes = 8.0 * N * c->alpha * (3.0 * nd + 2.0) * n_jobs;
    const dim3 grid(2 * n_jobs, N1, c->alpha);
#define NJ_PT(ND)                                                                                             \
    case ND:                                                                                                  \
        return launch(c, PROF_KEYIP, bytes, k_key_ip_ptile<ND>, grid, dim3(kNT), s, kj, level, c->L, c->alpha, \
                      c->n_q, c->d_info, c->log_n, pout, c->d_itw);
    switch (nd) {
        NJ_PT(1) NJ_PT(2) NJ_PT(3) NJ_PT(4)
    }
#undef NJ_PT
    return hipErrorInvalidValue;
}

// The column pass of an inverse transform whose tile pass already ran, in place, with
// the final factor scale[pidx] (N >= 8192); results stored as FP64 values, as above.
hipError_t launch_intt_cols_scaled(const nj_ctx *c, uint64_t *data, const LimbTab &lt, const double *scale,
                                   hipStream_t s)
{
    const int N = c->N, N1 = N / kT;
    if (N1 < 2) return hipErrorInvalidValue;
    if (lt.n == 0) return hipSuccess;
    return launch_cols<true, true>(c, PROF_NTT_COL_INV, 16.0 * N * lt.n, N1, dim3(kT / kNT, lt.n), s, data, nullptr,
                                   lt, c->d_itw, c->d_info, c->log_n, scale);
}

// Centred lift of n_polys coefficient-form limbs (prime src_pidx, at src + z N) into
// primes 0..n_out-1, fused with those limbs' column pass, into out [n_polys][n_out][N]
// (N >= 8192); the tile pass (launch_ntt_tiles) finishes the forward transform.
hipError_t launch_lift_col(const nj_ctx *c, const uint64_t *src, int src_pidx, int n_polys, int n_out, uint64_t *out,
                           hipStream_t s)
{
    const int N = c->N, N1 = N / kT;
    if (N1 < 2 || n_out < 1 || n_polys < 1) return hipErrorInvalidValue;
    const dim3 g(kT / kNT, n_out, n_polys);
    const double b = 8.0 * N * n_polys * (1 + n_out);
    switch (N1) {
    case 2: return launch(c, PROF_OTHER, b, k_lift_col<2>, g, dim3(kNT), s, src, src_pidx, n_out, out, c->d_tw, c->d_info, c->log_n);
    case 4: return launch(c, PROF_OTHER, b, k_lift_col<4>, g, dim3(kNT), s, src, src_pidx, n_out, out, c->d_tw, c->d_info, c->log_n);
    case 8: return launch(c, PROF_OTHER, b, k_lift_col<8>, g, dim3(kNT), s, src, src_pidx, n_out, out, c->d_tw, c->d_info, c->log_n);
    default: return launch(c, PROF_OTHER, b, k_lift_col<16>, g, dim3(kNT), s, src, src_pidx, n_out, out, c->d_tw, c->d_info, c->log_n);
    }
}

}  // namespace nj
