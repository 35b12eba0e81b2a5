// Host FP64 encoding and offline plan construction (not on the timed path).
//
//  * Slot encoding (Sec. 2.2): the plaintext f has f(zeta_j) = z_j, zeta_j = zeta^(5^j).
//    With V[j][i] = zeta_j^i (i < N/2) and w = V^{-1} z, f = (Re w | Im w) because
//    zeta_j^{N/2} = sqrt(-1).  V = T_{N/2} P (Sec. 2.3) and T_{N/2} = S_{N/4} ... S_1,
//    so V^{-1} z = P S_1^{-1} ... S_{N/4}^{-1} z: butterflies, then a bit reversal.
//  * Real CinS (Sec. 3.3.1, Appendix A): DFT'_{2l}(m) = T_l P_l fold(m).
//  * Fused conv (Sec. 3.3.2-3.3.4, Sec. 4): K^' = S_{N/2<-l} K^ applied column by
//    column; diagonal k holds K^'[c][(c+k) mod C] in slice c; BSGS pre-rotation.
//  * CoeffToSlot (Sec. 2.4): groups of consecutive inverse butterfly stages, each
//    turned into its cyclic diagonals by composing the stages' three diagonals.
#include <cmath>
#include <complex>
#include <map>
#include <vector>

#include "internal.h"

namespace nj {

typedef std::complex<double> cplx;

static int ilog2(int x)
{
    int r = 0;
    while ((1 << r) < x) r++;
    return r;
}

static int rev(int x, int bits)
{
    int r = 0;
    for (int i = 0; i < bits; i++) r = (r << 1) | ((x >> i) & 1);
    return r;
}

// W_k[t] = w_{8k}^(5^t mod 8k), t < k
static std::vector<cplx> w_diag(int k)
{
    std::vector<cplx> w(k);
    long long e = 1, mod = 8LL * k;
    for (int t = 0; t < k; t++) {
        double ang = 2.0 * M_PI * (double)e / (double)mod;
        w[t] = cplx(std::cos(ang), std::sin(ang));
        e = e * 5 % mod;
    }
    return w;
}

// x <- S_k x (or S_k^{-1} x) on blocks of 2k consecutive entries
static void butterfly_stage(std::vector<cplx> &x, int k, bool inverse)
{
    const std::vector<cplx> w = w_diag(k);
    const int n = (int)x.size();
    for (int b = 0; b < n; b += 2 * k)
        for (int t = 0; t < k; t++) {
            cplx a = x[b + t], c = x[b + k + t];
            if (!inverse) {
                cplx v = w[t] * c;
                x[b + t] = a + v;
                x[b + k + t] = a - v;
            } else {
                x[b + t] = 0.5 * (a + c);
                x[b + k + t] = 0.5 * (a - c) / w[t];
            }
        }
}

static void bit_reverse(std::vector<cplx> &x)
{
    const int n = (int)x.size(), bits = ilog2(n);
    for (int i = 0; i < n; i++) {
        int r = rev(i, bits);
        if (i < r) std::swap(x[i], x[r]);
    }
}

void encode_slots(int N, const double *z_re, const double *z_im, double scale, int64_t *out)
{
    const int n = N / 2;
    std::vector<cplx> x(n);
    for (int j = 0; j < n; j++) x[j] = cplx(z_re[j], z_im[j]);
    for (int k = n / 2; k >= 1; k /= 2) butterfly_stage(x, k, true);  // T^{-1} = S_1^{-1} ... S_{n/2}^{-1}
    bit_reverse(x);                                                    // P
    for (int i = 0; i < n; i++) {
        out[i] = (int64_t)std::nearbyint(scale * x[i].real());
        out[n + i] = (int64_t)std::nearbyint(scale * x[i].imag());
    }
}

void decode_slots(int N, const double *coeffs, double scale, double *z_re, double *z_im)
{
    const int n = N / 2;
    std::vector<cplx> x(n);
    for (int i = 0; i < n; i++) x[i] = cplx(coeffs[i] / scale, coeffs[n + i] / scale);
    bit_reverse(x);
    for (int k = 1; k < n; k *= 2) butterfly_stage(x, k, false);
    for (int j = 0; j < n; j++) z_re[j] = x[j].real(), z_im[j] = x[j].imag();
}

// DFT'_{2l}(m) = T_l P_l fold(m), fold(m)_i = m_i + sqrt(-1) m_{i+l}
static std::vector<cplx> dft_prime(const double *m, int ell)
{
    std::vector<cplx> x(ell);
    for (int i = 0; i < ell; i++) x[i] = cplx(m[i], m[i + ell]);
    bit_reverse(x);
    for (int k = 1; k < ell; k *= 2) butterfly_stage(x, k, false);
    return x;
}

void encode_cins(int N, const double *chans, int slice2, double scale, int64_t *out)
{
    const int ell = slice2 / 2, C = N / slice2;
    std::vector<double> zr(N / 2), zi(N / 2);
    for (int c = 0; c < C; c++) {
        std::vector<cplx> d = dft_prime(chans + (size_t)c * slice2, ell);
        for (int j = 0; j < ell; j++) zr[c * ell + j] = d[j].real(), zi[c * ell + j] = d[j].imag();
    }
    encode_slots(N, zr.data(), zi.data(), scale, out);
}

// ------------------------------------------------------------------ BSGS split

static int floordiv(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

void bsgs_split(nj_lt_t &lt, int n)
{
    lt.n_diag = (int)lt.js.size();
    if (lt.n1 <= 0) lt.n1 = (int)std::ceil(std::sqrt((double)lt.n_diag));
    lt.g_of.assign(lt.n_diag, 0);
    lt.i_of.assign(lt.n_diag, 0);
    std::map<int, int> bs, gs;
    for (int d = 0; d < lt.n_diag; d++) {
        int g = floordiv(lt.js[d], lt.n1);
        lt.g_of[d] = g;
        lt.i_of[d] = lt.js[d] - g * lt.n1;
        bs[lt.i_of[d]] = 1;
        gs[g] = 1;
    }
    lt.babies.clear();
    lt.giants.clear();
    for (auto &kv : bs) lt.babies.push_back(kv.first);
    for (auto &kv : gs) lt.giants.push_back(kv.first);
    (void)n;
}

// representative of offset r (a multiple of u) centred in [-h, n/u - h), h = (n/u)/2
static int centred_rep(long long r, int u, int n)
{
    const int span = n / u, h = span / 2;
    long long j = ((r / u) % span + span) % span;
    return (int)(((j + h) % span) - h);
}

static void rotr_inplace(std::vector<cplx> &v, long long r)
{
    const long long n = (long long)v.size();
    r = ((r % n) + n) % n;
    if (r == 0) return;
    std::vector<cplx> o(n);
    for (long long i = 0; i < n; i++) o[(i + r) % n] = v[i];
    v.swap(o);
}

// kernel polynomial: k(Y) = sum K[u][v] Y^{-((u-p)W + (v-p))} mod Y^{W^2} + 1
static std::vector<double> kernel_poly(const double *K, int f, int W)
{
    const int n = W * W, p = (f - 1) / 2;
    std::vector<double> k(n, 0.0);
    for (int u = 0; u < f; u++)
        for (int v = 0; v < f; v++) {
            int e = -((u - p) * W + (v - p));
            double val = K[u * f + v];
            if (e >= 0) k[e % n] += val;
            else k[(e + n) % n] -= val;  // Y^{-e'} = -Y^{n-e'}
        }
    return k;
}

// kernel polynomial of a tap list: k(Y) = sum w Y^{-(dy W + dx)} mod Y^{W^2} + 1
static std::vector<double> kernel_poly_taps(const std::vector<const nj_tap *> &taps, int W)
{
    const int n = W * W;
    std::vector<double> k(n, 0.0);
    for (const nj_tap *t : taps) {
        int e = -(t->dy * W + t->dx);
        if (e >= 0) k[e % n] += t->w;
        else k[(e + n) % n] -= t->w;
    }
    return k;
}

// Diagonals of a (possibly blocked) CinS conv given as taps (Sec. 3.3, Sec. 3.3.4):
// blocks (ob, ib) of C x C channels, diagonal k of a block holds K^[c][(c+k) mod C]
// (fuse: K^' = S'K^ instead).  The diagonal set is every k when fused, else the
// union of the nonzero ones over all blocks; nz[(ob bi + ib) nd + d] flags nonzero
// diagonals, zero ones are neither encoded nor multiplied.
nj_status build_block_diagonals(int N, int W, int c_in, int c_out, const nj_tap *taps, int n_taps, int fuse, int n1,
                                nj_lt_t &lt, std::vector<std::vector<double>> &dre,
                                std::vector<std::vector<double>> &dim)
{
    const int n = N / 2, ell = W * W / 2;
    if (W * W > N || ell < 1) return fail(NJ_EUNSUPPORTED, "conv plan: padded image larger than N");
    const int C = n / ell;
    const int bi = (c_in + C - 1) / C, bo = (c_out + C - 1) / C;
    std::map<std::pair<int, int>, std::vector<const nj_tap *>> by;
    for (int t = 0; t < n_taps; t++) {
        const nj_tap &tp = taps[t];
        if (tp.out_ch < 0 || tp.out_ch >= c_out || tp.in_ch < 0 || tp.in_ch >= c_in || std::abs(tp.dy) >= W ||
            std::abs(tp.dx) >= W)
            return fail(NJ_EINVAL, "conv plan: tap out of range");
        by[{tp.out_ch, tp.in_ch}].push_back(&tp);
    }
    std::vector<std::vector<std::vector<cplx>>> blocks((size_t)bo * bi);  // [ob bi + ib][k], empty = zero
    std::vector<char> used(C, fuse ? 1 : 0);
    for (int ob = 0; ob < bo; ob++)
        for (int ib = 0; ib < bi; ib++) {
            std::vector<std::vector<cplx>> Kh((size_t)C * C);  // [o][i] slices of length l, empty = zero
            bool any = false;
            for (int o = 0; o < C; o++)
                for (int i = 0; i < C; i++) {
                    auto it = by.find({ob * C + o, ib * C + i});
                    if (it == by.end()) continue;
                    std::vector<double> kp = kernel_poly_taps(it->second, W);
                    Kh[(size_t)o * C + i] = dft_prime(kp.data(), ell);
                    any = true;
                }
            auto &dg = blocks[(size_t)ob * bi + ib];
            dg.assign(C, {});
            if (!any) continue;
            if (fuse)  // columns of K^' = S_{n/2} ... S_l applied to (K^[0][i] | ... | K^[C-1][i])
                for (int i = 0; i < C; i++) {
                    std::vector<cplx> col((size_t)n, 0.0);
                    for (int o = 0; o < C; o++)
                        if (!Kh[(size_t)o * C + i].empty())
                            for (int j = 0; j < ell; j++) col[(size_t)o * ell + j] = Kh[(size_t)o * C + i][j];
                    for (int k = ell; k < n; k *= 2) butterfly_stage(col, k, false);
                    for (int o = 0; o < C; o++)
                        Kh[(size_t)o * C + i].assign(col.begin() + (size_t)o * ell, col.begin() + (size_t)(o + 1) * ell);
                }
            for (int k = 0; k < C; k++) {
                std::vector<cplx> v((size_t)n, 0.0);
                bool nz = false;
                for (int c = 0; c < C; c++) {
                    const auto &sl = Kh[(size_t)c * C + (c + k) % C];
                    if (sl.empty()) continue;
                    for (int j = 0; j < ell; j++) {
                        v[(size_t)c * ell + j] = sl[j];
                        nz = nz || sl[j] != cplx(0.0, 0.0);
                    }
                }
                if (!nz) continue;
                dg[k] = std::move(v);
                used[k] = 1;
            }
        }
    std::vector<int> ks;
    for (int k = 0; k < C; k++)
        if (used[k]) ks.push_back(k);
    if (ks.empty()) return fail(NJ_EINVAL, "conv plan: every weight is zero");
    lt.u = ell;
    lt.n1 = n1;
    lt.stages = fuse ? ilog2(C) : 0;  // StoC2 merged into the kernel matrix when fused
    lt.js.clear();
    for (int k : ks) lt.js.push_back(centred_rep((long long)k * ell, ell, n));
    bsgs_split(lt, n);
    const int nd = lt.n_diag;
    lt.bi = bi, lt.bo = bo;
    lt.nz.assign((size_t)bo * bi * nd, 0);
    dre.assign((size_t)bo * bi * nd, {});
    dim.assign((size_t)bo * bi * nd, {});
    for (int b = 0; b < bo * bi; b++)
        for (int d = 0; d < nd; d++) {
            std::vector<cplx> &v = blocks[b][ks[d]];
            if (v.empty()) continue;
            lt.nz[(size_t)b * nd + d] = 1;
            rotr_inplace(v, (long long)lt.g_of[d] * lt.n1 * lt.u);
            auto &r = dre[(size_t)b * nd + d], &m = dim[(size_t)b * nd + d];
            r.resize(n), m.resize(n);
            for (int j = 0; j < n; j++) r[j] = v[j].real(), m[j] = v[j].imag();
        }
    return NJ_OK;
}

// Slot permutations of the downsampling flows (Sec. 5, Algorithm 2; Appendix B), on one
// half (h = 0: the real CoeffToSlot output, slot j = coefficient rev(j); h = 1: the
// imaginary one, coefficient N/2 + rev(j)) of an image in the fused conv's coefficient
// layout, coefficient (y W + x) C + rev_C(c) = pixel (y, x) of channel c:
//   kind 0, decompose: (W, C) -> (W/2, 4C), channel 4 i + 2 b + a = phase image
//     I_i[a::2, b::2] (one block);
//   kind 1, densify: four sparse images (W, C) (stride-1 conv outputs) -> (W/2, 4C),
//     channel 4 i + m = even pixels I_i[0::2, 0::2] of input m (four blocks).
// Every output slot takes one input slot of the same half (0/1 diagonals, checked).
nj_status build_downsample_diagonals(int N, int kind, int W, int C, int half, int n1, nj_lt_t &lt,
                                     std::vector<std::vector<double>> &dre, std::vector<std::vector<double>> &dim)
{
    const int n = N / 2, ln = ilog2(n), lc = ilog2(C), W2 = W / 2, C2 = 4 * C, lc2 = lc + 2;
    if ((kind != 0 && kind != 1) || (half != 0 && half != 1) || W < 2 || W % 2 || C < 1 || (C & (C - 1)) ||
        (W & (W - 1)) || (long long)W * W * C != N)
        return fail(NJ_EINVAL, "downsample plan: need W, C powers of two with W^2 C = N, W >= 2");
    const int nb = kind == 0 ? 1 : 4;
    auto coef = [&](int c, int y, int x, int w, int cc, int lcc) { return (y * w + x) * cc + rev(c, lcc); };
    std::vector<std::vector<int>> src(nb, std::vector<int>(N, -1));  // output coefficient -> input coefficient
    for (int i = 0; i < C; i++)
        for (int y = 0; y < W2; y++)
            for (int x = 0; x < W2; x++) {
                if (kind == 0) {
                    for (int a = 0; a < 2; a++)
                        for (int b = 0; b < 2; b++)
                            src[0][coef(4 * i + 2 * b + a, y, x, W2, C2, lc2)] = coef(i, 2 * y + a, 2 * x + b, W, C, lc);
                } else {
                    for (int m = 0; m < 4; m++) src[m][coef(4 * i + m, y, x, W2, C2, lc2)] = coef(i, 2 * y, 2 * x, W, C, lc);
                }
            }
    std::vector<std::map<int, std::vector<cplx>>> blocks(nb);
    for (int b = 0; b < nb; b++)
        for (int j = 0; j < n; j++) {
            const int k = src[b][half * n + rev(j, ln)];
            if (k < 0) continue;
            if (k / n != half) return fail(NJ_EUNSUPPORTED, "downsample plan: a slot would cross the real/imaginary halves");
            const int js = rev(k % n, ln), r = ((js - j) % n + n) % n;
            std::vector<cplx> &v = blocks[b][r];
            if (v.empty()) v.assign(n, cplx(0.0, 0.0));
            v[j] = 1.0;
        }
    std::map<int, int> offs;
    for (auto &bl : blocks)
        for (auto &kv : bl) offs[centred_rep(kv.first, 1, n)] = kv.first;
    lt.u = 1;
    lt.n1 = n1;
    lt.stages = 0;
    lt.js.clear();
    for (auto &kv : offs) lt.js.push_back(kv.first);
    bsgs_split(lt, n);
    const int nd = lt.n_diag;
    lt.bi = nb, lt.bo = 1;
    lt.nz.assign((size_t)nb * nd, 0);
    dre.assign((size_t)nb * nd, {});
    dim.assign((size_t)nb * nd, {});
    for (int b = 0; b < nb; b++)
        for (int d = 0; d < nd; d++) {
            auto it = blocks[b].find(offs[lt.js[d]]);
            if (it == blocks[b].end()) continue;
            std::vector<cplx> v = it->second;
            lt.nz[(size_t)b * nd + d] = 1;
            rotr_inplace(v, (long long)lt.g_of[d] * lt.n1 * lt.u);
            auto &rr = dre[(size_t)b * nd + d], &mm = dim[(size_t)b * nd + d];
            rr.resize(n), mm.resize(n);
            for (int j = 0; j < n; j++) rr[j] = v[j].real(), mm[j] = v[j].imag();
        }
    if (nb == 1) lt.nz.clear();  // a single block: every diagonal is used
    return NJ_OK;
}

// A fully connected layer fused with the whole StoC (Sec. 4.2.1: slot encoding is CinS with
// l = 1, so the FC matrix takes the place of the conv's kernel matrix and StoC that of
// StoC2).  The input is slot-encoded with period n' (a power of two >= n_in, n_out): slots
// j, j + n', ... hold x_{j mod n'} (x_i = 0 for i >= n_in), i.e. the plaintext is a
// polynomial in X^{N/(2n')}.  With V' the decoding matrix of that subring (z' = V' w',
// g = (Re w' | Im w')), the transform applies M' = V' E W S (S: the first n_in slots, E:
// y into the real part of w') on every period, so the output's coefficient k N / (2n')
// holds y_k = (W x)_k: n' cyclic diagonals of period n'.
nj_status build_fc_diagonals(int N, int n_in, int n_out, const double *W, int n1, nj_lt_t &lt,
                             std::vector<std::vector<double>> &dre, std::vector<std::vector<double>> &dim)
{
    const int n = N / 2;
    int np = 1;
    while (np < n_in || np < n_out) np *= 2;
    if (n_in < 1 || n_out < 1 || np > n) return fail(NJ_EUNSUPPORTED, "FC plan: more features than N/2 slots");
    // column i of M' = V' applied to the real vector (W[0][i], ..., W[n_out-1][i], 0, ...)
    std::vector<std::vector<cplx>> M((size_t)np, std::vector<cplx>(np, cplx(0.0, 0.0)));  // M[row][col]
    for (int i = 0; i < n_in; i++) {
        std::vector<cplx> x(np, cplx(0.0, 0.0));
        for (int k = 0; k < n_out; k++) x[k] = cplx(W[(size_t)k * n_in + i], 0.0);
        bit_reverse(x);
        for (int k = 1; k < np; k *= 2) butterfly_stage(x, k, false);
        for (int r = 0; r < np; r++) M[r][i] = x[r];
    }
    lt.u = 1;
    lt.n1 = n1;
    lt.stages = ilog2(np);  // the whole StoC of the subring merged into the FC matrix
    lt.js.clear();
    for (int r = 0; r < np; r++) lt.js.push_back(centred_rep(r, 1, n));
    bsgs_split(lt, n);
    dre.assign(lt.n_diag, {});
    dim.assign(lt.n_diag, {});
    for (int d = 0; d < lt.n_diag; d++) {
        const int r = ((lt.js[d] % np) + np) % np;
        std::vector<cplx> v(n);
        for (int j = 0; j < n; j++) v[j] = M[j % np][(j % np + r) % np];
        rotr_inplace(v, (long long)lt.g_of[d] * lt.n1 * lt.u);
        dre[d].resize(n), dim[d].resize(n);
        for (int j = 0; j < n; j++) dre[d][j] = v[j].real(), dim[d][j] = v[j].imag();
    }
    return NJ_OK;
}

nj_status build_conv_diagonals(int N, int w0, int f, const double *weights, int n1, nj_lt_t &lt,
                               std::vector<std::vector<double>> &dre, std::vector<std::vector<double>> &dim)
{
    const int n = N / 2;
    const int p = (f - 1) / 2;
    int W = 1;
    while (W < w0 + p) W *= 2;
    const int ell = W * W / 2;
    if (W * W > N || f % 2 == 0) return fail(NJ_EUNSUPPORTED, "conv plan: image too large for N or even kernel");
    const int C = n / ell;
    // K^[o][i] = DFT'(k_{o,i}), then K^' columns = S_{n/2} ... S_l applied to (K^[0][i] | ... | K^[C-1][i])
    std::vector<std::vector<cplx>> Kp((size_t)C * C);  // [o][i] slices of length l
    for (int i = 0; i < C; i++) {
        std::vector<cplx> col(n);
        for (int o = 0; o < C; o++) {
            std::vector<double> kp = kernel_poly(weights + ((size_t)o * C + i) * f * f, f, W);
            std::vector<cplx> d = dft_prime(kp.data(), ell);
            for (int j = 0; j < ell; j++) col[(size_t)o * ell + j] = d[j];
        }
        for (int k = ell; k < n; k *= 2) butterfly_stage(col, k, false);
        for (int o = 0; o < C; o++) Kp[(size_t)o * C + i].assign(col.begin() + (size_t)o * ell, col.begin() + (size_t)(o + 1) * ell);
    }
    lt.u = ell;
    lt.n1 = n1;
    lt.stages = ilog2(C);  // StoC2 = S_{N/2 <- l} merged into the kernel matrix
    lt.js.clear();
    for (int k = 0; k < C; k++) lt.js.push_back(centred_rep((long long)k * ell, ell, n));
    bsgs_split(lt, n);
    dre.assign(lt.n_diag, {});
    dim.assign(lt.n_diag, {});
    for (int d = 0; d < lt.n_diag; d++) {
        const int k = ((lt.js[d] % C) + C) % C;
        std::vector<cplx> v(n);
        for (int c = 0; c < C; c++)
            for (int j = 0; j < ell; j++) v[(size_t)c * ell + j] = Kp[(size_t)c * C + (c + k) % C][j];
        rotr_inplace(v, (long long)lt.g_of[d] * lt.n1 * lt.u);
        dre[d].resize(n);
        dim[d].resize(n);
        for (int j = 0; j < n; j++) dre[d][j] = v[j].real(), dim[d][j] = v[j].imag();
    }
    return NJ_OK;
}

// Cyclic-diagonal form {r: v_r} of M = sum_r diag(v_r) (x <<< r), (x <<< r)[i] = x[i + r mod n]
typedef std::map<int, std::vector<cplx>> Diags;

static Diags inverse_stage_diags(int k, int n)
{
    const std::vector<cplx> w = w_diag(k);
    std::vector<cplx> v0(n), vp(n), vm(n);
    for (int i = 0; i < n; i++) {
        int t = i % (2 * k);
        if (t < k) v0[i] = 0.5, vp[i] = 0.5, vm[i] = 0.0;
        else v0[i] = -0.5 / w[t - k], vp[i] = 0.0, vm[i] = 0.5 / w[t - k];
    }
    Diags D;
    auto addd = [&](int r, const std::vector<cplx> &v) {
        r = ((r % n) + n) % n;
        auto it = D.find(r);
        if (it == D.end()) D[r] = v;
        else
            for (int i = 0; i < n; i++) it->second[i] += v[i];
    };
    addd(0, v0);
    addd(k, vp);
    addd(-k, vm);
    return D;
}

// S_k = diag(v0) + diag(vp)(.<<<k) + diag(vm)(.<<<-k): the forward butterflies
// (x_i + w x_{i+k}, x_{i-k} - w x_i) on every 2k-block
static Diags forward_stage_diags(int k, int n)
{
    const std::vector<cplx> w = w_diag(k);
    std::vector<cplx> v0(n), vp(n), vm(n);
    for (int i = 0; i < n; i++) {
        int t = i % (2 * k);
        if (t < k) v0[i] = 1.0, vp[i] = w[t], vm[i] = 0.0;
        else v0[i] = -w[t - k], vp[i] = 0.0, vm[i] = 1.0;
    }
    Diags D;
    auto addd = [&](int r, const std::vector<cplx> &v) {
        r = ((r % n) + n) % n;
        auto it = D.find(r);
        if (it == D.end()) D[r] = v;
        else
            for (int i = 0; i < n; i++) it->second[i] += v[i];
    };
    addd(0, v0);
    addd(k, vp);
    addd(-k, vm);
    return D;
}

// A B: diag(a_r)(.<<<r) diag(b_s)(.<<<s) = diag(a_r * (b_s <<< r)) (.<<<(r+s))
static Diags compose(const Diags &A, const Diags &B, int n)
{
    Diags Cm;
    for (auto &ra : A)
        for (auto &sb : B) {
            const int r = ra.first, t = (r + sb.first) % n;
            auto it = Cm.find(t);
            if (it == Cm.end()) it = Cm.emplace(t, std::vector<cplx>(n, 0.0)).first;
            std::vector<cplx> &dst = it->second;
            const std::vector<cplx> &a = ra.second, &b = sb.second;
            for (int i = 0; i < n; i++) dst[i] += a[i] * b[(i + r) % n];
        }
    return Cm;
}

nj_status build_cts_diagonals(int N, int groups, const int *n1s, std::vector<nj_lt_t> &lts,
                              std::vector<std::vector<std::vector<double>>> &dre,
                              std::vector<std::vector<std::vector<double>>> &dim)
{
    const int n = N / 2, S = ilog2(n);
    if (groups < 1 || groups > S) return fail(NJ_EINVAL, "CoeffToSlot plan: groups must be 1..log2(N/2)");
    std::vector<int> strides;
    for (int k = n / 2; k >= 1; k /= 2) strides.push_back(k);
    lts.assign(groups, nj_lt_t());
    dre.assign(groups, {});
    dim.assign(groups, {});
    int pos = 0;
    for (int g = 0; g < groups; g++) {
        const int sz = S / groups + (g < S % groups ? 1 : 0);
        Diags M;
        bool first = true;
        for (int s = pos; s < pos + sz; s++) {
            Diags D = inverse_stage_diags(strides[s], n);
            M = first ? D : compose(D, M, n);
            first = false;
        }
        const int u = strides[pos + sz - 1];
        pos += sz;
        if (g == groups - 1)
            for (auto &kv : M)
                for (auto &v : kv.second) v *= 0.5;
        nj_lt_t &lt = lts[g];
        lt.u = u;
        lt.n1 = n1s ? n1s[g] : 0;
        lt.stages = sz;
        lt.js.clear();
        std::vector<const std::vector<cplx> *> vecs;
        std::map<int, const std::vector<cplx> *> byj;
        for (auto &kv : M) byj[centred_rep(kv.first, u, n)] = &kv.second;
        for (auto &kv : byj) lt.js.push_back(kv.first);
        bsgs_split(lt, n);
        dre[g].assign(lt.n_diag, {});
        dim[g].assign(lt.n_diag, {});
        for (int d = 0; d < lt.n_diag; d++) {
            std::vector<cplx> v = *byj[lt.js[d]];
            rotr_inplace(v, (long long)lt.g_of[d] * lt.n1 * lt.u);
            dre[g][d].resize(n);
            dim[g][d].resize(n);
            for (int j = 0; j < n; j++) dre[g][d][j] = v[j].real(), dim[g][d][j] = v[j].imag();
        }
    }
    return NJ_OK;
}

// S_{l <- 1} = S_{l/2} ... S_1 (S_1 applied first) in `groups` consecutive groups of
// strides; a group's unit is its smallest stride
nj_status build_stoc1_diagonals(int N, int ell, int groups, std::vector<nj_lt_t> &lts,
                                std::vector<std::vector<std::vector<double>>> &dre,
                                std::vector<std::vector<std::vector<double>>> &dim)
{
    const int n = N / 2;
    if (ell < 2 || ell > n || (ell & (ell - 1))) return fail(NJ_EINVAL, "StoC1 plan: slice length must be a power of two in 2..N/2");
    const int S = ilog2(ell);
    if (groups < 1 || groups > S) return fail(NJ_EINVAL, "StoC1 plan: groups must be 1..log2(l)");
    std::vector<int> strides;
    for (int k = 1; k < ell; k *= 2) strides.push_back(k);
    lts.assign(groups, nj_lt_t());
    dre.assign(groups, {});
    dim.assign(groups, {});
    int pos = 0;
    for (int g = 0; g < groups; g++) {
        const int sz = S / groups + (g < S % groups ? 1 : 0);
        Diags M;
        for (int s = pos; s < pos + sz; s++) {
            Diags D = forward_stage_diags(strides[s], n);
            M = s == pos ? D : compose(D, M, n);
        }
        const int u = strides[pos];
        pos += sz;
        nj_lt_t &lt = lts[g];
        lt.u = u;
        lt.n1 = 0;
        lt.stages = sz;
        lt.js.clear();
        std::map<int, const std::vector<cplx> *> byj;
        for (auto &kv : M) byj[centred_rep(kv.first, u, n)] = &kv.second;
        for (auto &kv : byj) lt.js.push_back(kv.first);
        bsgs_split(lt, n);
        dre[g].assign(lt.n_diag, {});
        dim[g].assign(lt.n_diag, {});
        for (int d = 0; d < lt.n_diag; d++) {
            std::vector<cplx> v = *byj[lt.js[d]];
            rotr_inplace(v, (long long)lt.g_of[d] * lt.n1 * lt.u);
            dre[g][d].resize(n);
            dim[g][d].resize(n);
            for (int j = 0; j < n; j++) dre[g][d][j] = v[j].real(), dim[g][d][j] = v[j].imag();
        }
    }
    return NJ_OK;
}

// Chebyshev interpolant of degree `degree` at the first-kind nodes x_k = cos(pi (k + 1/2) / m),
// m = degree + 1: c_j = (2 - [j = 0]) / m * sum_k f(x_k) cos(pi j (k + 1/2) / m)
void cheb_interpolate_cos(int degree, double K, int r, double *c)
{
    const int m = degree + 1;
    std::vector<double> f(m);
    for (int k = 0; k < m; k++) {
        const double x = std::cos(M_PI * (k + 0.5) / m);
        f[k] = std::cos(2.0 * M_PI * (K * x - 0.25) / std::ldexp(1.0, r));
    }
    for (int j = 0; j < m; j++) {
        double acc = 0.0;
        for (int k = 0; k < m; k++) acc += f[k] * std::cos(M_PI * j * (k + 0.5) / m);
        c[j] = (j == 0 ? 1.0 : 2.0) * acc / m;
    }
}

}  // namespace nj
