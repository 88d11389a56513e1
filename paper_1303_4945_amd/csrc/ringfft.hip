// Per-ring FFTs of the paper's Eqs. 3 and 6 on gfx950.
//
// Synthesis (Eq. 3), per ring y: c_m = F_{m,y} e^{i m phi0_y} for |m| <= mmax
// (c_{-m} = conj c_m), aliased onto the Nphi_y bins b_k = sum_{m = k mod Nphi} c_m,
// then p_x = sum_k b_k e^{2 pi i k x / Nphi} (an unnormalised inverse real DFT).
// Analysis (Eq. 6): G_{m,y} = w_y e^{-i m phi0} sum_x p_x e^{-2 pi i m x / Nphi}.
//
// Each work item is one complex FFT held in LDS:
//   * even Nphi: one ring, the standard half-length packing z_n = x_2n + i x_2n+1;
//   * odd Nphi:  two rings of equal length (a ring and its mirror) packed as
//     z = a + i b.
// A complex length L that factors into 2,3,5,7,11,13 is done by an in-place
// mixed-radix transform (decimation in frequency: natural -> digit-reversed
// order; decimation in time: digit-reversed -> natural), the spectrum being
// read or written at digit-reversed positions so that no permutation pass is
// needed.  A prime L whose L-1 factors that way uses Rader's reordering into a
// cyclic convolution of length L-1 (two in-LDS transforms of length L-1).
// Other lengths use Bluestein's chirp transform with a power-of-two inner
// length M (>= 2L-1); when M complex doubles exceed the LDS, the inner
// transform is split by one radix-2 step into two halves processed one after
// the other, the first half's result being kept in registers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <tuple>
#include <vector>

#include "sht_internal.h"

namespace sht {

constexpr int FFT_MAXRAD = 16;

enum { FFT_DIRECT = 0, FFT_BLUE = 1, FFT_BLUE_SPLIT = 2, FFT_RADER = 3 };
// kernel variants: everything in LDS / split Bluestein / Rader
enum { KMODE_LDS = 0, KMODE_SPLIT = 1, KMODE_RADER = 2 };
constexpr int FFT_NREG = 8;   // register slots per thread in split and Rader mode
enum { ROW_PAIR = 0, ROW_HALF = 1 };

struct FftInner {       // an in-LDS complex FFT of length n
    int n;
    int nrad;
    int rad[FFT_MAXRAD];
    int fuse[FFT_MAXRAD];   // 1: pass i runs together with pass i + 1 in registers
    int64_t tw;         // offset of e^{-2 pi i j / n}, j < n
    int64_t pos;        // offset of pos_of_freq[f], f < n
};

struct FftLen {         // complex transform of length L
    int L;
    int kind;
    int M;              // Bluestein inner length (full M, also in split mode); Rader: L-1
    int inner;          // index of the FftInner used (length L, M, M/2 or L-1)
    int64_t chirp;      // Bluestein: L entries e^{+i pi n^2 / L};
                        // Rader: L-1 entries b_q = e^{+2 pi i g^{-q} / L}
    int64_t bhat_p;     // kernel spectrum for sign +  (M entries; split: even half then odd half)
    int64_t bhat_m;     // kernel spectrum for sign -
    int64_t wm;         // split: e^{-2 pi i n / M}, n < M/2
    int64_t rpos;       // Rader: itab offset of the LDS position of x_n, n < L: p with g^p = n, L-1 for n = 0
    int64_t qpos;       // Rader: itab offset of q(k) with g^{-q} = k mod L, 0 < k < L
    int lds_complex;    // LDS buffer size in complex elements
};

struct FftRow {
    int mode;           // ROW_PAIR or ROW_HALF
    int ya, yb;         // rings (yb = -1: none)
    int len;            // FftLen index
    int nphi;
    int64_t half_tw;    // ROW_HALF: e^{-2 pi i k / nphi}, k < nphi/2
};

struct FftView {
    const FftInner *inner;
    const FftLen *lens;
    const FftRow *rows;
    const double2 *ctab;     // complex tables
    const int *itab;         // integer tables
    const int64_t *ofs;      // ring pixel offsets
    int64_t stride;
    const double *weight;
    const double2 *rot;      // per ring: 64 fine + ncoarse coarse rotations e^{i m phi0}
    int nrot;                // entries per ring
    int rot_trivial;         // 1: phi0 = 0 on every ring (no rotation)
    const int *mvalid;       // per ring: largest meaningful m
    int mmax, nrings, ncomp;
    int64_t npix;
};

// ------------------------------------------------------------------ device

// LDS index with one complex of padding every 8 elements: the strided
// butterfly accesses of radix 2, 4 and 8 then fall into distinct bank groups.
// The Rader kernels of inner lengths that are not powers of two (their
// butterflies mostly read consecutive elements) run unpadded: there the
// padding only broke up contiguous accesses (PAD = false).
template <bool PAD>
__device__ __forceinline__ int padi(int i) { return PAD ? i + (i >> 3) : i; }
template <int MODE, bool POW2>
constexpr bool lds_pad() { return MODE != KMODE_RADER || POW2; }
__device__ __forceinline__ int PADI(int i) { return padi<true>(i); }
constexpr int lds_padded(int n) { return n + (n >> 3) + 1; }

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
// multiply by -i (fwd = true) or +i
__device__ __forceinline__ double2 cmul_mi(double2 a, bool fwd)
{
    return fwd ? make_double2(a.y, -a.x) : make_double2(-a.y, a.x);
}

// Element loop n = threadIdx.x + j blockDim.x over [0, count), U elements
// per thread at a time: get(n) for all of them first (their global loads in
// flight together: one memory latency per U elements instead of one per
// element), then put(n, value).  Indices past the end are clamped to
// count - 1 rather than branched on, so the gets form straight-line code.
// GUARD = false: put also runs for clamped indices (it must then be a plain
// store of get's value, which the owner of count - 1 stores too); GUARD = true
// (read-modify-write of shared data): put runs for n < count only.
// The synthesis kernels take four elements per thread at a time; the analysis
// kernels (two map reads per element in, two phase stores per element out)
// take two, which measured faster for them at the 8191-point rings.
constexpr int LOOP_U = 4;
constexpr int LOOP_U_ANAL = 2;
template <bool GUARD, int U, typename Get, typename Put>
__device__ __forceinline__ void batched_loop(int count, Get get, Put put)
{
    const int T = (int)blockDim.x;
    for (int n0 = threadIdx.x; n0 < count; n0 += U * T) {
        decltype(get(0)) v[U];
#pragma unroll
        for (int j = 0; j < U; ++j) v[j] = get(min(n0 + j * T, count - 1));
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const int n = n0 + j * T;
            if (!GUARD) put(min(n, count - 1), v[j]);
            else if (n < count) put(n, v[j]);
        }
    }
}

// small DFT out_k = sum_j v_j w_r^{jk}, w_r = e^{-2 pi i / r} (fwd) or conjugate.
template <int R>
__device__ __forceinline__ void small_dft(double2 *v, bool fwd, const double2 *tw, int n)
{
    if constexpr (R == 2) {
        double2 a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if constexpr (R == 4) {
        double2 a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
        double2 c = cadd(v[1], v[3]), d = cmul_mi(csub(v[1], v[3]), fwd);
        v[0] = cadd(a, c);
        v[2] = csub(a, c);
        v[1] = cadd(b, d);
        v[3] = csub(b, d);
    } else if constexpr (R == 8) {
        // two radix-4 DFTs over even/odd inputs, then a radix-2 combination
        double2 e[4] = {v[0], v[2], v[4], v[6]}, o[4] = {v[1], v[3], v[5], v[7]};
        small_dft<4>(e, fwd, tw, n);
        small_dft<4>(o, fwd, tw, n);
        const double h = 0.70710678118654752440;
        // o[k] *= w8^k
        o[1] = fwd ? make_double2(h * (o[1].x + o[1].y), h * (o[1].y - o[1].x))
                   : make_double2(h * (o[1].x - o[1].y), h * (o[1].y + o[1].x));
        o[2] = cmul_mi(o[2], fwd);
        o[3] = fwd ? make_double2(h * (-o[3].x + o[3].y), h * (-o[3].y - o[3].x))
                   : make_double2(h * (-o[3].x - o[3].y), h * (-o[3].y + o[3].x));
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[k] = cadd(e[k], o[k]);
            v[k + 4] = csub(e[k], o[k]);
        }
    } else {
        // generic odd radix: roots from the length-n table (n divisible by R)
        double2 w[R];
        const int step = n / R;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            double2 t = tw[j * step];
            w[j] = fwd ? t : cconj(t);
        }
        double2 out[R];
#pragma unroll
        for (int k = 0; k < R; ++k) {
            double2 s = v[0];
#pragma unroll
            for (int j = 1; j < R; ++j) {
                const double2 ww = w[(j * k) % R];
                s.x += v[j].x * ww.x - v[j].y * ww.y;
                s.y += v[j].x * ww.y + v[j].y * ww.x;
            }
            out[k] = s;
        }
#pragma unroll
        for (int k = 0; k < R; ++k) v[k] = out[k];
    }
}

// Twiddle w = tw[idx] (conjugated for the inverse).  Its powers w^k are
// formed by repeated multiplication where they are applied (one table load per
// butterfly; a few ulp of error for the radices used here).
__device__ __forceinline__ double2 tw_base(const double2 *tw, int idx, bool fwd)
{
    const double2 t = tw[idx];
    return fwd ? t : cconj(t);
}

// v[j S] *= w^j, j = 1 .. R-1
template <int R, int S = 1>
__device__ __forceinline__ void apply_powers(double2 *v, double2 w)
{
    double2 p = w;
#pragma unroll
    for (int j = 1; j < R; ++j) {
        v[j * S] = cmul(v[j * S], p);
        if (j + 1 < R) p = cmul(p, w);
    }
}

// one pass over the block of length Lb split by radix R (stride Ln = Lb / R)
template <int R, bool DIT, bool PAD = true>
__device__ __forceinline__ void fft_pass(double2 *buf, int n, int Lb, bool fwd, const double2 *tw)
{
    const int Ln = Lb / R;
    const int nb = n / R;
    const int tstep = n / Lb;
#pragma unroll 1
    for (int q = threadIdx.x; q < nb; q += blockDim.x) {
        const int b = q / Ln;
        const int n1 = q - b * Ln;
        const int base = b * Lb + n1;
        double2 v[R];
#pragma unroll
        for (int j = 0; j < R; ++j) v[j] = buf[padi<PAD>(base + j * Ln)];
        const double2 w = tw_base(tw, tstep * n1, fwd);
        if constexpr (DIT) {
            apply_powers<R>(v, w);
            small_dft<R>(v, fwd, tw, n);
        } else {
            small_dft<R>(v, fwd, tw, n);
            apply_powers<R>(v, w);
        }
#pragma unroll
        for (int j = 0; j < R; ++j) buf[padi<PAD>(base + j * Ln)] = v[j];
    }
    __syncthreads();
}

// cos and sin of 2 pi m / R for m = 1 .. (R-1)/2 (index 0 unused), rounded
// from extended-precision values
template <int R> struct OddRoots;
template <> struct OddRoots<3> {
    static constexpr double c[2] = {1.0, -0.5};
    static constexpr double s[2] = {0.0, 0.8660254037844386};
};
template <> struct OddRoots<5> {
    static constexpr double c[3] = {1.0, 0.30901699437494745, -0.8090169943749475};
    static constexpr double s[3] = {0.0, 0.9510565162951535, 0.5877852522924731};
};
template <> struct OddRoots<7> {
    static constexpr double c[4] = {1.0, 0.6234898018587335, -0.2225209339563144,
                                    -0.9009688679024191};
    static constexpr double s[4] = {0.0, 0.7818314824680298, 0.9749279121818236,
                                    0.4338837391175581};
};
template <> struct OddRoots<11> {
    static constexpr double c[6] = {1.0, 0.8412535328311812, 0.41541501300188644,
                                    -0.14231483827328514, -0.6548607339452851,
                                    -0.9594929736144974};
    static constexpr double s[6] = {0.0, 0.5406408174555976, 0.9096319953545183,
                                    0.9898214418809327, 0.7557495743542583,
                                    0.28173255684142967};
};
template <> struct OddRoots<13> {
    static constexpr double c[7] = {1.0, 0.8854560256532099, 0.5680647467311558,
                                    0.12053668025532305, -0.3546048870425356,
                                    -0.7485107481711011, -0.970941817426052};
    static constexpr double s[7] = {0.0, 0.46472317204376856, 0.8229838658936564,
                                    0.992708874098054, 0.9350162426854148,
                                    0.6631226582407952, 0.23931566428755777};
};

// One pass with an odd radix R, in the symmetric form: with s_j = v_j + v_{R-j}
// and d_j = v_j - v_{R-j}, out_k = A_k - i B_k and out_{R-k} = A_k + i B_k where
// A_k = v_0 + sum_j s_j cos(2 pi jk/R) and B_k = sum_j d_j sin(2 pi jk/R) (sine
// sign flipped for the inverse).  Outputs go to LDS as soon as they are formed,
// so no second register array is live.
template <int R, bool DIT, bool PAD = true>
__device__ __forceinline__ void fft_pass_odd(double2 *buf, int n, int Lb, bool fwd, const double2 *tw)
{
    constexpr int H = (R - 1) / 2;
    const int Ln = Lb / R;
    const int nb = n / R;
    const int tstep = n / Lb;
    const double ssign = fwd ? 1.0 : -1.0;   // w^m = cos - i ssign sin
#pragma unroll 1
    for (int q = threadIdx.x; q < nb; q += blockDim.x) {
        const int b = q / Ln;
        const int n1 = q - b * Ln;
        const int base = b * Lb + n1;
        double2 v[R];
#pragma unroll
        for (int j = 0; j < R; ++j) v[j] = buf[padi<PAD>(base + j * Ln)];
        const double2 w = tw_base(tw, tstep * n1, fwd);
        if constexpr (DIT) apply_powers<R>(v, w);
        // DIF: outputs k and R - k take w^k and w^(R-k), formed upwards from w
        // and downwards from w^(R-1)
        double2 pk = w, qk = make_double2(1.0, 0.0);
        if constexpr (!DIT) qk = tw_base(tw, tstep * n1 * (R - 1), fwd);
        const double2 wc = cconj(w);
        const double2 v0 = v[0];
        double2 sum0 = v0;
#pragma unroll
        for (int j = 1; j <= H; ++j) {
            const double2 sj = cadd(v[j], v[R - j]);
            const double2 dj = csub(v[j], v[R - j]);
            v[j] = sj;
            v[R - j] = dj;
            sum0 = cadd(sum0, sj);
        }
        buf[padi<PAD>(base)] = sum0;
#pragma unroll
        for (int k = 1; k <= H; ++k) {
            double2 A = v0, B = make_double2(0.0, 0.0);
#pragma unroll
            for (int j = 1; j <= H; ++j) {
                const int m = (j * k) % R;
                const double c = (m <= H) ? OddRoots<R>::c[m] : OddRoots<R>::c[R - m];
                const double sn = ssign * ((m <= H) ? OddRoots<R>::s[m] : -OddRoots<R>::s[R - m]);
                A.x += v[j].x * c;
                A.y += v[j].y * c;
                B.x += v[R - j].x * sn;
                B.y += v[R - j].y * sn;
            }
            double2 ok = make_double2(A.x + B.y, A.y - B.x);
            double2 okr = make_double2(A.x - B.y, A.y + B.x);
            if constexpr (!DIT) {
                ok = cmul(ok, pk);
                okr = cmul(okr, qk);
                pk = cmul(pk, w);
                qk = cmul(qk, wc);
            }
            buf[padi<PAD>(base + k * Ln)] = ok;
            buf[padi<PAD>(base + (R - k) * Ln)] = okr;
        }
    }
    __syncthreads();
}

// DFTs in registers over the elements v[j S], j < R (outputs back in place).
// Odd radices in the symmetric form of fft_pass_odd.
template <int R, int S>
__device__ __forceinline__ void dft_odd_reg(double2 *v, bool fwd)
{
    constexpr int H = (R - 1) / 2;
    const double ssign = fwd ? 1.0 : -1.0;
    double2 sv[H + 1], dv[H + 1];
    const double2 v0 = v[0];
    double2 sum0 = v0;
#pragma unroll
    for (int j = 1; j <= H; ++j) {
        sv[j] = cadd(v[j * S], v[(R - j) * S]);
        dv[j] = csub(v[j * S], v[(R - j) * S]);
        sum0 = cadd(sum0, sv[j]);
    }
    v[0] = sum0;
#pragma unroll
    for (int k = 1; k <= H; ++k) {
        double2 A = v0, B = make_double2(0.0, 0.0);
#pragma unroll
        for (int j = 1; j <= H; ++j) {
            const int m = (j * k) % R;
            const double c = (m <= H) ? OddRoots<R>::c[m] : OddRoots<R>::c[R - m];
            const double sn = ssign * ((m <= H) ? OddRoots<R>::s[m] : -OddRoots<R>::s[R - m]);
            A.x += sv[j].x * c;
            A.y += sv[j].y * c;
            B.x += dv[j].x * sn;
            B.y += dv[j].y * sn;
        }
        v[k * S] = make_double2(A.x + B.y, A.y - B.x);
        v[(R - k) * S] = make_double2(A.x - B.y, A.y + B.x);
    }
}

template <int R, int S>
__device__ __forceinline__ void dft_reg(double2 *v, bool fwd)
{
    if constexpr (R == 2) {
        const double2 a = v[0], b = v[S];
        v[0] = cadd(a, b);
        v[S] = csub(a, b);
    } else if constexpr (R == 4) {
        const double2 a = cadd(v[0], v[2 * S]), b = csub(v[0], v[2 * S]);
        const double2 c = cadd(v[S], v[3 * S]), d = cmul_mi(csub(v[S], v[3 * S]), fwd);
        v[0] = cadd(a, c);
        v[2 * S] = csub(a, c);
        v[S] = cadd(b, d);
        v[3 * S] = csub(b, d);
    } else if constexpr (R == 8) {
        // radix-4 DFTs of the even and odd elements, then a radix-2 combination
        dft_reg<4, 2 * S>(v, fwd);
        dft_reg<4, 2 * S>(v + S, fwd);
        const double h = 0.70710678118654752440;
        double2 o1 = v[3 * S], o2 = v[5 * S], o3 = v[7 * S];
        o1 = fwd ? make_double2(h * (o1.x + o1.y), h * (o1.y - o1.x))
                 : make_double2(h * (o1.x - o1.y), h * (o1.y + o1.x));
        o2 = cmul_mi(o2, fwd);
        o3 = fwd ? make_double2(h * (-o3.x + o3.y), h * (-o3.y - o3.x))
                 : make_double2(h * (-o3.x - o3.y), h * (-o3.y + o3.x));
        const double2 e0 = v[0], e1 = v[2 * S], e2 = v[4 * S], e3 = v[6 * S], o0 = v[S];
        v[0] = cadd(e0, o0);
        v[4 * S] = csub(e0, o0);
        v[S] = cadd(e1, o1);
        v[5 * S] = csub(e1, o1);
        v[2 * S] = cadd(e2, o2);
        v[6 * S] = csub(e2, o2);
        v[3 * S] = cadd(e3, o3);
        v[7 * S] = csub(e3, o3);
    } else {
        dft_odd_reg<R, S>(v, fwd);
    }
}

// Two consecutive passes (radix R1 on blocks of Lb, then radix R2 on blocks of
// Lb / R1) in one sweep: each thread owns the R1 R2 elements
// base + j LnA + jb LnB (LnA = Lb / R1, LnB = LnA / R2), which both passes
// combine only among themselves, so the intermediate values stay in registers
// and the data cross LDS once.  DIT runs the two passes in the reverse order
// with the twiddles before each DFT.  Same results as fft_pass twice.
template <int R1, int R2, bool DIT, bool PAD = true>
__device__ __forceinline__ void fft_pass2(double2 *buf, int n, int Lb, bool fwd, const double2 *tw)
{
    const int LnA = Lb / R1;
    const int LnB = LnA / R2;
    const int nb = n / (R1 * R2);
    const int tA = n / Lb, tB = n / LnA;   // twiddle steps of the two passes
#pragma unroll 1
    for (int q = threadIdx.x; q < nb; q += blockDim.x) {
        const int b = q / LnB;
        const int n1 = q - b * LnB;
        const int base = b * Lb + n1;
        // element (j, jb) at v[j R2 + jb]
        double2 v[R1 * R2];
#pragma unroll
        for (int j = 0; j < R1; ++j)
#pragma unroll
            for (int jb = 0; jb < R2; ++jb) v[j * R2 + jb] = buf[padi<PAD>(base + j * LnA + jb * LnB)];
        if constexpr (!DIT) {
#pragma unroll
            for (int jb = 0; jb < R2; ++jb) {
                dft_reg<R1, R2>(v + jb, fwd);
                apply_powers<R1, R2>(v + jb, tw_base(tw, tA * (n1 + jb * LnB), fwd));
            }
            const double2 wb = tw_base(tw, tB * n1, fwd);
#pragma unroll
            for (int k = 0; k < R1; ++k) {
                dft_reg<R2, 1>(v + k * R2, fwd);
                apply_powers<R2, 1>(v + k * R2, wb);
            }
        } else {
            const double2 wb = tw_base(tw, tB * n1, fwd);
#pragma unroll
            for (int j = 0; j < R1; ++j) {
                apply_powers<R2, 1>(v + j * R2, wb);
                dft_reg<R2, 1>(v + j * R2, fwd);
            }
#pragma unroll
            for (int kb = 0; kb < R2; ++kb) {
                apply_powers<R1, R2>(v + kb, tw_base(tw, tA * (n1 + kb * LnB), fwd));
                dft_reg<R1, R2>(v + kb, fwd);
            }
        }
#pragma unroll
        for (int k = 0; k < R1; ++k)
#pragma unroll
            for (int kb = 0; kb < R2; ++kb) buf[padi<PAD>(base + k * LnA + kb * LnB)] = v[k * R2 + kb];
    }
    __syncthreads();
}

// fused pairs that occur (the host orders each pair with R1 >= R2)
template <bool DIT, bool POW2, bool PAD = true>
__device__ __forceinline__ void fft_pass2_any(double2 *buf, int n, int Lb, int r1, int r2, bool fwd,
                                              const double2 *tw)
{
    switch (r1 * 16 + r2) {
    case 2 * 16 + 2: fft_pass2<2, 2, DIT, PAD>(buf, n, Lb, fwd, tw); break;
    case 4 * 16 + 2: fft_pass2<4, 2, DIT, PAD>(buf, n, Lb, fwd, tw); break;
    default:
        if constexpr (!POW2) {
            switch (r1 * 16 + r2) {
            case 3 * 16 + 2: fft_pass2<3, 2, DIT, PAD>(buf, n, Lb, fwd, tw); break;
            case 3 * 16 + 3: fft_pass2<3, 3, DIT, PAD>(buf, n, Lb, fwd, tw); break;
            case 5 * 16 + 2: fft_pass2<5, 2, DIT, PAD>(buf, n, Lb, fwd, tw); break;
            case 7 * 16 + 2: fft_pass2<7, 2, DIT, PAD>(buf, n, Lb, fwd, tw); break;
            default: break;
            }
        }
        break;
    }
}

// POW2: only radices 2, 4, 8 occur (keeps the odd-radix code, and its
// registers, out of the power-of-two kernels)
template <bool DIT, bool POW2, bool PAD = true>
__device__ __forceinline__ void fft_pass_any(double2 *buf, int n, int Lb, int r, bool fwd, const double2 *tw)
{
    switch (r) {
    case 2: fft_pass<2, DIT, PAD>(buf, n, Lb, fwd, tw); break;
    case 4: fft_pass<4, DIT, PAD>(buf, n, Lb, fwd, tw); break;
    case 8: fft_pass<8, DIT, PAD>(buf, n, Lb, fwd, tw); break;
    default:
        if constexpr (!POW2) {
            switch (r) {
            case 3: fft_pass_odd<3, DIT, PAD>(buf, n, Lb, fwd, tw); break;
            case 5: fft_pass_odd<5, DIT, PAD>(buf, n, Lb, fwd, tw); break;
            case 7: fft_pass_odd<7, DIT, PAD>(buf, n, Lb, fwd, tw); break;
            case 11: fft_pass_odd<11, DIT, PAD>(buf, n, Lb, fwd, tw); break;
            case 13: fft_pass_odd<13, DIT, PAD>(buf, n, Lb, fwd, tw); break;
            default: break;
            }
        }
        break;
    }
}

// natural order in, digit-reversed out
template <bool POW2, bool PAD = true>
__device__ __forceinline__ void fft_dif(double2 *buf, const FftInner &in, bool fwd, const double2 *ctab)
{
    const double2 *tw = ctab + in.tw;
    int Lb = in.n;
    for (int i = 0; i < in.nrad;) {
        if (in.fuse[i]) {
            fft_pass2_any<false, POW2, PAD>(buf, in.n, Lb, in.rad[i], in.rad[i + 1], fwd, tw);
            Lb /= in.rad[i] * in.rad[i + 1];
            i += 2;
        } else {
            fft_pass_any<false, POW2, PAD>(buf, in.n, Lb, in.rad[i], fwd, tw);
            Lb /= in.rad[i];
            i += 1;
        }
    }
}

// digit-reversed in, natural order out
template <bool POW2, bool PAD = true>
__device__ __forceinline__ void fft_dit(double2 *buf, const FftInner &in, bool fwd, const double2 *ctab)
{
    const double2 *tw = ctab + in.tw;
    int Lb = 1;
    for (int i = in.nrad - 1; i >= 0;) {
        if (i >= 1 && in.fuse[i - 1]) {
            Lb *= in.rad[i - 1] * in.rad[i];
            fft_pass2_any<true, POW2, PAD>(buf, in.n, Lb, in.rad[i - 1], in.rad[i], fwd, tw);
            i -= 2;
        } else {
            Lb *= in.rad[i];
            fft_pass_any<true, POW2, PAD>(buf, in.n, Lb, in.rad[i], fwd, tw);
            i -= 1;
        }
    }
}

// Complex DFT of length L with sign fwd (e^{-}) or inverse (e^{+}), natural
// order in and out, by Bluestein's chirp convolution of length M (a power of
// two).  buf holds the input x_n, n < L; on return buf holds X_k, k < L.
template <bool POW2>
__device__ __forceinline__ void bluestein(double2 *buf, const FftView &fv, const FftLen &d, bool fwd)
{
    const FftInner &in = fv.inner[d.inner];
    const double2 *chirp = fv.ctab + d.chirp;
    const double2 *bh = fv.ctab + (fwd ? d.bhat_m : d.bhat_p);
    const int L = d.L;
    // chirp for sign s: w_n = e^{s i pi n^2/L}; table holds s = +
    auto wch = [&](int n) { double2 c = chirp[n]; return fwd ? cconj(c) : c; };
    const int M = d.M;
    auto put = [&](int n, double2 v) { buf[PADI(n)] = v; };
    batched_loop<true, LOOP_U>(M, [&](int n) { return n < L ? cmul(buf[PADI(n)], wch(n)) : make_double2(0.0, 0.0); },
                       put);
    __syncthreads();
    fft_dif<POW2>(buf, in, true, fv.ctab);
    batched_loop<true, LOOP_U>(M, [&](int p) { return cmul(buf[PADI(p)], bh[p]); }, put);
    __syncthreads();
    fft_dit<POW2>(buf, in, false, fv.ctab);
    batched_loop<true, LOOP_U>(L, [&](int k) { return cmul(buf[PADI(k)], wch(k)); }, put);
    __syncthreads();
}

// Bluestein with the length-M convolution done as two length-M/2 halves (even
// and odd output frequencies of the first radix-2 step), for lengths whose M
// does not fit LDS.  The input is not kept: load(n) produces x_n (n < L) again
// for the second half.  Requires NREG * blockDim.x >= M/2.  On return buf holds
// X_k, k < L, in natural order.
template <int NREG, bool POW2, typename Load>
__device__ __forceinline__ void bluestein_split(double2 *buf, const FftView &fv, const FftLen &d, bool fwd,
                                Load load)
{
    const FftInner &in = fv.inner[d.inner];
    const double2 *chirp = fv.ctab + d.chirp;
    const double2 *bh = fv.ctab + (fwd ? d.bhat_m : d.bhat_p);
    const int L = d.L;
    auto wch = [&](int n) { double2 c = chirp[n]; return fwd ? cconj(c) : c; };
    const int Mh = d.M / 2;
    const double2 *wm = fv.ctab + d.wm;
    double2 er[NREG];
    // even frequencies: FFT_{M/2}(a), a_n = x_n w_n, times kernel, inverse
    for (int n = threadIdx.x; n < Mh; n += blockDim.x)
        buf[PADI(n)] = (n < L) ? cmul(load(n), wch(n)) : make_double2(0.0, 0.0);
    __syncthreads();
    fft_dif<POW2>(buf, in, true, fv.ctab);
    for (int p = threadIdx.x; p < Mh; p += blockDim.x) buf[PADI(p)] = cmul(buf[PADI(p)], bh[p]);
    __syncthreads();
    fft_dit<POW2>(buf, in, false, fv.ctab);
#pragma unroll
    for (int j = 0; j < NREG; ++j) {
        const int n = threadIdx.x + j * blockDim.x;
        er[j] = (n < Mh) ? buf[PADI(n)] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    // odd frequencies: FFT_{M/2}(a_n w_M^n)
    for (int n = threadIdx.x; n < Mh; n += blockDim.x)
        buf[PADI(n)] = (n < L) ? cmul(cmul(load(n), wch(n)), wm[n]) : make_double2(0.0, 0.0);
    __syncthreads();
    fft_dif<POW2>(buf, in, true, fv.ctab);
    for (int p = threadIdx.x; p < Mh; p += blockDim.x) buf[PADI(p)] = cmul(buf[PADI(p)], bh[Mh + p]);
    __syncthreads();
    fft_dit<POW2>(buf, in, false, fv.ctab);
    // c_n = E_n + w_M^{-n} O_n ; X_n = w_n c_n (each thread rewrites its own entries)
#pragma unroll
    for (int j = 0; j < NREG; ++j) {
        const int n = threadIdx.x + j * blockDim.x;
        if (n < L) {
            const double2 c = cadd(er[j], cmul(buf[PADI(n)], cconj(wm[n])));
            buf[PADI(n)] = cmul(c, wch(n));
        }
    }
    __syncthreads();
}

// e^{i m phi0} of ring y for 0 <= m (fine/coarse split by 64)
__device__ __forceinline__ double2 ring_rot(const FftView &fv, int y, int m)
{
    const double2 *r = fv.rot + (int64_t)y * fv.nrot;
    return cmul(r[m & 63], r[64 + (m >> 6)]);
}

// a e^{i m phi0} (conj: a e^{-i m phi0}); no table loads where every ring starts at phi = 0
__device__ __forceinline__ double2 rotate(const FftView &fv, double2 a, int y, int m)
{
    return fv.rot_trivial ? a : cmul(a, ring_rot(fv, y, m));
}
__device__ __forceinline__ double2 rotate_conj(const FftView &fv, double2 a, int y, int m)
{
    return fv.rot_trivial ? a : cmul(a, cconj(ring_rot(fv, y, m)));
}

// Folded Hermitian spectrum bin k of ring y for component row `row`:
// b_k = sum over m = k mod N, |m| <= mv, of F_m e^{i m phi0} (conjugated for m < 0).
__device__ __forceinline__ double2 fold_bin(const FftView &fv, const double2 *Frow, int y, int N, int mv, int k)
{
    double2 s = make_double2(0.0, 0.0);
    for (int m = k; m <= mv; m += N) s = cadd(s, rotate(fv, Frow[m], y, m));
    for (int m = N - k; m <= mv; m += N) {
        if (m == 0) continue;
        s = cadd(s, cconj(rotate(fv, Frow[m], y, m)));
    }
    return s;
}

// fold_bin for N > 2 mv, where bin k holds at most one term (m = k, or
// m = N - k conjugated): no loops, so that the loads of several bins can be
// issued together.
__device__ __forceinline__ double2 fold_bin_single(const FftView &fv, const double2 *Frow, int y, int N, int mv,
                                                   int k)
{
    const bool refl = k > mv;
    const int m = refl ? N - k : k;
    const bool ok = m <= mv;
    const int mc = ok ? m : 0;
    const double2 t = rotate(fv, Frow[mc], y, mc);
    const double2 z = refl ? cconj(t) : t;
    return ok ? z : make_double2(0.0, 0.0);
}

// Rader's algorithm for a prime length L with smooth L-1: with a generator g
// of the multiplicative group mod L, a_p = x_{g^p} and b_q = w^{g^{-q}}
// (w = e^{-+2 pi i / L}), X_{g^{-q}} = x_0 + (a (*) b)_q, a cyclic convolution of
// length L-1 done with two in-LDS transforms.  buf holds a_p at p < L-1 and x_0
// at L-1 on entry (the input is stored there directly, no reordering pass); on
// return buf[q] holds (a (*) b)_q, and x0 = x_0, X0 = X_0 = sum x_n.
struct RaderEnds {
    double2 x0, X0;
};

template <bool POW2>
__device__ __forceinline__ RaderEnds rader(double2 *buf, const FftView &fv, const FftLen &d, bool fwd)
{
    const FftInner &in = fv.inner[d.inner];
    const int Lm = d.L - 1;
    const double2 *bh = fv.ctab + (fwd ? d.bhat_m : d.bhat_p);
    const double2 x0 = buf[padi<POW2>(Lm)];
    fft_dif<POW2, POW2>(buf, in, true, fv.ctab);
    const double2 A0 = buf[padi<POW2>(0)];        // DC of the reordered input: sum_{n>0} x_n
    __syncthreads();
    batched_loop<true, LOOP_U>(Lm, [&](int p) { return cmul(buf[padi<POW2>(p)], bh[p]); },
                       [&](int p, double2 v) { buf[padi<POW2>(p)] = v; });
    __syncthreads();
    fft_dit<POW2, POW2>(buf, in, false, fv.ctab);
    return RaderEnds{x0, cadd(x0, A0)};
}

// Spectrum bin k (k < L) of a length-L transform finished in LDS by the mode.
template <int MODE, bool PAD>
struct SpecRead {
    const double2 *buf;
    const int *pos;      // LDS mode, direct kind: digit-reversed position; else null
    const int *qpos;     // Rader
    double2 x0, X0;
    __device__ __forceinline__ double2 operator()(int k) const
    {
        if constexpr (MODE == KMODE_RADER) {
            const double2 v = cadd(x0, buf[padi<PAD>(qpos[k])]);   // qpos[0] exists (unused)
            return k == 0 ? X0 : v;
        } else {
            return buf[padi<PAD>(pos ? pos[k] : k)];
        }
    }
};

// Runs the length-L transform of the row in LDS.  load(n), n < L, gives the
// input (read UI elements per thread at a time).  Returns the reader of the result in natural frequency order.
template <int MODE, bool POW2, int UI = LOOP_U, typename Load>
__device__ __forceinline__ SpecRead<MODE, lds_pad<MODE, POW2>()> ring_transform(double2 *buf, const FftView &fv,
                                                         const FftLen &d, bool fwd, Load load)
{
    const FftInner &in = fv.inner[d.inner];
    const int L = d.L;
    SpecRead<MODE, lds_pad<MODE, POW2>()> r{buf, nullptr, nullptr, make_double2(0.0, 0.0), make_double2(0.0, 0.0)};
    if constexpr (MODE == KMODE_SPLIT) {
        bluestein_split<FFT_NREG, POW2>(buf, fv, d, fwd, load);
    } else if constexpr (MODE == KMODE_RADER) {
        const int *rp = fv.itab + d.rpos;   // x_n goes straight to its place in Rader's order
        batched_loop<false, UI>(L, load, [&](int n, double2 v) { buf[padi<POW2>(rp[n])] = v; });
        __syncthreads();
        const RaderEnds e = rader<POW2>(buf, fv, d, fwd);
        r.x0 = e.x0;
        r.X0 = e.X0;
        r.qpos = fv.itab + d.qpos;
    } else {
        const bool direct = d.kind == FFT_DIRECT;
        if (direct && !fwd) {
            // inverse: spectrum in at digit-reversed positions, signal out natural
            const int *pos = fv.itab + in.pos;
            batched_loop<false, UI>(L, load, [&](int n, double2 v) { buf[PADI(pos[n])] = v; });
            __syncthreads();
            fft_dit<POW2>(buf, in, false, fv.ctab);
        } else {
            batched_loop<false, UI>(L, load, [&](int n, double2 v) { buf[PADI(n)] = v; });
            __syncthreads();
            if (direct) {
                fft_dif<POW2>(buf, in, true, fv.ctab);
                r.pos = fv.itab + in.pos;
            } else {
                bluestein<POW2>(buf, fv, d, fwd);
            }
        }
    }
    return r;
}

template <int MODE, bool POW2>
__global__ __launch_bounds__(1024) void k_ring_synth(FftView fv, const int *__restrict__ rowlist,
                                                    const double *__restrict__ phase,
                                                    double *__restrict__ map, int use_weights)
{
    extern __shared__ double2 buf[];
    const FftRow row = fv.rows[rowlist[blockIdx.x]];
    const int tc = blockIdx.y;   // transform * ncomp + component
    const FftLen d = fv.lens[row.len];
    const int N = row.nphi;
    const int64_t rowF = (int64_t)tc * fv.nrings;
    const double2 *Fa = reinterpret_cast<const double2 *>(phase) + (rowF + row.ya) * (fv.mmax + 1);
    // adjoint of analysis: each ring times its weight
    const double wa = use_weights ? fv.weight[row.ya] : 1.0;
    const double wb = (use_weights && row.yb >= 0) ? fv.weight[row.yb] : 1.0;
    const int mva = min(fv.mvalid[row.ya], fv.mmax);
    double *mp = map + (int64_t)tc * fv.npix;

    if (row.mode == ROW_PAIR) {
        const double2 *Fb = nullptr;
        int mvb = -1;
        if (row.yb >= 0) {
            Fb = reinterpret_cast<const double2 *>(phase) + (rowF + row.yb) * (fv.mmax + 1);
            mvb = min(fv.mvalid[row.yb], fv.mmax);
        }
        auto zin = [&](int k) {
            double2 A = fold_bin(fv, Fa, row.ya, N, mva, k);
            double2 B = make_double2(0.0, 0.0);
            if (Fb) B = fold_bin(fv, Fb, row.yb, N, mvb, k);
            return make_double2(A.x - B.y, A.y + B.x);   // A + iB
        };
        // no aliasing: one term per bin; a missing second ring reads ring a's
        // row with mv = -1 (no term)
        const double2 *Fbs = Fb ? Fb : Fa;
        const int ybs = Fb ? row.yb : row.ya;
        auto zin1 = [&](int k) {
            const double2 A = fold_bin_single(fv, Fa, row.ya, N, mva, k);
            const double2 B = fold_bin_single(fv, Fbs, ybs, N, mvb, k);
            return make_double2(A.x - B.y, A.y + B.x);
        };
        SpecRead<MODE, lds_pad<MODE, POW2>()> out;
        if (N > 2 * max(mva, mvb)) out = ring_transform<MODE, POW2>(buf, fv, d, false, zin1);
        else out = ring_transform<MODE, POW2>(buf, fv, d, false, zin);
        const int64_t oa = fv.ofs[row.ya], ob = row.yb >= 0 ? fv.ofs[row.yb] : oa;
        const bool hasb = row.yb >= 0;
        batched_loop<false, LOOP_U>(N, out, [&](int x, double2 z) {
            mp[oa + (int64_t)x * fv.stride] = wa * z.x;
            if (hasb) mp[ob + (int64_t)x * fv.stride] = wb * z.y;
        });
    } else {
        // even N = 2h: Z_k = X_k (1 + i w^k) + conj(X_{h-k}) (1 - i w^k), w = e^{2 pi i/N}
        const int h = N / 2;
        const double2 *htw = fv.ctab + row.half_tw;   // e^{-2 pi i k/N}
        auto pack = [&](double2 X, double2 Y, int k) {
            double2 w = cconj(htw[k]);
            double2 iw = make_double2(-w.y, w.x);
            return cadd(cadd(X, cmul(X, iw)), csub(Y, cmul(Y, iw)));
        };
        auto zin = [&](int k) {
            return pack(fold_bin(fv, Fa, row.ya, N, mva, k), cconj(fold_bin(fv, Fa, row.ya, N, mva, h - k)), k);
        };
        auto zin1 = [&](int k) {
            return pack(fold_bin_single(fv, Fa, row.ya, N, mva, k),
                        cconj(fold_bin_single(fv, Fa, row.ya, N, mva, h - k)), k);
        };
        SpecRead<MODE, lds_pad<MODE, POW2>()> out;
        if (N > 2 * mva) out = ring_transform<MODE, POW2>(buf, fv, d, false, zin1);
        else out = ring_transform<MODE, POW2>(buf, fv, d, false, zin);
        const int64_t oa = fv.ofs[row.ya];
        batched_loop<false, LOOP_U>(h, out, [&](int n, double2 z) {
            mp[oa + (int64_t)(2 * n) * fv.stride] = wa * z.x;
            mp[oa + (int64_t)(2 * n + 1) * fv.stride] = wa * z.y;
        });
    }
}

template <int MODE, bool POW2>
__global__ __launch_bounds__(1024) void k_ring_anal(FftView fv, const int *__restrict__ rowlist,
                                                   const double *__restrict__ map,
                                                   double *__restrict__ phase, int use_weights)
{
    extern __shared__ double2 buf[];
    const FftRow row = fv.rows[rowlist[blockIdx.x]];
    const int tc = blockIdx.y;
    const FftLen d = fv.lens[row.len];
    const int N = row.nphi;
    const int64_t rowF = (int64_t)tc * fv.nrings;
    const double *mp = map + (int64_t)tc * fv.npix;

    if (row.mode == ROW_PAIR) {
        // row pointers hoisted out of the element loop; ring b absent: ring a
        // is read a second time and replaced by zero (a select, no branch)
        const double *pa = mp + fv.ofs[row.ya];
        const bool hb = row.yb >= 0;
        const double *pb = mp + fv.ofs[hb ? row.yb : row.ya];
        const int64_t st = fv.stride;
        auto xin = [&](int x) {
            const double b = pb[(int64_t)x * st];
            return make_double2(pa[(int64_t)x * st], hb ? b : 0.0);
        };
        const auto rd = ring_transform<MODE, POW2, LOOP_U_ANAL>(buf, fv, d, true, xin);
        // ring a: (Zk + conj Z_(N-k)) / 2, ring b: (Zk - conj Z_(N-k)) / (2i), both
        // from one read of the two bins
        const bool hasb = row.yb >= 0;
        const int yb = hasb ? row.yb : row.ya;
        const int mva = min(fv.mvalid[row.ya], fv.mmax), mvb = hasb ? min(fv.mvalid[yb], fv.mmax) : -1;
        const double wa = use_weights ? fv.weight[row.ya] : 1.0, wb = use_weights ? fv.weight[yb] : 1.0;
        double2 *Ga = reinterpret_cast<double2 *>(phase) + (rowF + row.ya) * (fv.mmax + 1);
        double2 *Gb = reinterpret_cast<double2 *>(phase) + (rowF + yb) * (fv.mmax + 1);
        struct GPair {
            double2 a, b;
        };
        batched_loop<false, LOOP_U_ANAL>(max(mva, mvb) + 1, [&](int m) {
            // bins of m and -m; a division only for aliased terms (m >= N)
            const int k = m < N ? m : m % N;
            const int kc = k == 0 ? 0 : N - k;
            const double2 Zk = rd(k), Zc = cconj(rd(kc));
            const double2 dd = csub(Zk, Zc);
            const double2 Sa = make_double2(0.5 * (Zk.x + Zc.x), 0.5 * (Zk.y + Zc.y));
            const double2 Sb = make_double2(0.5 * dd.y, -0.5 * dd.x);
            const double2 ga = rotate_conj(fv, Sa, row.ya, m), gb = rotate_conj(fv, Sb, yb, m);
            return GPair{make_double2(wa * ga.x, wa * ga.y), make_double2(wb * gb.x, wb * gb.y)};
        }, [&](int m, GPair g) {
            if (m <= mva) Ga[m] = g.a;
            if (m <= mvb) Gb[m] = g.b;
        });
    } else {
        const int h = N / 2;
        const double *pa = mp + fv.ofs[row.ya];
        const int64_t st = fv.stride;
        auto xin = [&](int n) { return make_double2(pa[(int64_t)(2 * n) * st], pa[(int64_t)(2 * n + 1) * st]); };
        const auto rd = ring_transform<MODE, POW2, LOOP_U_ANAL>(buf, fv, d, true, xin);
        const double2 *htw = fv.ctab + row.half_tw;   // e^{-2 pi i k/N}, k < h
        const int y = row.ya;
        const int mv = min(fv.mvalid[y], fv.mmax);
        const double w = use_weights ? fv.weight[y] : 1.0;
        double2 *G = reinterpret_cast<double2 *>(phase) + (rowF + y) * (fv.mmax + 1);
        batched_loop<false, LOOP_U_ANAL>(mv + 1, [&](int m) {
            int k = m < N ? m : m % N;
            const bool cj = k > h;                   // X_{N-k} = conj X_k
            if (cj) k = N - k;
            // X_k = E_k + e^{-2 pi i k/N} O_k, E/O from Z_k and conj Z_{h-k} (indices mod h)
            const int k1 = k == h ? 0 : k, k2 = k1 == 0 ? 0 : h - k1;
            const double2 Zk = rd(k1), Zc = cconj(rd(k2));
            const double2 E = make_double2(0.5 * (Zk.x + Zc.x), 0.5 * (Zk.y + Zc.y));
            const double2 dd = csub(Zk, Zc);
            const double2 O = make_double2(0.5 * dd.y, -0.5 * dd.x);
            const double2 t = htw[k < h ? k : 0];
            const double2 tw = k < h ? t : make_double2(-1.0, 0.0);   // k == h: e^{-i pi}
            double2 X = cadd(E, cmul(tw, O));
            if (cj) X = cconj(X);
            const double2 g = rotate_conj(fv, X, y, m);
            return make_double2(w * g.x, w * g.y);
        }, [&](int m, double2 g) { G[m] = g; });
    }
}

// Bluestein kernel spectra: Bhat = FFT_M(b) / M, b_j = conj(w_j) for |j| < L
// (w for the given sign), stored in the inner transform's digit-reversed order.
template <bool POW2>
__global__ __launch_bounds__(512) void k_blue_prep(FftView fv, int len_id, int fwd_sign,
                                                   double2 *out)
{
    extern __shared__ double2 buf[];
    const FftLen d = fv.lens[len_id];
    const FftInner &in = fv.inner[d.inner];
    const double2 *chirp = fv.ctab + d.chirp;
    const int L = d.L, M = d.M;
    // b_j for sign s: conj(w_j) with w_j = e^{s i pi j^2/L}; table holds s = +
    auto bval = [&](int j) -> double2 {
        int jj = j;
        if (jj >= M - L + 1 && jj > 0) jj = M - jj;
        else if (jj >= L) return make_double2(0.0, 0.0);
        double2 c = chirp[jj];
        return fwd_sign ? c : cconj(c);   // s = -: conj(conj(c)) = c
    };
    const double invM = 1.0 / (double)M;
    if (d.kind == FFT_BLUE) {
        for (int j = threadIdx.x; j < M; j += blockDim.x) buf[PADI(j)] = bval(j);
        __syncthreads();
        fft_dif<POW2>(buf, in, true, fv.ctab);
        for (int p = threadIdx.x; p < M; p += blockDim.x)
            out[p] = make_double2(buf[PADI(p)].x * invM, buf[PADI(p)].y * invM);
    } else {
        const int Mh = M / 2;
        const double2 *wm = fv.ctab + d.wm;
        for (int half = 0; half < 2; ++half) {
            for (int j = threadIdx.x; j < Mh; j += blockDim.x) {
                double2 a = bval(j), b = bval(j + Mh);
                buf[PADI(j)] = half ? cmul(csub(a, b), wm[j]) : cadd(a, b);
            }
            __syncthreads();
            fft_dif<POW2>(buf, in, true, fv.ctab);
            for (int p = threadIdx.x; p < Mh; p += blockDim.x)
                out[half * Mh + p] = make_double2(buf[PADI(p)].x * invM, buf[PADI(p)].y * invM);
            __syncthreads();
        }
    }
}

// Rader kernel spectra: Bhat = FFT_{L-1}(b) / (L-1) with b_q = w^{g^{-q}},
// w = e^{+2 pi i / L} (minus = 0) or its conjugate, in the inner transform's
// digit-reversed order.
template <bool POW2>
__global__ __launch_bounds__(512) void k_rader_prep(FftView fv, int len_id, int minus, double2 *out)
{
    extern __shared__ double2 buf[];
    const FftLen d = fv.lens[len_id];
    const FftInner &in = fv.inner[d.inner];
    const double2 *bq = fv.ctab + d.chirp;
    const int Lm = d.L - 1;
    for (int q = threadIdx.x; q < Lm; q += blockDim.x) buf[PADI(q)] = minus ? cconj(bq[q]) : bq[q];
    __syncthreads();
    fft_dif<POW2>(buf, in, true, fv.ctab);
    const double inv = 1.0 / (double)Lm;
    for (int p = threadIdx.x; p < Lm; p += blockDim.x)
        out[p] = make_double2(buf[PADI(p)].x * inv, buf[PADI(p)].y * inv);
}

// ------------------------------------------------------------------ host

static bool factor_smooth(int n, std::vector<int> &rad)
{
    rad.clear();
    int m = n;
    while (m % 8 == 0 && m > 8) { rad.push_back(8); m /= 8; }
    while (m % 4 == 0) { rad.push_back(4); m /= 4; }
    while (m % 2 == 0) { rad.push_back(2); m /= 2; }
    const int odd[] = {3, 5, 7, 11, 13};
    for (int r : odd)
        while (m % r == 0) { rad.push_back(r); m /= r; }
    if (m == 8) rad.push_back(8), m = 1;
    return m == 1 && (int)rad.size() <= FFT_MAXRAD;
}

// Pass plan of an inner transform: which consecutive passes run fused in
// registers (fft_pass2), and in which order.  Fused pairs (larger radix first)
// keep at most 14 complex values per thread (with 15 or 16 the 1024-thread
// kernels spill registers).  The grouping minimises the
// butterfly rounds a work group of the given size executes, plus one per LDS
// sweep (each sweep ends in a barrier).  Smaller groups go first: late DIF
// passes use few distinct twiddles, so the large radices are cheapest there.
static bool fusable(int r1, int r2)
{
    static const int ok[][2] = {{2, 2}, {4, 2}, {3, 2}, {3, 3}, {5, 2}, {7, 2}};
    for (const auto &q : ok)
        if (q[0] == r1 && q[1] == r2) return true;
    return false;
}

static int inner_threads(int n)
{
    int c = 1;
    while (c < n) c *= 2;
    return c >= 8192 ? 1024 : (c >= 2048 ? 512 : 256);
}

static void best_grouping(int n, int threads, std::vector<int> rest, std::vector<std::vector<int>> &cur,
                          double &best_cost, std::vector<std::vector<int>> &best)
{
    if (rest.empty()) {
        double cost = 0.0;
        for (const auto &g : cur) {
            int prod = 1;
            for (int r : g) prod *= r;
            const int nb = n / prod;
            cost += (double)((nb + threads - 1) / threads) + 1.0;
        }
        if (cost < best_cost) { best_cost = cost; best = cur; }
        return;
    }
    const int f = rest[0];
    std::vector<int> tail(rest.begin() + 1, rest.end());
    cur.push_back({f});
    best_grouping(n, threads, tail, cur, best_cost, best);
    cur.pop_back();
    for (size_t i = 0; i < tail.size(); ++i) {
        if (i > 0 && tail[i] == tail[i - 1]) continue;
        const int a = std::max(f, tail[i]), b = std::min(f, tail[i]);
        if (!fusable(a, b)) continue;
        std::vector<int> t2 = tail;
        t2.erase(t2.begin() + (long)i);
        cur.push_back({a, b});
        best_grouping(n, threads, t2, cur, best_cost, best);
        cur.pop_back();
    }
}

static void plan_passes(int n, std::vector<int> &rad, std::vector<int> &fuse)
{
    std::vector<int> f = rad;
    std::sort(f.begin(), f.end());
    std::vector<std::vector<int>> cur, best;
    double cost = 1e30;
    best_grouping(n, inner_threads(n), f, cur, cost, best);
    std::stable_sort(best.begin(), best.end(), [](const std::vector<int> &x, const std::vector<int> &y) {
        int px = 1, py = 1;
        for (int r : x) px *= r;
        for (int r : y) py *= r;
        return px < py;
    });
    rad.clear();
    fuse.clear();
    for (const auto &g : best) {
        for (size_t i = 0; i < g.size(); ++i) {
            rad.push_back(g[i]);
            fuse.push_back(g.size() == 2 && i == 0 ? 1 : 0);
        }
    }
}

static bool is_prime(int n)
{
    if (n < 2) return false;
    for (int d = 2; (int64_t)d * d <= n; ++d)
        if (n % d == 0) return false;
    return true;
}

static int64_t powmod(int64_t b, int64_t e, int64_t m)
{
    int64_t r = 1;
    b %= m;
    while (e) {
        if (e & 1) r = r * b % m;
        b = b * b % m;
        e >>= 1;
    }
    return r;
}

// smallest generator of the multiplicative group modulo the prime p
static int primitive_root(int p)
{
    std::vector<int> fac;
    int m = p - 1;
    for (int d = 2; d * d <= m; ++d)
        if (m % d == 0) {
            fac.push_back(d);
            while (m % d == 0) m /= d;
        }
    if (m > 1) fac.push_back(m);
    for (int g = 2; g < p; ++g) {
        bool ok = true;
        for (int q : fac)
            if (powmod(g, (p - 1) / q, p) == 1) { ok = false; break; }
        if (ok) return g;
    }
    return 1;   // p = 2
}

struct FftHost {
    std::vector<double2> ctab;
    std::vector<int> itab;
    std::vector<FftInner> inner;
    std::vector<FftLen> lens;
    std::vector<FftRow> rows;
    std::map<int, int> inner_of_n, len_of_L, halftw_of_N;
};

static const long double kPi = 3.14159265358979323846264338327950288L;

static int add_inner(FftHost &H, int n)
{
    auto it = H.inner_of_n.find(n);
    if (it != H.inner_of_n.end()) return it->second;
    FftInner in{};
    in.n = n;
    std::vector<int> rad, fuse;
    factor_smooth(n, rad);
    plan_passes(n, rad, fuse);
    in.nrad = (int)rad.size();
    for (int i = 0; i < in.nrad; ++i) {
        in.rad[i] = rad[i];
        in.fuse[i] = fuse[i];
    }
    in.tw = (int64_t)H.ctab.size();
    for (int j = 0; j < n; ++j) {
        long double a = -2.0L * kPi * (long double)j / (long double)n;
        H.ctab.push_back(make_double2((double)cosl(a), (double)sinl(a)));
    }
    // digit-reversed position of each frequency for the DIF pass sequence:
    // position p = sum_i k_i L_{i+1}, frequency f = k_0 + r_0 (k_1 + r_1 (...))
    in.pos = (int64_t)H.itab.size();
    H.itab.resize(H.itab.size() + n);
    for (int f = 0; f < n; ++f) {
        int rem = f, p = 0, Lb = n;
        for (int i = 0; i < in.nrad; ++i) {
            const int r = in.rad[i];
            const int k = rem % r;
            rem /= r;
            Lb /= r;
            p += k * Lb;
        }
        H.itab[in.pos + f] = p;
    }
    int id = (int)H.inner.size();
    H.inner.push_back(in);
    H.inner_of_n[n] = id;
    return id;
}

static int lds_limit_complex()
{
    int dev = 0;
    (void)hipGetDevice(&dev);
    int bytes = 0;
    if (hipDeviceGetAttribute(&bytes, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
        (void)hipGetLastError();
        bytes = 65536;
    }
    int c = 1;
    while (lds_padded(c * 2) * 16 <= bytes) c *= 2;
    return c;
}

static int add_len(FftHost &H, int L, int cmax, int &err)
{
    auto it = H.len_of_L.find(L);
    if (it != H.len_of_L.end()) return it->second;
    FftLen d{};
    d.L = L;
    std::vector<int> rad;
    if (factor_smooth(L, rad) && L <= cmax) {
        d.kind = FFT_DIRECT;
        d.M = L;
        d.inner = add_inner(H, L);
        d.lds_complex = L;
    } else if (L > 2 && L <= cmax && L - 1 <= FFT_NREG * 1024 && is_prime(L) &&
               factor_smooth(L - 1, rad)) {
        d.kind = FFT_RADER;
        d.M = L - 1;
        d.inner = add_inner(H, L - 1);
        d.lds_complex = L;       // the reordered input and x_0
        const int g = primitive_root(L);
        const int ginv = (int)powmod(g, L - 2, L);
        d.rpos = (int64_t)H.itab.size();
        H.itab.resize(H.itab.size() + L, 0);
        H.itab[d.rpos] = L - 1;   // x_0 after the L - 1 reordered values
        for (int64_t p = 0, v = 1; p < L - 1; ++p, v = v * g % L) H.itab[d.rpos + v] = (int)p;   // g^p = v
        d.qpos = (int64_t)H.itab.size();
        H.itab.resize(H.itab.size() + L, 0);
        d.chirp = (int64_t)H.ctab.size();
        for (int64_t q = 0, v = 1; q < L - 1; ++q, v = v * ginv % L) {
            H.itab[d.qpos + v] = (int)q;           // g^{-q} = v
            const long double a = 2.0L * kPi * (long double)v / (long double)L;
            H.ctab.push_back(make_double2((double)cosl(a), (double)sinl(a)));
        }
        d.bhat_p = (int64_t)H.ctab.size();
        H.ctab.resize(H.ctab.size() + (L - 1));
        d.bhat_m = (int64_t)H.ctab.size();
        H.ctab.resize(H.ctab.size() + (L - 1));
    } else {
        int M = 1;
        while (M < 2 * L - 1) M *= 2;
        d.M = M;
        if (M <= cmax) {
            d.kind = FFT_BLUE;
            d.inner = add_inner(H, M);
            d.lds_complex = M;
        } else if (M / 2 <= cmax) {
            d.kind = FFT_BLUE_SPLIT;
            d.inner = add_inner(H, M / 2);
            d.lds_complex = M / 2;
            d.wm = (int64_t)H.ctab.size();
            for (int n = 0; n < M / 2; ++n) {
                long double a = -2.0L * kPi * (long double)n / (long double)M;
                H.ctab.push_back(make_double2((double)cosl(a), (double)sinl(a)));
            }
        } else {
            err = 1;
            return -1;
        }
        d.chirp = (int64_t)H.ctab.size();
        for (int n = 0; n < L; ++n) {
            // e^{+i pi n^2 / L} with n^2 reduced mod 2L
            long long q = ((long long)n * n) % (2LL * L);
            long double a = kPi * (long double)q / (long double)L;
            H.ctab.push_back(make_double2((double)cosl(a), (double)sinl(a)));
        }
        d.bhat_p = (int64_t)H.ctab.size();
        H.ctab.resize(H.ctab.size() + M);
        d.bhat_m = (int64_t)H.ctab.size();
        H.ctab.resize(H.ctab.size() + M);
    }
    int id = (int)H.lens.size();
    H.lens.push_back(d);
    H.len_of_L[L] = id;
    return id;
}

static int64_t add_half_tw(FftHost &H, int N)
{
    auto it = H.halftw_of_N.find(N);
    if (it != H.halftw_of_N.end()) return it->second;
    int64_t o = (int64_t)H.ctab.size();
    for (int k = 0; k < N / 2; ++k) {
        long double a = -2.0L * kPi * (long double)k / (long double)N;
        H.ctab.push_back(make_double2((double)cosl(a), (double)sinl(a)));
    }
    H.halftw_of_N[N] = (int)o;
    return o;
}

// launch groups: rows sharing LDS size class, kernel mode and radix class
struct FftGroup {
    int lds_complex;   // power of two >= every row's LDS need
    int mode;          // KMODE_*
    bool pow2;         // inner length a power of two
    std::vector<int> rows;
};

// threads per work group; split and Rader modes need FFT_NREG * threads >= lds_complex
static int threads_for(const FftGroup &gr)
{
    if (gr.lds_complex >= 8192) return 1024;
    if (gr.lds_complex >= 2048) return 512;
    return 256;
}

struct FftDev {
    FftInner *inner = nullptr;
    FftLen *lens = nullptr;
    FftRow *rows = nullptr;
    double2 *ctab = nullptr;
    int *itab = nullptr;
    int64_t *ofs = nullptr;
    double *weight = nullptr;
    double2 *rot = nullptr;
    int *mvalid = nullptr;
    int nrot = 0;
    int rot_trivial = 0;      // every ring has phi0 = 0
    std::vector<FftGroup> groups;
    std::vector<int *> group_rows;
    // plans with several ring-length groups run the groups' launches on
    // concurrent streams (each group alone is too small to fill the GPU):
    // forked from and joined back to the caller's stream with events
    std::vector<hipStream_t> aux;
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> join;
};

constexpr int FFT_MAX_AUX = 3;   // extra streams of a plan's ring FFT step

}  // namespace sht

namespace sht {

static FftView view_of(const Plan &p, const FftDev &D)
{
    FftView v{};
    v.inner = D.inner;
    v.lens = D.lens;
    v.rows = D.rows;
    v.ctab = D.ctab;
    v.itab = D.itab;
    v.ofs = D.ofs;
    v.stride = p.geom.stride;
    v.weight = D.weight;
    v.rot = D.rot;
    v.nrot = D.nrot;
    v.rot_trivial = D.rot_trivial;
    v.mvalid = D.mvalid;
    v.mmax = p.mmax;
    v.nrings = p.geom.nrings;
    v.ncomp = p.ncomp;
    v.npix = p.geom.npix;
    return v;
}

static int mode_of(const FftLen &d)
{
    if (d.kind == FFT_BLUE_SPLIT) return KMODE_SPLIT;
    if (d.kind == FFT_RADER) return KMODE_RADER;
    return KMODE_LDS;
}

static int prepare_groups(const FftDev &D);

int fft_plan_build(Plan &p)
{
    const Geom &g = p.geom;
    FftHost H;
    const int cmax = lds_limit_complex();
    int err = 0;
    // rows: even nphi -> half rows; odd nphi -> pairs of mirror rings of equal length
    std::vector<int> done(g.nrings, 0);
    for (const SlotHost &s : p.slots) {
        const int ya = s.yn, yb = s.ys;
        if (ya >= 0 && yb >= 0 && g.nphi[ya] == g.nphi[yb] && (g.nphi[ya] & 1)) {
            FftRow r{};
            r.mode = ROW_PAIR;
            r.ya = ya;
            r.yb = yb;
            r.nphi = (int)g.nphi[ya];
            r.len = add_len(H, r.nphi, cmax, err);
            H.rows.push_back(r);
            done[ya] = done[yb] = 1;
        }
    }
    for (int y = 0; y < g.nrings; ++y) {
        if (done[y]) continue;
        FftRow r{};
        r.ya = y;
        r.yb = -1;
        r.nphi = (int)g.nphi[y];
        if (r.nphi % 2 == 0) {
            r.mode = ROW_HALF;
            r.len = add_len(H, r.nphi / 2, cmax, err);
            r.half_tw = add_half_tw(H, r.nphi);
        } else {
            r.mode = ROW_PAIR;
            r.len = add_len(H, r.nphi, cmax, err);
        }
        H.rows.push_back(r);
    }
    if (err) {
        set_error("ring length too large for the LDS FFT (max complex length %d)", cmax);
        return SHT_EUNSUPPORTED;
    }
    // per-ring tables
    std::vector<int> slot_of_ring(g.nrings, -1);
    for (int i = 0; i < p.nslots; ++i) {
        if (p.slots[i].yn >= 0) slot_of_ring[p.slots[i].yn] = i;
        if (p.slots[i].ys >= 0) slot_of_ring[p.slots[i].ys] = i;
    }
    std::vector<int> mvalid(g.nrings, -1);
    for (int y = 0; y < g.nrings; ++y) {
        int sl = slot_of_ring[y];
        mvalid[y] = (sl >= 0) ? p.tile_mlim[sl / p.slots_per_tile] : -1;
    }
    const int ncoarse = p.mmax / 64 + 1;
    const int nrot = 64 + ncoarse;
    std::vector<double2> rot((size_t)g.nrings * nrot);
    for (int y = 0; y < g.nrings; ++y) {
        const long double ph = g.phi0[y];
        for (int j = 0; j < 64; ++j)
            rot[(size_t)y * nrot + j] = make_double2((double)cosl(j * ph), (double)sinl(j * ph));
        for (int j = 0; j < ncoarse; ++j)
            rot[(size_t)y * nrot + 64 + j] =
                make_double2((double)cosl(64.0L * j * ph), (double)sinl(64.0L * j * ph));
    }
    // groups by LDS class
    std::map<std::tuple<int, int, int>, int> gid;
    FftDev *D = new FftDev();
    for (int i = 0; i < (int)H.rows.size(); ++i) {
        const FftLen &d = H.lens[H.rows[i].len];
        int c = 256;
        while (c < d.lds_complex) c *= 2;
        const int mode = mode_of(d);
        const int n_in = H.inner[d.inner].n;
        const bool pow2 = (n_in & (n_in - 1)) == 0;
        auto key = std::make_tuple(c, mode, (int)pow2);
        auto it = gid.find(key);
        if (it == gid.end()) {
            gid[key] = (int)D->groups.size();
            D->groups.push_back(FftGroup{c, mode, pow2, {}});
            it = gid.find(key);
        }
        D->groups[it->second].rows.push_back(i);
    }
    for (auto &gr : D->groups)
        if (gr.mode != KMODE_LDS && FFT_NREG * threads_for(gr) < gr.lds_complex) {
            set_error("FFT of %d complex points exceeds the register slots of its work group",
                      gr.lds_complex);
            delete D;
            return SHT_EUNSUPPORTED;
        }
    int rc;
    auto up = [&](void **dst, const void *src, size_t bytes, const char *what) -> int {
        int r = dev_alloc(dst, bytes ? bytes : 16, what);
        if (r) return r;
        return bytes ? dev_upload(*dst, src, bytes, what) : SHT_OK;
    };
    if ((rc = up((void **)&D->inner, H.inner.data(), H.inner.size() * sizeof(FftInner), "fft tables")) ||
        (rc = up((void **)&D->lens, H.lens.data(), H.lens.size() * sizeof(FftLen), "fft tables")) ||
        (rc = up((void **)&D->rows, H.rows.data(), H.rows.size() * sizeof(FftRow), "fft tables")) ||
        (rc = up((void **)&D->ctab, H.ctab.data(), H.ctab.size() * sizeof(double2), "fft tables")) ||
        (rc = up((void **)&D->itab, H.itab.data(), H.itab.size() * sizeof(int), "fft tables")) ||
        (rc = up((void **)&D->ofs, g.ofs.data(), g.ofs.size() * sizeof(int64_t), "fft tables")) ||
        (rc = up((void **)&D->weight, g.weight.data(), g.weight.size() * sizeof(double), "fft tables")) ||
        (rc = up((void **)&D->rot, rot.data(), rot.size() * sizeof(double2), "fft tables")) ||
        (rc = up((void **)&D->mvalid, mvalid.data(), mvalid.size() * sizeof(int), "fft tables"))) {
        p.fft.d_rows = D;
        return rc;
    }
    D->nrot = nrot;
    D->rot_trivial = std::all_of(g.phi0.begin(), g.phi0.end(), [](double x) { return x == 0.0; }) ? 1 : 0;
    for (auto &gr : D->groups) {
        int *dr = nullptr;
        if ((rc = up((void **)&dr, gr.rows.data(), gr.rows.size() * sizeof(int), "fft rows"))) {
            p.fft.d_rows = D;
            return rc;
        }
        D->group_rows.push_back(dr);
    }
    p.fft.d_rows = D;
    p.fft.nrows = (int)H.rows.size();
    p.fft.table_bytes = H.ctab.size() * sizeof(double2) + H.itab.size() * sizeof(int);
    if ((rc = prepare_groups(*D))) return rc;
    if (D->groups.size() > 1) {
        const int naux = (int)std::min<size_t>(D->groups.size() - 1, FFT_MAX_AUX);
        if ((rc = check_hip(hipEventCreateWithFlags(&D->fork, hipEventDisableTiming), "fft events"))) return rc;
        for (int i = 0; i < naux; ++i) {
            hipStream_t st = nullptr;
            hipEvent_t e = nullptr;
            if ((rc = check_hip(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "fft streams"))) return rc;
            D->aux.push_back(st);
            if ((rc = check_hip(hipEventCreateWithFlags(&e, hipEventDisableTiming), "fft events"))) return rc;
            D->join.push_back(e);
        }
    }
    // Bluestein kernel spectra on the device
    FftView v = view_of(p, *D);
    for (int li = 0; li < (int)H.lens.size(); ++li) {
        const FftLen &d = H.lens[li];
        if (d.kind == FFT_DIRECT) continue;
        if (d.kind == FFT_RADER) {
            const int n_in = H.inner[d.inner].n;
            const bool pow2 = (n_in & (n_in - 1)) == 0;
            const void *fn = pow2 ? (const void *)k_rader_prep<true> : (const void *)k_rader_prep<false>;
            const size_t lds = (size_t)lds_padded(d.lds_complex) * sizeof(double2);
            if (lds > 65536)
                if ((rc = check_hip(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                        (int)lds),
                                    "fft LDS attribute")))
                    return rc;
            if (pow2) {
                hipLaunchKernelGGL(k_rader_prep<true>, dim3(1), dim3(512), lds, 0, v, li, 0, D->ctab + d.bhat_p);
                hipLaunchKernelGGL(k_rader_prep<true>, dim3(1), dim3(512), lds, 0, v, li, 1, D->ctab + d.bhat_m);
            } else {
                hipLaunchKernelGGL(k_rader_prep<false>, dim3(1), dim3(512), lds, 0, v, li, 0, D->ctab + d.bhat_p);
                hipLaunchKernelGGL(k_rader_prep<false>, dim3(1), dim3(512), lds, 0, v, li, 1, D->ctab + d.bhat_m);
            }
            continue;
        }
        // the inner length of a Bluestein transform is a power of two
        const size_t lds = (size_t)lds_padded(d.lds_complex) * sizeof(double2);
        if (lds > 65536)
            if ((rc = check_hip(hipFuncSetAttribute((const void *)k_blue_prep<true>,
                                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds),
                                "fft LDS attribute")))
                return rc;
        hipLaunchKernelGGL(k_blue_prep<true>, dim3(1), dim3(512), lds, 0, v, li, 0, D->ctab + d.bhat_p);
        hipLaunchKernelGGL(k_blue_prep<true>, dim3(1), dim3(512), lds, 0, v, li, 1, D->ctab + d.bhat_m);
    }
    if ((rc = check_hip(hipGetLastError(), "bluestein preparation"))) return rc;
    if ((rc = check_hip(hipDeviceSynchronize(), "bluestein preparation"))) return rc;
    return SHT_OK;
}

void fft_plan_free(FftPlan &f)
{
    FftDev *D = reinterpret_cast<FftDev *>(f.d_rows);
    if (!D) return;
    dev_free(D->inner); dev_free(D->lens); dev_free(D->rows); dev_free(D->ctab);
    dev_free(D->itab); dev_free(D->ofs); dev_free(D->weight); dev_free(D->rot);
    dev_free(D->mvalid);
    for (int *r : D->group_rows) dev_free(r);
    for (hipStream_t st : D->aux) (void)hipStreamDestroy(st);
    for (hipEvent_t e : D->join) (void)hipEventDestroy(e);
    if (D->fork) (void)hipEventDestroy(D->fork);
    delete D;
    f.d_rows = nullptr;
}

// Allows the group's kernels their dynamic LDS size (once, at plan time, so that
// launches stay pure stream work and can be captured in a graph).
template <int MODE, bool POW2>
static int prepare_group(const FftGroup &gr)
{
    const size_t lds = (size_t)lds_padded(gr.lds_complex) * sizeof(double2);
    if (lds <= 65536) return SHT_OK;
    int rc = check_hip(hipFuncSetAttribute((const void *)k_ring_synth<MODE, POW2>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds),
                       "fft LDS attribute");
    if (rc) return rc;
    return check_hip(hipFuncSetAttribute((const void *)k_ring_anal<MODE, POW2>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds),
                     "fft LDS attribute");
}

static int prepare_groups(const FftDev &D)
{
    for (const FftGroup &gr : D.groups) {
        int rc;
        if (gr.mode == KMODE_SPLIT) rc = prepare_group<KMODE_SPLIT, true>(gr);
        else if (gr.mode == KMODE_RADER && gr.pow2) rc = prepare_group<KMODE_RADER, true>(gr);
        else if (gr.mode == KMODE_RADER) rc = prepare_group<KMODE_RADER, false>(gr);
        else if (gr.pow2) rc = prepare_group<KMODE_LDS, true>(gr);
        else rc = prepare_group<KMODE_LDS, false>(gr);
        if (rc) return rc;
    }
    return SHT_OK;
}

template <int MODE, bool POW2>
static int launch_group_synth(const FftView &v, const FftGroup &gr, const int *rows,
                              const double *phase, double *map, int ntc, int usew, hipStream_t s)
{
    const size_t lds = (size_t)lds_padded(gr.lds_complex) * sizeof(double2);
    hipLaunchKernelGGL((k_ring_synth<MODE, POW2>), dim3((unsigned)gr.rows.size(), (unsigned)ntc),
                       dim3(threads_for(gr)), lds, s, v, rows, phase, map, usew);
    return SHT_OK;
}

template <int MODE, bool POW2>
static int launch_group_anal(const FftView &v, const FftGroup &gr, const int *rows, const double *map,
                             double *phase, int ntc, int usew, hipStream_t s)
{
    const size_t lds = (size_t)lds_padded(gr.lds_complex) * sizeof(double2);
    hipLaunchKernelGGL((k_ring_anal<MODE, POW2>), dim3((unsigned)gr.rows.size(), (unsigned)ntc),
                       dim3(threads_for(gr)), lds, s, v, rows, map, phase, usew);
    return SHT_OK;
}

// Whether the groups run on the plan's extra streams: only for plain launches.
// A caller's stream under capture keeps every group (serial launches): a batch
// capture that also forked the groups onto these streams ended in a host-side
// crash inside the runtime, whose cause was not established.
static bool fft_concurrent(const FftDev &D, hipStream_t s)
{
    if (D.aux.empty()) return false;
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return st == hipStreamCaptureStatusNone;
}

// Stream of group i: the caller's stream for the first, the plan's extra
// streams round robin for the others (after fft_fork; conc = fft_concurrent).
static hipStream_t group_stream(const FftDev &D, size_t i, hipStream_t s, bool conc)
{
    if (!conc) return s;
    const size_t n = D.aux.size() + 1;
    return (i % n == 0) ? s : D.aux[i % n - 1];
}

static int fft_fork(const FftDev &D, hipStream_t s, bool conc)
{
    if (!conc) return SHT_OK;
    int rc;
    if ((rc = check_hip(hipEventRecord(D.fork, s), "fft fork"))) return rc;
    for (hipStream_t st : D.aux)
        if ((rc = check_hip(hipStreamWaitEvent(st, D.fork, 0), "fft fork"))) return rc;
    return SHT_OK;
}

static int fft_join(const FftDev &D, hipStream_t s, bool conc)
{
    if (!conc) return SHT_OK;
    int rc;
    for (size_t j = 0; j < D.aux.size(); ++j) {
        if ((rc = check_hip(hipEventRecord(D.join[j], D.aux[j]), "fft join"))) return rc;
        if ((rc = check_hip(hipStreamWaitEvent(s, D.join[j], 0), "fft join"))) return rc;
    }
    return SHT_OK;
}

int launch_ring_synth(const Plan &p, const double *phase, double *map, bool use_weights, hipStream_t s0)
{
    const FftDev *D = reinterpret_cast<const FftDev *>(p.fft.d_rows);
    const FftView v = view_of(p, *D);
    const int ntc = p.ntrans * p.ncomp;
    const int usew = use_weights ? 1 : 0;
    const bool conc = fft_concurrent(*D, s0);
    int rc0;
    if ((rc0 = fft_fork(*D, s0, conc))) return rc0;
    for (size_t i = 0; i < D->groups.size(); ++i) {
        const FftGroup &gr = D->groups[i];
        const int *rows = D->group_rows[i];
        const hipStream_t s = group_stream(*D, i, s0, conc);
        log_msg(3, "launch ring FFT (%s) plan %llu: group %zu, mode %d, %zu rows x %d, LDS %d complex, stream %p",
                "synthesis", (unsigned long long)p.serial, i, gr.mode, gr.rows.size(), ntc, gr.lds_complex, (void *)s);
        int rc;
        // split Bluestein always has a power-of-two inner length
        if (gr.mode == KMODE_SPLIT) rc = launch_group_synth<KMODE_SPLIT, true>(v, gr, rows, phase, map, ntc, usew, s);
        else if (gr.mode == KMODE_RADER && gr.pow2) rc = launch_group_synth<KMODE_RADER, true>(v, gr, rows, phase, map, ntc, usew, s);
        else if (gr.mode == KMODE_RADER) rc = launch_group_synth<KMODE_RADER, false>(v, gr, rows, phase, map, ntc, usew, s);
        else if (gr.pow2) rc = launch_group_synth<KMODE_LDS, true>(v, gr, rows, phase, map, ntc, usew, s);
        else rc = launch_group_synth<KMODE_LDS, false>(v, gr, rows, phase, map, ntc, usew, s);
        if (rc) return rc;
    }
    if ((rc0 = check_hip(hipGetLastError(), "ring synthesis launch"))) return rc0;
    return fft_join(*D, s0, conc);
}

int launch_ring_anal(const Plan &p, const double *map, double *phase, bool use_weights, hipStream_t s0)
{
    const FftDev *D = reinterpret_cast<const FftDev *>(p.fft.d_rows);
    const FftView v = view_of(p, *D);
    const int ntc = p.ntrans * p.ncomp;
    const int uw = use_weights ? 1 : 0;
    const bool conc = fft_concurrent(*D, s0);
    int rc0;
    if ((rc0 = fft_fork(*D, s0, conc))) return rc0;
    for (size_t i = 0; i < D->groups.size(); ++i) {
        const FftGroup &gr = D->groups[i];
        const int *rows = D->group_rows[i];
        const hipStream_t s = group_stream(*D, i, s0, conc);
        log_msg(3, "launch ring FFT (%s) plan %llu: group %zu, mode %d, %zu rows x %d, LDS %d complex, stream %p",
                "analysis", (unsigned long long)p.serial, i, gr.mode, gr.rows.size(), ntc, gr.lds_complex, (void *)s);
        int rc;
        if (gr.mode == KMODE_SPLIT) rc = launch_group_anal<KMODE_SPLIT, true>(v, gr, rows, map, phase, ntc, uw, s);
        else if (gr.mode == KMODE_RADER && gr.pow2) rc = launch_group_anal<KMODE_RADER, true>(v, gr, rows, map, phase, ntc, uw, s);
        else if (gr.mode == KMODE_RADER) rc = launch_group_anal<KMODE_RADER, false>(v, gr, rows, map, phase, ntc, uw, s);
        else if (gr.pow2) rc = launch_group_anal<KMODE_LDS, true>(v, gr, rows, map, phase, ntc, uw, s);
        else rc = launch_group_anal<KMODE_LDS, false>(v, gr, rows, map, phase, ntc, uw, s);
        if (rc) return rc;
    }
    if ((rc0 = check_hip(hipGetLastError(), "ring analysis launch"))) return rc0;
    return fft_join(*D, s0, conc);
}

// Zeroes the phase entries above each ring's last kept m (the terms the polar
// criterion drops; neither step writes them and the full transforms never read
// them), so that the staged steps hand over fully defined phases.
__global__ __launch_bounds__(256) void k_phase_tail_zero(double2 *phase, const int *mvalid, int nrings, int mmax,
                                                         int ntc)
{
    const int y = blockIdx.x;
    const int mv = min(mvalid[y], mmax);
    for (int tc = 0; tc < ntc; ++tc) {
        double2 *row = phase + ((int64_t)tc * nrings + y) * (mmax + 1);
        for (int m = mv + 1 + (int)threadIdx.x; m <= mmax; m += blockDim.x) row[m] = make_double2(0.0, 0.0);
    }
}

int launch_phase_tail_zero(const Plan &p, double *phase, hipStream_t s)
{
    const FftDev *D = reinterpret_cast<const FftDev *>(p.fft.d_rows);
    if (p.geom.nrings == 0) return SHT_OK;
    hipLaunchKernelGGL(k_phase_tail_zero, dim3((unsigned)p.geom.nrings), dim3(256), 0, s,
                       reinterpret_cast<double2 *>(phase), D->mvalid, p.geom.nrings, p.mmax, p.ntrans * p.ncomp);
    return check_hip(hipGetLastError(), "phase tail launch");
}

}  // namespace sht
