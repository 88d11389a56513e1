// Legendre step on gfx950 matrix cores (Eqs. 4 and 5 of the paper).
//
// For each m and each slot (a ring at colatitude t <= pi/2 and its mirror at
// pi - t), lambda_lm is produced by the three-term recursion in l of Eq. 11
// in the rescaled form
//   mu_{l+1} = (alpha_l x +- beta_l) mu_l - mu_{l-1},  lambda_l = f_l mu_l,
// one chain per wavefront lane, with an extended exponent (Sect. 4.1): a lane
// carries an integer scale k (true value = mu 2^(S k)) and contributes nothing
// while k < 0, i.e. while |lambda| < 2^-(S/2).
// Close to the poles the step factor is ~2 and the recursion amplifies any
// error in x = cos t by ~l^2; there the difference form
//   d_{l+1} = (t_l - 2) mu_l + d_l,   mu_{l+1} = mu_l + d_{l+1},
//   t_l - 2 = (alpha_l +- beta_l - 2) - 2 alpha_l sin^2(t/2)
// is used instead (tiles are ordered pole-first, so the choice is per tile).
// lambda never leaves the chip (Sect. 3.2: each value is used as soon as it is
// computed): each chunk of degrees is staged in LDS and fed to MFMA tiles.
//
// Synthesis (Eq. 4), per (m, slot tile):
//   C[slot][col] += sum_k Lambda[slot][k] Coef[k][col]
// k runs over degrees (spin 0) or (degree, W/X) pairs (spin s > 0) of one
// parity class, col over (transform, component, re/im).  For spin s the -s
// chain carries the factor sigma = (-1)^s (real Q, U: Q - iU = sigma sum -s_a
// -s_Y), W, X = (s_lambda +- sigma -s_lambda)/2, and then
// W(pi-t) = sigma (-1)^(l+m) W(t), X(pi-t) = -sigma (-1)^(l+m) X(t) (spin 0:
// lambda(pi-t) = (-1)^(l+m) lambda(t), sigma = 1), so two class accumulators
// A0, A1 give both rings: t: A0 + A1, pi - t: sigma (A0 - A1).
// Column maps (+-s a = -(E +- iB), the HEALPix convention for s = 2):
//   Q_re = -E_re W + B_im X,  Q_im = -E_im W - B_re X,
//   U_re = -B_re W - E_im X,  U_im = -B_im W + E_re X.
//
// Analysis (Eq. 5), per m: out[l][col] = sum_slot Lambda[l][slot] G[slot][col]
// with the ring pair folded into G_t +- G_(pi-t); a work group of ana_nw
// wavefronts walks the active tiles ana_nw * ana_tpw at a time, reduces the
// wavefronts' partial sums in LDS and accumulates them into the output in a
// fixed order (deterministic, no atomics).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "sht_internal.h"

namespace sht {

typedef double dv4 __attribute__((ext_vector_type(4)));
typedef float fv4 __attribute__((ext_vector_type(4)));

template <bool F32>
struct MT;
template <>
struct MT<false> {
    using T = double;
    using V = dv4;
};
template <>
struct MT<true> {
    using T = float;
    using V = fv4;
};

__device__ __forceinline__ dv4 mfma(double a, double b, dv4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ fv4 mfma(float a, float b, fv4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Row of the 16x16 result held in register r of this lane (column = lane & 15);
// the FP64 and FP32 instructions use different result layouts.
template <bool F32>
__device__ __forceinline__ int c_row(int lane, int r)
{
    return F32 ? 4 * (lane >> 4) + r : (lane >> 4) + 4 * r;
}

// base^p for base in [0, 1], p >= 0, as mantissa * 2^ex (mantissa in [0.5, 1)).
__device__ inline void xpow(double base, int p, double &mant, int &ex)
{
    mant = 1.0;
    ex = 0;
    if (p == 0) return;
    if (!(base > 0.0)) {
        mant = 0.0;
        return;
    }
    int eb;
    double mb = frexp(base, &eb);
    for (;;) {
        if (p & 1) {
            int d;
            mant = frexp(mant * mb, &d);
            ex += eb + d;
        }
        p >>= 1;
        if (!p) break;
        int d;
        mb = frexp(mb * mb, &d);
        eb = 2 * eb + d;
    }
}

// ---------------------------------------------------------------- recursion

// One recursion chain per lane.  A wavefront runs chains of a single sign
// (+s or -s), so the per-step coefficients are wave-uniform LDS broadcasts.
struct Chain {
    double x;      // cos t
    double ms2;    // -2 sin^2(t/2)
    double mu;     // mu_l
    double aux;    // mu_{l-1} (plain form) or mu_l - mu_{l-1} (difference form)
    int k;         // scale index (value = mu * 2^(S k)), k <= 0
};

__device__ inline Chain chain_init(const LegView &v, int m, int slot, int chain)
{
    Chain c;
    c.mu = 0.0;
    c.aux = 0.0;
    c.k = 0;
    c.x = 0.0;
    c.ms2 = 0.0;
    if (slot >= v.nslots) return c;
    const double x = v.slot_cos[slot], st = v.slot_sin[slot];
    const double sh = v.slot_shalf[slot];
    c.x = x;
    c.ms2 = -2.0 * sh * sh;
    if (v.polar_T >= 0.0) {
        const double s = (double)v.spin, mm = (double)m;
        double q = mm * mm + s * s - 2.0 * mm * s * x;
        double crit = sqrt(q > 0.0 ? q : 0.0) - (double)v.lmax * st;
        if (crit > v.polar_T) return c;   // skipped term (Sect. 3.3)
    }
    const StartCoef sc = v.start[2 * m + chain];
    double mc, ms;
    int ec, es;
    xpow(v.slot_chalf[slot], sc.p, mc, ec);
    xpow(sh, sc.q, ms, es);
    int d;
    double mant = frexp(sc.kmant * mc * ms, &d);
    if (mant == 0.0) return c;
    const int e = sc.kexp + ec + es + d;
    const int S = v.rescale_bits, T = v.thresh_bits;
    int kk = 0;
    if (e < T) kk = (T - e) / S;
    c.k = -kk;
    c.mu = (double)sc.sign * ldexp(mant, e + S * kk);
    return c;
}

// Per-chain step coefficients of one degree, staged in LDS:
// (alpha_l, +-beta_l, alpha_l +- beta_l - 2, scale * f_l) for the chain's sign;
// the last entry turns mu into the value written out (lambda times a constant).
__device__ inline double4 chain_coef(const double4 c, bool minus, double fs)
{
    return minus ? double4{c.x, -c.y, c.w, fs} : double4{c.x, c.y, c.z, fs};
}

// Run the recursion over the degrees lc .. lc+LC-1, writing mu (SCALE: times
// cf.w, i.e. c f_l mu = c lambda) to out[row(t) * stride]; 0 while the lane's
// scale k < 0 and outside [l0, lmax].  Without SCALE the caller applies f_l on
// the side of the product with fewer values per degree.
// Row of degree offset t in the chunk: natural order, or (PSPLIT) the even
// offsets first and then the odd ones.
template <int LC, bool PSPLIT>
__device__ __forceinline__ int chunk_row(int t)
{
    return PSPLIT ? (t & 1) * (LC / 2) + (t >> 1) : t;
}

template <typename T, int LC, bool PSPLIT, bool SCALE>
__device__ inline void chain_chunk(Chain &c, const double4 *__restrict__ cf, bool diff, bool slow,
                                   int l0, int lc, int lmax, T *out, int stride, double thr,
                                   double down)
{
    if (!slow) {
#pragma unroll 4
        for (int t = 0; t < LC; ++t) {
            const int l = lc + t;
            out[chunk_row<LC, PSPLIT>(t) * stride] =
                (l >= l0 && l <= lmax) ? (T)(SCALE ? c.mu * cf[t].w : c.mu) : (T)0;
            if (l >= l0 && l < lmax) {
                const double4 q = cf[t];
                if (diff) {
                    const double eps = fma(q.x, c.ms2, q.z);
                    c.aux = fma(eps, c.mu, c.aux);
                    c.mu += c.aux;
                } else {
                    const double tt = fma(q.x, c.x, q.y);
                    const double nx = fma(tt, c.mu, -c.aux);
                    c.aux = c.mu;
                    c.mu = nx;
                }
            }
        }
    } else {
        for (int t = 0; t < LC; ++t) {
            const int l = lc + t;
            out[chunk_row<LC, PSPLIT>(t) * stride] =
                (l >= l0 && l <= lmax && c.k == 0) ? (T)(SCALE ? c.mu * cf[t].w : c.mu) : (T)0;
            if (l >= l0 && l < lmax) {
                const double4 q = cf[t];
                if (diff) {
                    const double eps = fma(q.x, c.ms2, q.z);
                    c.aux = fma(eps, c.mu, c.aux);
                    c.mu += c.aux;
                } else {
                    const double tt = fma(q.x, c.x, q.y);
                    const double nx = fma(tt, c.mu, -c.aux);
                    c.aux = c.mu;
                    c.mu = nx;
                }
                if (c.k < 0 && fabs(c.mu) >= thr) {
                    c.mu *= down;
                    c.aux *= down;
                    c.k += 1;
                }
            }
        }
    }
}

// Fast path of chain_chunk: every degree of the chunk lies in [l0, lmax) and
// every lane of the wavefront already has k = 0 (no masking, no rescaling).
template <typename T, int LC, bool PSPLIT, bool SCALE>
__device__ __forceinline__ void chain_chunk_fast(Chain &c, const double4 *__restrict__ cf, bool diff,
                                                 T *out, int stride)
{
    if (diff) {
#pragma unroll
        for (int t = 0; t < LC; ++t) {
            const double4 q = cf[t];
            out[chunk_row<LC, PSPLIT>(t) * stride] = (T)(SCALE ? c.mu * q.w : c.mu);
            const double eps = fma(q.x, c.ms2, q.z);
            c.aux = fma(eps, c.mu, c.aux);
            c.mu += c.aux;
        }
    } else {
#pragma unroll
        for (int t = 0; t < LC; ++t) {
            const double4 q = cf[t];
            out[chunk_row<LC, PSPLIT>(t) * stride] = (T)(SCALE ? c.mu * q.w : c.mu);
            const double nx = fma(fma(q.x, c.x, q.y), c.mu, -c.aux);
            c.aux = c.mu;
            c.mu = nx;
        }
    }
}

__device__ __forceinline__ bool wave_any(bool p)
{
    return __builtin_amdgcn_ballot_w64(p) != 0;
}

// wavefronts with a slot of cos t above this use the difference form
constexpr double DIFF_FORM_COS = 0.7;

// ---------------------------------------------------------------- synthesis

constexpr int SYN_LC = 16;          // degrees per chunk
constexpr int SYN_ROW = 64 + 8;     // LDS row of lambda: one degree, 64 chains (+ pad)

// Exchange of values between lanes q and 3 - q of every group of four lanes
// (the four columns Q_re, Q_im, U_re, U_im of one transform).
__device__ __forceinline__ float quad_rev(float x)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x1B, 0xF, 0xF, false));
}
__device__ __forceinline__ double quad_rev(double x)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffLL), 0x1B, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x1B, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// One wavefront per work item (m, slot tile, group of transforms); no data is
// shared between wavefronts, so there is no work-group barrier beyond the
// wavefront itself.
//
// Recursion: lane = chain * 32 + slot (spin 2: chain 0 = +2, 1 = -2) or lane =
// slot (spin 0); each chunk of SYN_LC degrees of mu_l is written to LDS, and
// the factor c f_l (c = 1/2 for spin 2, 1 for spin 0) goes onto the
// coefficients (four degrees per lane instead of sixteen recursion steps).
//
// Products (Eq. 4) on 16x16x4 matrix-core tiles, rows = 16 slots, columns =
// 16 of the group's (transform, component, re/im) columns, k = 4 degrees of
// one parity class (degrees lc + 8h + 2kk + parity, lc + m even):
//   spin 0:  A = lambda,  B = (Re a_lm, Im a_lm) per transform;
//   spin 2:  rows W = -(lambda_+ + lambda_-)/2 and X = (lambda_+ - lambda_-)/2,
//            B_W[o] = (E_re, E_im, B_re, B_im)[o] and B_X[o] = s_o B_W[3 - o],
//            s = (+, -, -, +), for the columns o = (Q_re, Q_im, U_re, U_im).
// The B operand is read from a_lm straight into registers (one chunk ahead),
// the X form by a lane exchange inside groups of four.  Class 0 collects the
// terms whose mirror-ring sign is +1 (W at l + m even, X at l + m odd), class
// 1 the others; ring t gets A0 + A1, ring pi - t gets A0 - A1.
template <int SPIN, bool F32>
struct SynShared {
    typename MT<F32>::T lam[SYN_LC][SYN_ROW];
    double4 cfs[2][SPIN ? 2 : 1][SYN_LC];
};

template <int SPIN, int NCB, bool F32>
__device__ __forceinline__ void synth_item(const LegView &v, const WaveItem it,
                                           const double *__restrict__ alm, double *__restrict__ phase,
                                           int flush_chunks, int deriv, SynShared<SPIN, F32> &sh)
{
    using T = typename MT<F32>::T;
    using V = typename MT<F32>::V;
    constexpr int SPT = SPIN ? 32 : 64;          // slots per tile
    constexpr int NSB = SPT / 16;                // 16-slot row blocks
    constexpr int NCH = SPIN ? 2 : 1;
    constexpr int LC = SYN_LC;
    constexpr int NCOMP = SPIN ? 2 : 1;
    constexpr int CPJ = SPIN ? 4 : 2;            // columns per transform
    auto &lam = sh.lam;
    auto &cfs = sh.cfs;

    const int lane = threadIdx.x;
    const int i16 = lane & 15, kk = lane >> 4;
    if (it.m < 0) return;
    const int m = it.m, tile = it.tile, t0 = it.t0;
    const int lmax = v.lmax;
    const int l0 = (SPIN && v.spin > m) ? v.spin : m;
    const double ssign = (SPIN && (v.spin & 1)) ? -1.0 : 1.0;   // sigma = (-1)^s of the mirror ring
    const int lstart = l0 - ((l0 + m) & 1);
    const double4 *coef = v.coef + v.coef_ofs[m];
    const double *flm = v.fl + v.coef_ofs[m];
    const int64_t mbase = (int64_t)m * (2 * (int64_t)lmax + 1 - m) / 2;
    const double thr = ldexp(1.0, v.thresh_bits), down = ldexp(1.0, -v.rescale_bits);
    const double fscale = SPIN ? 0.5 : 1.0;

    // recursion role
    const int rslot = SPIN ? (lane & 31) : lane;
    const int rchain = SPIN ? (lane >> 5) : 0;
    Chain cs = chain_init(v, m, tile * SPT + rslot, rchain);
    const bool diff = wave_any(cs.x > DIFF_FORM_COS);
    if (diff) cs.aux = cs.mu;
    bool slow = wave_any(cs.k < 0);

    // B operand sources: this lane's column in each column block (columns that
    // take no part -- beyond the last transform, Im at m = 0, B of a derivative
    // synthesis -- read zeros).  Derivative synthesis (spin-1 plan): the input
    // holds one component per transform, taken as E with B = 0.
    if (!SPIN) deriv = 0;
    const int ncin = deriv ? 1 : NCOMP;
    const double *bp[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
        const int col = i16 + 16 * cb;
        const int t = t0 + col / CPJ, o = col % CPJ;
        const int comp = SPIN ? (o >> 1) : 0, reim = o & 1;
        const bool ok = t < v.ntrans && !(m == 0 && reim) && !(deriv && comp);
        bp[cb] = ok ? alm + (((int64_t)t * ncin + comp) * v.nalm + mbase) * 2 + reim : v.zeros;
    }
    // The X products need sigma_o = (+, -, -, +) times the coefficient of column
    // 3 - o.  FP64: the staged coefficients carry tau_o = (+, +, -, +) instead
    // (tau_o tau_(3-o) = sigma_o), taken by the lane exchange with no sign; the
    // sums then hold tau_o times the result, undone once in the epilogue (FP32:
    // measured slower, the exchanged operand is negated where sigma_o = -1).
    const bool tneg = SPIN && !F32 && (i16 & 3) == 2;
    const bool xneg = SPIN && F32 && ((i16 & 3) == 1 || (i16 & 3) == 2);

    // coefficients of a chunk: R[par][h][cb] = a(column, lc + 8h + 2kk + par),
    // loaded one chunk ahead from clamped addresses; degrees outside [l0, lmax]
    // meet lambda = 0 in the products, so the values there need no masking
    double R[2][2][NCB], Rn[2][2][NCB];
    auto loadB = [&](int lc, double (&dst)[2][2][NCB]) {
        if (lc >= l0 && lc + LC <= lmax + 1) {
            // the whole chunk lies in [l0, lmax]: one address per column block,
            // the four degrees of this lane at fixed offsets from it
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                const double *p = bp[cb] + 2 * (int64_t)(lc + 2 * kk);
#pragma unroll
                for (int par = 0; par < 2; ++par)
#pragma unroll
                    for (int h = 0; h < 2; ++h) dst[par][h][cb] = p[2 * (8 * h + par)];
            }
        } else {
#pragma unroll
            for (int par = 0; par < 2; ++par)
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int cb = 0; cb < NCB; ++cb) {
                        const int l = lc + 8 * h + 2 * kk + par;
                        const int lcl = l < l0 ? l0 : (l > lmax ? lmax : l);
                        dst[par][h][cb] = bp[cb][2 * (int64_t)lcl];
                    }
        }
    };
    double4 c0n = double4{0, 0, 0, 0};
    double f0n = 0.0;
    auto loadC = [&](int lc) {
        const int l = lc + lane % LC;
        const int lcl = l < l0 ? l0 : (l > lmax ? lmax : l);   // clamped address
        c0n = coef[lcl];
        f0n = flm[lcl];
    };
    // f_l of a derivative synthesis also carries sqrt(l (l + 1)): E_lm of the
    // gradient of a scalar field is sqrt(l (l + 1)) a_lm (a table lookup: an
    // FP64 square root here would cost registers at the loop's peak)
    auto storeC = [&](int buf, int lc) {
        const int l = lc + lane % LC;
        const double4 c = (l >= l0 && l < lmax) ? c0n : double4{0, 0, 0, 0};
        const double kd = deriv ? v.dfac[l <= lmax ? l : lmax] : 1.0;
        const double f = (l >= l0 && l <= lmax) ? f0n * fscale * kd : 0.0;
        if (lane < NCH * LC) cfs[buf][lane / LC][lane % LC] = chain_coef(c, lane >= LC, f);
    };
    // c f_l onto the coefficients of the chunk staged in cfs[buf] (zero outside
    // [l0, lmax]): the recursion then writes plain mu
    auto scaleB = [&](int buf, double (&dst)[2][2][NCB]) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int par = 0; par < 2; ++par) {
                const double f0 = cfs[buf][0][8 * h + 2 * kk + par].w;
                const double f = tneg ? -f0 : f0;
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb) dst[par][h][cb] *= f;
            }
    };

    V acc[2][NSB][NCB];
    double acc64[F32 ? 2 : 1][F32 ? NSB : 1][F32 ? NCB : 1][4];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int sb = 0; sb < NSB; ++sb)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) acc[p][sb][cb] = V{0, 0, 0, 0};
    if constexpr (F32) {
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int sb = 0; sb < NSB; ++sb)
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc64[p][sb][cb][r] = 0.0;
    }

    loadB(lstart, R);
    loadC(lstart);
    storeC(0, lstart);
    __syncthreads();
    scaleB(0, R);
    int chunk = 0;
    for (int lc = lstart; lc <= lmax; lc += LC, ++chunk) {
        const int buf = chunk & 1;
        const bool more = lc + LC <= lmax;
        if (more) {
            loadB(lc + LC, Rn);
            loadC(lc + LC);
        }
        T *out = &lam[0][lane];
        if (!slow && lc >= l0 && lc + LC <= lmax) {
            chain_chunk_fast<T, LC, false, false>(cs, cfs[buf][rchain], diff, out, SYN_ROW);
        } else {
            chain_chunk<T, LC, false, false>(cs, cfs[buf][rchain], diff, slow, l0, lc, lmax, out, SYN_ROW, thr,
                                            down);
            slow = wave_any(cs.k < 0);
        }
        __syncthreads();
        if constexpr (SPIN == 0) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                T b0[NCB], b1[NCB];
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb) {
                    b0[cb] = (T)R[0][h][cb];
                    b1[cb] = (T)R[1][h][cb];
                }
#pragma unroll
                for (int sb = 0; sb < NSB; ++sb) {
                    const T a0 = lam[8 * h + 2 * kk][sb * 16 + i16];
                    const T a1 = lam[8 * h + 2 * kk + 1][sb * 16 + i16];
#pragma unroll
                    for (int cb = 0; cb < NCB; ++cb) {
                        acc[0][sb][cb] = mfma(a0, b0[cb], acc[0][sb][cb]);
                        acc[1][sb][cb] = mfma(a1, b1[cb], acc[1][sb][cb]);
                    }
                }
            }
        } else {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                T bwe[NCB], bwo[NCB], bxe[NCB], bxo[NCB];
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb) {
                    bwe[cb] = (T)R[0][h][cb];
                    bwo[cb] = (T)R[1][h][cb];
                    const T xe = quad_rev(bwe[cb]), xo = quad_rev(bwo[cb]);
                    bxe[cb] = xneg ? -xe : xe;
                    bxo[cb] = xneg ? -xo : xo;
                }
#pragma unroll
                for (int sb = 0; sb < NSB; ++sb) {
                    const int te = 8 * h + 2 * kk;
                    const T upe = lam[te][sb * 16 + i16], ume = lam[te][32 + sb * 16 + i16];
                    const T upo = lam[te + 1][sb * 16 + i16], umo = lam[te + 1][32 + sb * 16 + i16];
                    const T awe = -(upe + ume), axe = upe - ume;
                    const T awo = -(upo + umo), axo = upo - umo;
#pragma unroll
                    for (int cb = 0; cb < NCB; ++cb) {
                        acc[0][sb][cb] = mfma(awe, bwe[cb], acc[0][sb][cb]);
                        acc[0][sb][cb] = mfma(axo, bxo[cb], acc[0][sb][cb]);
                        acc[1][sb][cb] = mfma(awo, bwo[cb], acc[1][sb][cb]);
                        acc[1][sb][cb] = mfma(axe, bxe[cb], acc[1][sb][cb]);
                    }
                }
            }
        }
        if constexpr (F32) {
            if ((chunk + 1) % flush_chunks == 0) {
#pragma unroll
                for (int p = 0; p < 2; ++p)
#pragma unroll
                    for (int sb = 0; sb < NSB; ++sb)
#pragma unroll
                        for (int cb = 0; cb < NCB; ++cb) {
#pragma unroll
                            for (int r = 0; r < 4; ++r) acc64[p][sb][cb][r] += (double)acc[p][sb][cb][r];
                            acc[p][sb][cb] = V{0, 0, 0, 0};
                        }
            }
        }
        if (more) {
            storeC(buf ^ 1, lc + LC);
#pragma unroll
            for (int par = 0; par < 2; ++par)
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int cb = 0; cb < NCB; ++cb) R[par][h][cb] = Rn[par][h][cb];
        }
        __syncthreads();
        if (more) scaleB(buf ^ 1, R);
    }

    // ring indices of this lane's output rows, all loaded before any store
    int eyn[NSB][4], eys[NSB][4];
#pragma unroll
    for (int sb = 0; sb < NSB; ++sb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int slot = tile * SPT + sb * 16 + c_row<F32>(lane, r);   // < ntiles * SPT
            eyn[sb][r] = v.slot_yn[slot];
            eys[sb][r] = v.slot_ys[slot];
        }

    // epilogue: ring t = A0 + A1, ring pi - t = sigma (A0 - A1), both times tau_o
#pragma unroll
    for (int sb = 0; sb < NSB; ++sb)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                double c0, c1;
                if constexpr (F32) {
                    c0 = acc64[0][sb][cb][r] + (double)acc[0][sb][cb][r];
                    c1 = acc64[1][sb][cb][r] + (double)acc[1][sb][cb][r];
                } else {
                    c0 = acc[0][sb][cb][r];
                    c1 = acc[1][sb][cb][r];
                }
                const int row = c_row<F32>(lane, r);
                const int slot = tile * SPT + sb * 16 + row;
                if (slot >= v.nslots) continue;
                const int col = i16 + 16 * cb;
                const int t = t0 + col / CPJ, o = col % CPJ;
                if (t >= v.ntrans) continue;
                const int comp = SPIN ? (o >> 1) : 0, reim = o & 1;
                const int yn = eyn[sb][r], ys = eys[sb][r];
                const int64_t rowbase = ((int64_t)t * NCOMP + comp) * v.nrings;
                const double ts = tneg ? -1.0 : 1.0;   // undo tau_o
                if (yn >= 0) phase[((rowbase + yn) * (v.mmax + 1) + m) * 2 + reim] = ts * (c0 + c1);
                if (ys >= 0) phase[((rowbase + ys) * (v.mmax + 1) + m) * 2 + reim] = (ssign * ts) * (c0 - c1);
            }
}

template <int SPIN, int NCB, bool F32>
__global__ __launch_bounds__(64) void k_legendre_synth(LegView v, const WaveItem *__restrict__ items,
                                                       const double *__restrict__ alm,
                                                       double *__restrict__ phase, int flush_chunks, int deriv)
{
    __shared__ SynShared<SPIN, F32> sh;
    synth_item<SPIN, NCB, F32>(v, items[blockIdx.x], alm, phase, flush_chunks, deriv, sh);
}

// ---------------------------------------------------------------- analysis

constexpr int ANA_LC = 32;   // degrees per chunk (16 per parity class)
// slot tiles per wavefront and pass: two, except where the stationary phases
// of two 64-slot tiles and 32 columns would not fit the registers
template <int SPIN, int NCB>
constexpr int ana_tpw() { return (SPIN == 0 && NCB == 2) ? 1 : 2; }

// Orders the LDS traffic of one wavefront at this point (the LDS executes a
// wavefront's requests in issue order; this keeps the compiler from moving
// them across).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Work group = one m and a group of transforms.  The m's active slot tiles are
// taken NW * TPW at a time (TPW per wavefront).  For every chunk of
// degrees each wavefront runs the recursion of one of its tiles (lane =
// chain * 32 + slot, or slot) into its own LDS region, multiplies lambda^T (16
// degrees of one parity x 4 slots) with that tile's phases held in registers
// as G_t +- G_(pi-t) on 16x16x4 matrix-core tiles, and repeats for its next
// tile into the same accumulators; it then leaves its partial sums in the same
// region, and after one work-group barrier the partial sums of the wavefronts
// are added in a fixed order and accumulated into a_lm (deterministic, no
// atomics).  Every pass over the tiles reads and writes the m's a_lm once, so
// TPW > 1 divides that traffic by TPW at the cost of registers.
template <int SPIN, bool F32>
struct AnaShape {
    static constexpr int SPT = SPIN ? 32 : 64;
    static constexpr int NCH = SPIN ? 2 : 1;
    static constexpr int LDP = SPT + 1;
    static constexpr int LAMW = NCH * ANA_LC * LDP;
};
// LDS slot of partial-sum element e: rows of 64 elements padded by two.  The
// sixteen lanes of one accumulator store cover eight rows of 64 (transform and
// component) at the same offset and re/im, which unpadded fall on two banks.
__device__ __forceinline__ constexpr int psidx(int e) { return e + 2 * (e >> 6); }

template <int SPIN, int NCB, bool F32>
struct AnaShared {
    // FP32 form: the partial sums (FP32 products) get a region of their own,
    // double-buffered by chunk, so one work-group barrier per chunk suffices;
    // the FP64 partial sums reuse the lambda region (two barriers per chunk):
    // a second region would not fit the 160 KB of LDS next to eight wavefronts'
    // lambda
    static constexpr bool PSEP = F32;
    static constexpr int LAMB = AnaShape<SPIN, F32>::LAMW * (int)sizeof(typename MT<F32>::T);
    static constexpr int NOUT = ANA_LC * NCB * 16;
    static constexpr int NOUTP = NOUT + 2 * (NOUT / 64);   // padded (psidx)
    static constexpr int NOUTB = NOUTP * 8;
    static constexpr int REG_D = ((PSEP ? LAMB : (LAMB > NOUTB ? LAMB : NOUTB)) + 7) / 8;
    static constexpr int NW = ana_nw(F32, SPIN != 0);
    double smem[NW * REG_D];
    float psum[PSEP ? 2 * NW * NOUTP : 1];
    double4 cfs[NW][SPIN ? 2 : 1][ANA_LC];
    double fls[PSEP ? 2 : 1][ANA_LC];   // c f_l of the chunk's degrees (c = 1/2 for spin 2), applied to the sums
};

template <int SPIN, int NCB, bool F32, int TPW>
__device__ __forceinline__ void anal_item(const LegView &v, const int m, const int t0,
                                          const double *__restrict__ phase, double *__restrict__ alm,
                                          int mode, AnaShared<SPIN, NCB, F32> &sh)
{
    using T = typename MT<F32>::T;
    using V = typename MT<F32>::V;
    constexpr int SPT = SPIN ? 32 : 64;
    constexpr int LC = ANA_LC;
    constexpr int KSA = SPT / 4;       // k-steps (4 slots each) per tile
    constexpr int NCH = SPIN ? 2 : 1;
    constexpr int NCOMP = SPIN ? 2 : 1;
    constexpr int LDP = SPT + 1;       // padded LDS row
    constexpr int NW = ana_nw(F32, SPIN != 0);
    constexpr int NT = 64 * NW;
    constexpr int CPJ = SPIN ? 4 : 2;  // columns per transform
    constexpr int NCOL = NCB * 16;
    constexpr int NOUT = LC * NCOL;    // output elements per chunk
    constexpr int NOUTP = AnaShared<SPIN, NCB, F32>::NOUTP;
    static_assert(NOUT % 64 == 0 && NOUTP == NOUT + 2 * (NOUT / 64), "partial-sum layout");
    constexpr int OPT = (NOUT + NT - 1) / NT;
    constexpr int LAMW = NCH * LC * LDP;   // lambda elements per wavefront
    // per wavefront: lambda [chain][row][LDP] (rows: even degree offsets, then
    // odd ones), reused for the wavefront's partial sums once its products are done
    constexpr int REG_D = AnaShared<SPIN, NCB, F32>::REG_D;
    double *smem = sh.smem;
    auto &cfs = sh.cfs;

    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int i16 = lane & 15, kk = lane >> 4;
    const int lmax = v.lmax;
    const int l0 = (SPIN && v.spin > m) ? v.spin : m;
    const double ssign = (SPIN && (v.spin & 1)) ? -1.0 : 1.0;   // sigma = (-1)^s of the mirror ring
    const int lstart = l0 - ((l0 + m) & 1);
    const double4 *coef = v.coef + v.coef_ofs[m];
    const double *flm = v.fl + v.coef_ofs[m];
    const int64_t mbase = (int64_t)m * (2 * (int64_t)lmax + 1 - m) / 2;
    const double thr = ldexp(1.0, v.thresh_bits), down = ldexp(1.0, -v.rescale_bits);
    T *lam_w = reinterpret_cast<T *>(smem + wave * REG_D);
    double *part_w = smem + wave * REG_D;
    const int rslot = SPIN ? (lane & 31) : lane;
    const int rchain = SPIN ? (lane >> 5) : 0;
    T *lam_out = lam_w + rchain * LC * LDP + rslot;
    // mode bit 0: real-field gradient factor fac_m; bit 1 (spin-1 plans): adjoint
    // of the derivative synthesis, whose output is sqrt(l (l + 1)) times the E
    // component alone (one component per transform)
    const bool grad = mode & ANA_MODE_GRAD;
    const bool deriv = SPIN && (mode & ANA_MODE_DERIV);

    // this thread's output elements of a chunk: element e = tid + j NT ->
    // (row tc = transform * NCOMP + component, degree offset, re/im), consecutive
    // e consecutive in memory.  The degree offset and re/im do not depend on j,
    // and the row advances by TCS per j.
    static_assert((NT / 2) % LC == 0, "output element mapping");
    constexpr int TCS = NT / 2 / LC;
    static_assert(TCS % 2 == 0, "rows of one thread share their component");
    const int oreim = tid & 1, oloff = (tid >> 1) % LC, tc0 = (tid >> 1) / LC;
    unsigned ovalid = 0;   // bit j: element j exists (row in this group, transform < ntrans)
#pragma unroll
    for (int j = 0; j < OPT; ++j) {
        const int tc = tc0 + TCS * j;
        if (tc < NCOL / 2 && t0 + tc / NCOMP < v.ntrans && !(deriv && (tc % NCOMP))) ovalid |= 1u << j;
    }
    // output row of (transform, component): t NCOMP + comp, or t alone (derivative adjoint)
    const int64_t ostride = (int64_t)(deriv ? TCS / NCOMP : TCS) * v.nalm * 2;
    const int64_t orow0 = deriv ? (int64_t)t0 + tc0 / NCOMP : (int64_t)t0 * NCOMP + tc0;
    // row tc0 of this group (only dereferenced for valid elements; loads of
    // invalid ones go to the start of alm instead)
    double *const obase = alm + (orow0 * v.nalm + mbase) * 2 + oreim;

    // degrees m .. l0-1 (spin s > m) are zero by convention
    {
        const int nz = l0 - m;
        for (int e = tid; e < nz * 2 * NCOMP * (NCOL / CPJ); e += NT) {
            const int l = m + e % nz;
            const int rest = e / nz;
            const int reim = rest & 1, tc = rest >> 1;
            const int t = t0 + tc / NCOMP, comp = tc % NCOMP;
            if (t < v.ntrans && !(deriv && comp))
                alm[(((int64_t)t * (deriv ? 1 : NCOMP) + comp) * v.nalm + mbase + l) * 2 + reim] = 0.0;
        }
    }

    int ntiles_act = 0;
    for (int t = 0; t < v.ntiles; ++t) ntiles_act += v.tile_mlim[t] >= m;
    int tcount = 0, tscan = 0;
    bool first = true;
    // column sign tau_o = (+, +, +, -) for o = 0..3 (see the stationary operand)
    const bool tneg = SPIN && (i16 & 3) == 3;
    constexpr bool PSEP = AnaShared<SPIN, NCB, F32>::PSEP;
    int cidx = 0;   // chunks done (selects the partial-sum buffer)
    while (tcount < ntiles_act || first) {
        int ptile[TPW];    // this wavefront's tiles in this pass (-1: none)
#pragma unroll
        for (int i = 0; i < TPW; ++i) ptile[i] = -1;
        {
            int k = 0;
            for (; tscan < v.ntiles && k < NW * TPW; ++tscan) {
                if (v.tile_mlim[tscan] < m) continue;
#pragma unroll
                for (int i = 0; i < TPW; ++i)
                    if (k == i * NW + wave) ptile[i] = tscan;
                ++k;
            }
            tcount += k;
        }
        // stationary phase fragments B[kk][j] for slot 4 ks + kk and column j + 16 cb:
        // gw[i][q] multiplies W (spin 2) or lambda (spin 0) rows of tile i; q = 0:
        // G_t + G_(pi-t), q = 1: G_t - G_(pi-t).  For output o the X rows take
        // sigma_o times the W operand of column 3 - o, sigma = (-, +, +, -).  The
        // operand is stored times tau_o = (+, +, +, -) and the X rows take the
        // column 3 - o of it by a lane exchange within the four columns of a
        // transform, with no sign: the sums then hold tau_o (W_o + sigma_o X_o)
        // (tau_o tau_(3-o) = sigma_o), and tau_o is applied once per chunk when
        // they leave the registers.
        // (all loads unconditional from clamped addresses, so that they are
        // issued together rather than one conditional block at a time)
        T gw[TPW][2][KSA][NCB];
        Chain cs[TPW];
        bool diff[TPW], slow[TPW];
#pragma unroll
        for (int i = 0; i < TPW; ++i) {
            const bool active = ptile[i] >= 0;
            const int slot0 = active ? ptile[i] * SPT : 0;
            int ynv[KSA], ysv[KSA];
#pragma unroll
            for (int ks = 0; ks < KSA; ++ks) {
                const int slot = slot0 + 4 * ks + kk;     // < ntiles * SPT (tables padded)
                const int yn = v.slot_yn[slot], ys = v.slot_ys[slot];
                const bool ok = active && slot < v.nslots;
                ynv[ks] = ok ? yn : -1;
                ysv[ks] = ok ? ys : -1;
            }
#pragma unroll
            for (int ks = 0; ks < KSA; ++ks) {
                const int yn = ynv[ks], ys = ysv[ks];
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb) {
                    const int col = i16 + 16 * cb;
                    const int tl = col / CPJ, o = col % CPJ;
                    const int t = t0 + tl;
                    const int comp = SPIN ? (o >> 1) : 0, reim = o & 1;
                    const bool tok = t < v.ntrans;
                    const int64_t rowbase = ((int64_t)(tok ? t : 0) * NCOMP + comp) * v.nrings;
                    const double gn0 = phase[((rowbase + (yn >= 0 ? yn : 0)) * (v.mmax + 1) + m) * 2 + reim];
                    const double gs0 = phase[((rowbase + (ys >= 0 ? ys : 0)) * (v.mmax + 1) + m) * 2 + reim];
                    const double gn = (tok && yn >= 0) ? gn0 : 0.0;
                    const double gs = (tok && ys >= 0) ? ssign * gs0 : 0.0;
                    const double sg = SPIN ? ((o == 3) ? 1.0 : -1.0) : 1.0;   // -tau_o (spin > 0)
                    gw[i][0][ks][cb] = (T)(sg * (gn + gs));
                    gw[i][1][ks][cb] = (T)(sg * (gn - gs));
                }
            }
            cs[i] = chain_init(v, m, active ? ptile[i] * SPT + rslot : v.nslots, rchain);
            diff[i] = wave_any(cs[i].x > DIFF_FORM_COS);
            if (diff[i]) cs[i].aux = cs[i].mu;
            slow[i] = wave_any(cs[i].k < 0);
        }
        const bool any_active = ptile[0] >= 0;   // tiles are dealt to slot 0 first
        // step coefficients of this lane's (chain, degree) entry, loaded one
        // chunk ahead from a clamped address and masked when staged
        double4 c0n = double4{0, 0, 0, 0};
        double f0n = 0.0;
        auto loadC = [&](int lc) {
            const int l = lc + (lane % LC);
            const int lcl = l < l0 ? l0 : (l > lmax ? lmax : l);
            c0n = coef[lcl];
            f0n = flm[lcl];
        };
        loadC(lstart);
        for (int lc = lstart; lc <= lmax; lc += LC) {
            V acc[2][NCB];   // [class][column block]
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb) acc[p][cb] = V{0, 0, 0, 0};
            {
                const int l = lc + (lane % LC);
                const double kd = deriv ? v.dfac[l <= lmax ? l : lmax] : 1.0;
                const double f = (l >= l0 && l <= lmax) ? f0n * (SPIN ? 0.5 : 1.0) * kd : 0.0;
                if (wave == 0 && lane < LC) sh.fls[PSEP ? (cidx & 1) : 0][lane] = f;
                if (any_active) {
                    const double4 c = (l >= l0 && l < lmax) ? c0n : double4{0, 0, 0, 0};
                    if (lane < NCH * LC) cfs[wave][lane / LC][lane % LC] = chain_coef(c, lane >= LC, f);
                }
            }
            if (lc + LC <= lmax) loadC(lc + LC);
#pragma unroll
            for (int i = 0; i < TPW; ++i) {
                if (ptile[i] < 0) continue;
                wave_sync();
                if (!slow[i] && lc >= l0 && lc + LC <= lmax) {
                    chain_chunk_fast<T, LC, true, false>(cs[i], cfs[wave][rchain], diff[i], lam_out, LDP);
                } else {
                    chain_chunk<T, LC, true, false>(cs[i], cfs[wave][rchain], diff[i], slow[i], l0, lc, lmax,
                                                    lam_out, LDP, thr, down);
                    slow[i] = wave_any(cs[i].k < 0);
                }
                wave_sync();
#pragma unroll
                for (int p = 0; p < 2; ++p) {
#pragma unroll
                    for (int ks = 0; ks < KSA; ++ks) {
                        // A[i][kk] = Lambda[degree lc + p + 2 i][slot 4 ks + kk] (rows split by parity)
                        if constexpr (SPIN == 0) {
                            const T a = lam_w[(p * (LC / 2) + i16) * LDP + 4 * ks + kk];
#pragma unroll
                            for (int cb = 0; cb < NCB; ++cb) acc[p][cb] = mfma(a, gw[i][p][ks][cb], acc[p][cb]);
                        } else {
                            const T up = lam_w[(0 * LC + p * (LC / 2) + i16) * LDP + 4 * ks + kk];
                            const T um = lam_w[(1 * LC + p * (LC / 2) + i16) * LDP + 4 * ks + kk];
                            const T aw = up + um, ax = up - um;
#pragma unroll
                            for (int cb = 0; cb < NCB; ++cb) {
                                acc[p][cb] = mfma(aw, gw[i][p][ks][cb], acc[p][cb]);
                                const T q = quad_rev(gw[i][1 - p][ks][cb]);
                                acc[p][cb] = mfma(ax, q, acc[p][cb]);
                            }
                        }
                    }
                }
                wave_sync();   // lambda reads issued: the region takes the next tile or the partial sums
            }
            // the previous passes' sums of this thread's outputs (loaded after the
            // products, so that they take no registers during them)
            double pold[OPT];
            if (!first) {
#pragma unroll
                for (int j = 0; j < OPT; ++j) {
                    const int l = lc + oloff;
                    const int lcl = l < l0 ? l0 : (l > lmax ? lmax : l);
                    const double *src = ((ovalid >> j) & 1) ? obase + j * ostride : alm;
                    pold[j] = src[2 * (int64_t)lcl];   // used only where l is in range
                }
            }
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = c_row<F32>(lane, r);
                        const int col = i16 + 16 * cb;
                        const int tl = col / CPJ, o = col % CPJ;
                        const int comp = SPIN ? (o >> 1) : 0, reim = o & 1;
                        const int e = (((tl * NCOMP + comp) * LC) + p + 2 * row) * 2 + reim;
                        const T a = tneg ? -acc[p][cb][r] : acc[p][cb][r];
                        if constexpr (PSEP)
                            sh.psum[((cidx & 1) * NW + wave) * NOUTP + psidx(e)] = any_active ? (float)a : 0.0f;
                        else
                            part_w[psidx(e)] = any_active ? (double)a : 0.0;
                    }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < OPT; ++j) {
                const int e = tid + j * NT;
                const int l = lc + oloff;
                if (!((ovalid >> j) & 1) || l < l0 || l > lmax) continue;
                double s = 0.0;
#pragma unroll
                for (int w = 0; w < NW; ++w) {
                    if constexpr (PSEP) s += (double)sh.psum[((cidx & 1) * NW + w) * NOUTP + psidx(e)];
                    else s += smem[w * REG_D + psidx(e)];
                }
                s *= sh.fls[PSEP ? (cidx & 1) : 0][oloff];
                if (grad && m > 0) s *= 2.0;   // fac_m of the real-field gradient
                if (m == 0 && oreim) s = 0.0;
                obase[j * ostride + 2 * (int64_t)l] = first ? s : pold[j] + s;
            }
            if constexpr (!PSEP) __syncthreads();
            ++cidx;
        }
        first = false;
    }
}

template <int SPIN, int NCB, bool F32>
__global__ __launch_bounds__(64 * ana_nw(F32, SPIN != 0), 2) void k_legendre_anal(LegView v, const int *__restrict__ mlist,
                                                                  const double *__restrict__ phase,
                                                                  double *__restrict__ alm,
                                                                  int jobs_per_group, int mode)
{
    __shared__ AnaShared<SPIN, NCB, F32> sh;
    anal_item<SPIN, NCB, F32, ana_tpw<SPIN, NCB>()>(v, mlist[blockIdx.x], (int)blockIdx.y * jobs_per_group, phase, alm, mode, sh);
}

// Persistent form for a batch of plans (one queue, atomic counter).
template <int SPIN, int NCB, bool F32>
__global__ __launch_bounds__(64 * ana_nw(F32, SPIN != 0), 2) void k_legendre_anal_batch(const LegView *__restrict__ views,
                                                                        const BatchAnaItem *__restrict__ items,
                                                                        int nitems, BatchPtrs ptrs, int mode,
                                                                        unsigned *counter)
{
    __shared__ AnaShared<SPIN, NCB, F32> sh;
    __shared__ unsigned sidx;
    for (;;) {
        if (threadIdx.x == 0) sidx = atomicAdd(counter, 1u);
        __syncthreads();
        const unsigned idx = __builtin_amdgcn_readfirstlane(sidx);
        __syncthreads();
        if (idx >= (unsigned)nitems) break;
        const BatchAnaItem bi = items[idx];
        anal_item<SPIN, NCB, F32, ana_tpw<SPIN, NCB>()>(views[bi.plan], bi.m, bi.t0, ptrs.in[bi.plan], ptrs.out[bi.plan], mode, sh);
        __syncthreads();
        if (bi.m2 >= 0) {
            anal_item<SPIN, NCB, F32, ana_tpw<SPIN, NCB>()>(views[bi.plan], bi.m2, bi.t0, ptrs.in[bi.plan], ptrs.out[bi.plan], mode, sh);
            __syncthreads();
        }
    }
}

// Persistent synthesis for a batch of plans: the queue has one segment per
// accelerator die (blocks of consecutive m of a plan on one die, as in the
// plans' own item lists), each with its own counter 64 bytes apart.  A
// wavefront takes items from its die's segment (work groups go to the dies
// round robin), then from the others' until every segment is empty; all lanes
// read the same index, so the whole wavefront moves on and leaves together.
template <int SPIN, int NCB, bool F32>
__global__ __launch_bounds__(64) void k_legendre_synth_batch(const LegView *__restrict__ views,
                                                             const BatchSynItem *__restrict__ items, SynQueues q,
                                                             BatchPtrs ptrs, int flush_chunks, int deriv,
                                                             unsigned *counters)
{
    __shared__ SynShared<SPIN, F32> sh;
    const int die = (int)(blockIdx.x % NUM_XCD);
    int k = 0;
    for (;;) {
        const int d = (die + k) % NUM_XCD;
        const unsigned n = (unsigned)(q.ofs[d + 1] - q.ofs[d]);
        unsigned got = 0;
        if (threadIdx.x == 0) got = atomicAdd(counters + 16 * d, 1u);
        const unsigned idx = __builtin_amdgcn_readfirstlane(got);   // lane 0's value
        if (idx >= n) {
            if (++k == NUM_XCD) break;   // every segment empty
            continue;
        }
        const BatchSynItem bi = items[q.ofs[d] + idx];
        synth_item<SPIN, NCB, F32>(views[bi.plan], WaveItem{bi.m, bi.tile, bi.t0, 0}, ptrs.in[bi.plan],
                                   ptrs.out[bi.plan], flush_chunks, deriv, sh);
        __syncthreads();   // this item's LDS reads are done before the next item's writes
        if (bi.m2 >= 0) {
            synth_item<SPIN, NCB, F32>(views[bi.plan], WaveItem{bi.m2, bi.tile, bi.t0, 0}, ptrs.in[bi.plan],
                                       ptrs.out[bi.plan], flush_chunks, deriv, sh);
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------- vector path
//
// For one or two spin-0 transforms, or one spin transform, most matrix-core
// columns would be empty (2 of 16 for one scalar transform, 4 of 16 for one
// spin transform), so the products run on the vector units instead, with no
// empty columns: every FMA is one of the algorithm's (the loop nests of Sect.
// 3.2, several ring slots per lane).  A lane runs the recursion chains of K
// slots (slots lane + 64 k of its group of 64-slot units; spin: the +s and -s
// chains of each), so that each wave-uniform step coefficient serves all of
// them.  The coefficients of a
// chunk of degrees are loaded with vector loads one chunk ahead, staged in
// LDS and read back as broadcasts.
//   synthesis: per degree, per slot the recursion's two FMAs and per transform
//     two FMAs with f_l a_lm into the slot's even and odd class accumulators;
//     no reduction at all;
//   analysis: per degree, per slot two FMAs per transform with the stationary
//     phases G_t +- G_(pi-t) of the slot, summed over the lane's K slots in
//     registers; every few degrees the 64 lanes' partial sums (8 values) are
//     reduced by halving steps (permlane32/16 swaps, a DPP mirror) to eight
//     partial sums per value, stored to LDS; the output stage adds them and the
//     wavefronts' sums in a fixed order (deterministic, no atomics).

// One step of a chain with the staged coefficients q = (alpha, beta, delta+,
// delta-) of the degree, delta+- = alpha +- beta - 2 (the difference form's
// constant); MINUS: the -s chain of a spin transform (-beta and delta-).
template <bool DIFF, bool MINUS = false>
__device__ __forceinline__ void chain_step(Chain &c, const double4 q)
{
    if (DIFF) {
        const double eps = fma(q.x, c.ms2, MINUS ? q.w : q.z);
        c.aux = fma(eps, c.mu, c.aux);
        c.mu += c.aux;
    } else {
        const double nx = fma(fma(q.x, c.x, MINUS ? -q.y : q.y), c.mu, -c.aux);
        c.aux = c.mu;
        c.mu = nx;
    }
}

// One chunk of LC degrees lc .. lc+LC-1 of the K chains of every lane, in
// groups of G degrees: emit(u, k, mu, d) for each degree offset t = g + u and
// chain k, with mu = mu_l (0 outside [l0, lmax] and while the chain's scale
// k < 0) and d = load(t) (the staged wave-uniform data of the degree: step
// coefficients in .q), then gend(g) at the end of the group.  Only the G
// degrees of a group are unrolled, so the caller's registers are indexed by u
// alone and the compiler cannot keep the mu of the whole chunk alive.
template <int LC, int G, int K, bool DIFF, int NCH, typename Load, typename Emit, typename GroupEnd>
__device__ __forceinline__ void chains_chunk(Chain (&c)[K], bool &slow, int l0, int lc, int lmax, double thr,
                                             double down, Load load, Emit emit, GroupEnd gend)
{
    // K chains; with NCH = 2 chain k is the (k % 2 ? -s : +s) chain of slot k / 2
    static_assert(LC % G == 0, "whole groups");
    if (!slow && lc >= l0 && lc + LC <= lmax) {
        // every degree steps and every chain is at scale 0: no masks
#pragma unroll 1
        for (int g = 0; g < LC; g += G) {
#pragma unroll
            for (int u = 0; u < G; ++u) {
                const auto d = load(g + u);
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    emit(u, k, c[k].mu, d);
                    if (NCH == 2 && (k & 1)) chain_step<DIFF, true>(c[k], d.q);
                    else chain_step<DIFF>(c[k], d.q);
                }
            }
            gend(g);
        }
        return;
    }
    // Masked form: a chain contributes only at scale 0; its scale is checked
    // once per group (between two checks |mu| grows by less than 3^G, far
    // below the headroom above the threshold), so a chain that crosses the
    // threshold inside a group enters at the next group -- the terms left out
    // are below 2^-(S/2) 3^G relative and do not show in double precision.
#pragma unroll 1
    for (int g = 0; g < LC; g += G) {
        double on[K];   // 1 at scale 0, else 0
#pragma unroll
        for (int k = 0; k < K; ++k) on[k] = c[k].k == 0 ? 1.0 : 0.0;
        if (lc + g >= l0 && lc + g + G <= lmax) {
            // the group lies inside [l0, lmax): every degree counts and steps
#pragma unroll
            for (int u = 0; u < G; ++u) {
                const auto d = load(g + u);
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    emit(u, k, c[k].mu * on[k], d);
                    if (NCH == 2 && (k & 1)) chain_step<DIFF, true>(c[k], d.q);
                    else chain_step<DIFF>(c[k], d.q);
                }
            }
        } else {
#pragma unroll
            for (int u = 0; u < G; ++u) {
                const int l = lc + g + u;
                const bool in = l >= l0 && l <= lmax, steps = l >= l0 && l < lmax;
                const auto d = load(g + u);
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    emit(u, k, in ? c[k].mu * on[k] : 0.0, d);
                    if (steps) {
                        if (NCH == 2 && (k & 1)) chain_step<DIFF, true>(c[k], d.q);
                        else chain_step<DIFF>(c[k], d.q);
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const bool up = c[k].k < 0 && fabs(c[k].mu) >= thr;
            c[k].mu = up ? c[k].mu * down : c[k].mu;
            c[k].aux = up ? c[k].aux * down : c[k].aux;
            c[k].k += up ? 1 : 0;
        }
        gend(g);
    }
    bool any = false;
#pragma unroll
    for (int k = 0; k < K; ++k) any = any || c[k].k < 0;
    slow = wave_any(any);
}

// chains of the K slots of this lane (tile[k] < 0: none), the form (difference
// form if any slot of the wave is close to a pole) and the scale flag
template <int K, int NCH = 1>
__device__ __forceinline__ void chains_init(const LegView &v, int m, const int (&tile)[K], int lane,
                                            Chain (&c)[K * NCH], bool &diff, bool &slow)
{
    bool d = false, s = false;
#pragma unroll
    for (int k = 0; k < K * NCH; ++k) {
        const int kt = k / NCH;
        c[k] = chain_init(v, m, tile[kt] >= 0 ? tile[kt] * 64 + lane : v.nslots, k % NCH);
        d = d || c[k].x > DIFF_FORM_COS;
        s = s || c[k].k < 0;
    }
    diff = wave_any(d);
    slow = wave_any(s);
    if (diff)
#pragma unroll
        for (int k = 0; k < K * NCH; ++k) c[k].aux = c[k].mu;
}

constexpr int VSYN_LC = 16;   // degrees per chunk of the vector synthesis

// staged data of one degree of the vector synthesis
template <int J>
struct SynStage {
    double4 q;        // alpha, beta, alpha + beta - 2, 0
    double2 co[J];    // f_l a_lm per transform (zero beyond lmax and for absent transforms)
};

// Work item (m, tile group of K tiles from it.tile, J transforms from t0), one wavefront.
template <int J, int K>
__global__ __launch_bounds__(64) void k_legendre_synth_valu(LegView v, const WaveItem *__restrict__ items,
                                                            const double *__restrict__ alm,
                                                            double *__restrict__ phase)
{
    constexpr int LC = VSYN_LC;
    __shared__ SynStage<J> st[2][LC];
    const WaveItem it = items[blockIdx.x];
    if (it.m < 0) return;
    const int lane = threadIdx.x;
    const int m = it.m, t0 = it.t0, lmax = v.lmax;
    const int l0 = m;   // spin 0: l0 + m even, chunks start at l0 (class of offset t = t & 1)
    const double4 *coef = v.coef + v.coef_ofs[m];
    const double *flm = v.fl + v.coef_ofs[m];
    const int64_t mbase = (int64_t)m * (2 * (int64_t)lmax + 1 - m) / 2;
    const double thr = ldexp(1.0, v.thresh_bits), down = ldexp(1.0, -v.rescale_bits);
    int tile[K];
#pragma unroll
    for (int k = 0; k < K; ++k) tile[k] = it.tile + k < v.ntiles ? it.tile + k : -1;
    Chain cs[K];
    bool diff, slow;
    chains_init<K>(v, m, tile, lane, cs, diff, slow);

    // lane t < LC fetches degree lc + t of a chunk (clamped addresses; masked
    // when staged)
    double4 nq;
    double nf;
    double2 na[J];
    auto fetch = [&](int lc) {
        const int l = lc + (lane % LC);
        const int lcl = l > lmax ? lmax : l;
        nq = coef[lcl];
        nf = flm[lcl];
#pragma unroll
        for (int tr = 0; tr < J; ++tr) {
            const double2 *ar = reinterpret_cast<const double2 *>(alm) +
                                (int64_t)(t0 + tr < v.ntrans ? t0 + tr : 0) * v.nalm + mbase;
            na[tr] = ar[lcl];
        }
    };
    auto stage = [&](int buf, int lc) {
        if (lane < LC) {
            const int l = lc + lane;
            SynStage<J> e;
            e.q = (l < lmax) ? double4{nq.x, nq.y, nq.z, 0.0} : double4{0, 0, 0, 0};
            const double f = l <= lmax ? nf : 0.0;
#pragma unroll
            for (int tr = 0; tr < J; ++tr)
                e.co[tr] = (t0 + tr < v.ntrans) ? make_double2(na[tr].x * f, m == 0 ? 0.0 : na[tr].y * f)
                                                : make_double2(0.0, 0.0);
            st[buf][lane] = e;
        }
    };

    double2 acc[2][K][J];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int tr = 0; tr < J; ++tr) acc[p][k][tr] = make_double2(0.0, 0.0);
    fetch(l0);
    stage(0, l0);
    wave_sync();
    auto run = [&](auto form) {
        constexpr bool DIFF = decltype(form)::value;
        int chunk = 0;
        for (int lc = l0; lc <= lmax; lc += LC, ++chunk) {
            const int buf = chunk & 1;
            const bool more = lc + LC <= lmax;
            if (more) fetch(lc + LC);
            chains_chunk<LC, 4, K, DIFF, 1>(
                cs, slow, l0, lc, lmax, thr, down, [&](int t) -> const SynStage<J> & { return st[buf][t]; },
                [&](int u, int k, double mu, const SynStage<J> &d) {
#pragma unroll
                    for (int tr = 0; tr < J; ++tr) {   // class of the degree: u & 1 (groups of four)
                        acc[u & 1][k][tr].x = fma(mu, d.co[tr].x, acc[u & 1][k][tr].x);
                        acc[u & 1][k][tr].y = fma(mu, d.co[tr].y, acc[u & 1][k][tr].y);
                    }
                },
                [](int) {});
            wave_sync();   // this chunk's reads of the other buffer are issued
            if (more) stage(buf ^ 1, lc + LC);
            wave_sync();
        }
    };
    if (diff) run(std::true_type{});
    else run(std::false_type{});

    // ring t = A0 + A1, ring pi - t = A0 - A1
    double2 *ph = reinterpret_cast<double2 *>(phase);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if (tile[k] < 0) continue;
        const int slot = tile[k] * 64 + lane;
        if (slot >= v.nslots) continue;
        const int yn = v.slot_yn[slot], ys = v.slot_ys[slot];
#pragma unroll
        for (int tr = 0; tr < J; ++tr) {
            const int t = t0 + tr;
            if (t >= v.ntrans) break;
            const int64_t rowbase = (int64_t)t * v.nrings;
            const double2 a0 = acc[0][k][tr], a1 = acc[1][k][tr];
            if (yn >= 0) ph[(rowbase + yn) * (v.mmax + 1) + m] = make_double2(a0.x + a1.x, a0.y + a1.y);
            if (ys >= 0) ph[(rowbase + ys) * (v.mmax + 1) + m] = make_double2(a0.x - a1.x, a0.y - a1.y);
        }
    }
}

// staged data of one degree of the spin vector synthesis
template <int J>
struct SynStageS {
    double4 q;        // step coefficients: alpha, beta, delta+, delta- (the -s chain takes -beta, delta-)
    double4 co[J];    // c f_l (E_re, E_im, B_re, B_im) per transform, c = 1/2 (zero outside [l0, lmax])
};

// Spin s > 0, work item (m, K units of 64 slots from slot 32 it.tile, J
// transforms): a lane runs the +s and -s chains of K ring slots.  Per degree and slot W = -(mu_+ + mu_-) and
// X = mu_+ - mu_- (the -s chain carries (-1)^s), and per transform
//   Q_re += W E_re + X B_im,   Q_im += W E_im - X B_re,
//   U_re += W B_re - X E_im,   U_im += W B_im + X E_re
// (E, B times c f_l), the W terms into the class of the degree's l + m parity
// and the X terms into the other (their mirror-ring signs are opposite); ring
// t gets A0 + A1, ring pi - t gets (-1)^s (A0 - A1).  Derivative synthesis
// (spin-1 plan): one input component per transform, E = sqrt(l (l + 1)) a_lm
// and B = 0.
template <int J, int K>
__global__ __launch_bounds__(64) void k_legendre_synth_valu_s(LegView v, const WaveItem *__restrict__ items,
                                                              const double *__restrict__ alm,
                                                              double *__restrict__ phase, int deriv)
{
    constexpr int LC = VSYN_LC;
    __shared__ SynStageS<J> st[2][LC];
    const WaveItem it = items[blockIdx.x];
    if (it.m < 0) return;
    const int lane = threadIdx.x;
    const int m = it.m, t0 = it.t0, lmax = v.lmax;
    const int l0 = v.spin > m ? v.spin : m;
    const int lstart = l0 - ((l0 + m) & 1);   // l + m even at every chunk start: class of offset t = t & 1
    const double sig = (v.spin & 1) ? -1.0 : 1.0;
    const double4 *coef = v.coef + v.coef_ofs[m];
    const double *flm = v.fl + v.coef_ofs[m];
    const int64_t mbase = (int64_t)m * (2 * (int64_t)lmax + 1 - m) / 2;
    const double thr = ldexp(1.0, v.thresh_bits), down = ldexp(1.0, -v.rescale_bits);
    // units of 64 consecutive slots (two 32-slot tiles; items start at even tiles)
    int tile[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int u = (it.tile >> 1) + k;
        tile[k] = u * 64 < v.nslots ? u : -1;
    }
    Chain cs[2 * K];   // chain 2k: +s of slot k, 2k + 1: -s
    bool diff, slow;
    chains_init<K, 2>(v, m, tile, lane, cs, diff, slow);
    const int ncin = deriv ? 1 : 2;   // input components per transform

    // lane t < LC fetches degree lc + t of a chunk (clamped addresses; masked when staged)
    double4 nq;
    double nf, nd = 1.0;
    double2 nE[J], nB[J];
    auto fetch = [&](int lc) {
        const int l = lc + (lane % LC);
        const int lcl = l < l0 ? l0 : (l > lmax ? lmax : l);
        nq = coef[lcl];
        nf = flm[lcl];
        if (deriv) nd = v.dfac[lcl];
#pragma unroll
        for (int tr = 0; tr < J; ++tr) {
            const int t = t0 + tr < v.ntrans ? t0 + tr : 0;
            const double2 *er = reinterpret_cast<const double2 *>(alm) + (int64_t)t * ncin * v.nalm + mbase;
            nE[tr] = er[lcl];
            nB[tr] = deriv ? make_double2(0.0, 0.0) : er[v.nalm + lcl];
        }
    };
    auto stage = [&](int buf, int lc) {
        if (lane < LC) {
            const int l = lc + lane;
            SynStageS<J> e;
            e.q = (l >= l0 && l < lmax) ? nq : double4{0, 0, 0, 0};
            const double f = (l >= l0 && l <= lmax) ? 0.5 * nf * nd : 0.0;
            const double fi = m == 0 ? 0.0 : f;   // Im a_l0 takes no part
#pragma unroll
            for (int tr = 0; tr < J; ++tr)
                e.co[tr] = (t0 + tr < v.ntrans) ? double4{nE[tr].x * f, nE[tr].y * fi, nB[tr].x * f, nB[tr].y * fi}
                                                : double4{0, 0, 0, 0};
            st[buf][lane] = e;
        }
    };

    double4 acc[2][K][J];   // class, slot, transform: (Q_re, Q_im, U_re, U_im)
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int tr = 0; tr < J; ++tr) acc[p][k][tr] = double4{0, 0, 0, 0};
    fetch(lstart);
    stage(0, lstart);
    wave_sync();
    double mu_p[K];   // the +s chain's value of the current degree (emitted before the -s chain)
    auto run = [&](auto form) {
        constexpr bool DIFF = decltype(form)::value;
        int chunk = 0;
        for (int lc = lstart; lc <= lmax; lc += LC, ++chunk) {
            const int buf = chunk & 1;
            const bool more = lc + LC <= lmax;
            if (more) fetch(lc + LC);
            chains_chunk<LC, 4, 2 * K, DIFF, 2>(
                cs, slow, l0, lc, lmax, thr, down, [&](int t) -> const SynStageS<J> & { return st[buf][t]; },
                [&](int u, int kc, double mu, const SynStageS<J> &d) {
                    const int k = kc >> 1;
                    if (!(kc & 1)) {
                        mu_p[k] = mu;
                        return;
                    }
                    const double w = -(mu_p[k] + mu), x = mu_p[k] - mu;
                    const int cw = u & 1, cx = cw ^ 1;   // groups of four degrees from an even offset
#pragma unroll
                    for (int tr = 0; tr < J; ++tr) {
                        const double4 c = d.co[tr];
                        double4 &aw = acc[cw][k][tr];
                        double4 &ax = acc[cx][k][tr];
                        aw.x = fma(w, c.x, aw.x);
                        aw.y = fma(w, c.y, aw.y);
                        aw.z = fma(w, c.z, aw.z);
                        aw.w = fma(w, c.w, aw.w);
                        ax.x = fma(x, c.w, ax.x);
                        ax.y = fma(-x, c.z, ax.y);
                        ax.z = fma(-x, c.y, ax.z);
                        ax.w = fma(x, c.x, ax.w);
                    }
                },
                [](int) {});
            wave_sync();   // this chunk's reads of the other buffer are issued
            if (more) stage(buf ^ 1, lc + LC);
            wave_sync();
        }
    };
    if (diff) run(std::true_type{});
    else run(std::false_type{});

    // ring t = A0 + A1, ring pi - t = (-1)^s (A0 - A1); component 0: Q, 1: U
    double2 *ph = reinterpret_cast<double2 *>(phase);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if (tile[k] < 0) continue;
        const int slot = tile[k] * 64 + lane;
        if (slot >= v.nslots) continue;
        const int yn = v.slot_yn[slot], ys = v.slot_ys[slot];
#pragma unroll
        for (int tr = 0; tr < J; ++tr) {
            const int t = t0 + tr;
            if (t >= v.ntrans) break;
            const double4 a0 = acc[0][k][tr], a1 = acc[1][k][tr];
            const int64_t rq = (int64_t)t * 2 * v.nrings, ru = rq + v.nrings;
            if (yn >= 0) {
                ph[(rq + yn) * (v.mmax + 1) + m] = make_double2(a0.x + a1.x, a0.y + a1.y);
                ph[(ru + yn) * (v.mmax + 1) + m] = make_double2(a0.z + a1.z, a0.w + a1.w);
            }
            if (ys >= 0) {
                ph[(rq + ys) * (v.mmax + 1) + m] = make_double2(sig * (a0.x - a1.x), sig * (a0.y - a1.y));
                ph[(ru + ys) * (v.mmax + 1) + m] = make_double2(sig * (a0.z - a1.z), sig * (a0.w - a1.w));
            }
        }
    }
}

// ---- butterfly reduction of 32 values over the 64 lanes of a wavefront

__device__ __forceinline__ double dpp_f64(double x, int ctrl)
{
    const long long b = __double_as_longlong(x);
    int lo = (int)(b & 0xffffffffLL), hi = (int)(b >> 32);
    switch (ctrl) {   // the control must be a constant of the builtin
    case 0x140:
        lo = __builtin_amdgcn_mov_dpp(lo, 0x140, 0xF, 0xF, false);
        hi = __builtin_amdgcn_mov_dpp(hi, 0x140, 0xF, 0xF, false);
        break;
    case 0x141:
        lo = __builtin_amdgcn_mov_dpp(lo, 0x141, 0xF, 0xF, false);
        hi = __builtin_amdgcn_mov_dpp(hi, 0x141, 0xF, 0xF, false);
        break;
    case 0x4E:
        lo = __builtin_amdgcn_mov_dpp(lo, 0x4E, 0xF, 0xF, false);
        hi = __builtin_amdgcn_mov_dpp(hi, 0x4E, 0xF, 0xF, false);
        break;
    default:
        lo = __builtin_amdgcn_mov_dpp(lo, 0xB1, 0xF, 0xF, false);
        hi = __builtin_amdgcn_mov_dpp(hi, 0xB1, 0xF, 0xF, false);
        break;
    }
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Lanes L < 32 get a_L + a_(L+32), lanes L >= 32 get b_(L-32) + b_L.
__device__ __forceinline__ double swap32_add(double a, double b)
{
    const long long ia = __double_as_longlong(a), ib = __double_as_longlong(b);
    const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)(ia & 0xffffffffLL), (unsigned)(ib & 0xffffffffLL),
                                                     false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(ia >> 32), (unsigned)(ib >> 32), false, false);
    const double r0 = __longlong_as_double(((long long)hi[0] << 32) | lo[0]);
    const double r1 = __longlong_as_double(((long long)hi[1] << 32) | lo[1]);
    return r0 + r1;
}

// The same within each half of 32 lanes: bit 4 of the lane clear: a_L + a_(L+16),
// set: b_(L-16) + b_L.
__device__ __forceinline__ double swap16_add(double a, double b)
{
    const long long ia = __double_as_longlong(a), ib = __double_as_longlong(b);
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)(ia & 0xffffffffLL), (unsigned)(ib & 0xffffffffLL),
                                                     false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(ia >> 32), (unsigned)(ib >> 32), false, false);
    const double r0 = __longlong_as_double(((long long)hi[0] << 32) | lo[0]);
    const double r1 = __longlong_as_double(((long long)hi[1] << 32) | lo[1]);
    return r0 + r1;
}

// One halving step with a DPP partner that differs from the lane in bit `bit`
// (and possibly lower bits): the lane keeps a (bit clear) or b (bit set) and
// adds the partner's copy of the same value.
template <int CTRL>
__device__ __forceinline__ double dpp_half_add(double a, double b, bool upper)
{
    const double keep = upper ? b : a, send = upper ? a : b;
    return keep + dpp_f64(send, CTRL);
}

// x[0..7] of every lane -> every lane L holds a partial sum of x[L >> 3] over
// 8 of the 64 lanes (halving steps over lane bits 5, 4 and 3); the 8 lanes of
// an octet (lane bits 0-2) hold the 8 partial sums of the same value, whose
// total the caller forms later (once per output element rather than per group).
__device__ __forceinline__ double wave_reduce8_octet(double (&x)[8], int lane)
{
#pragma unroll
    for (int i = 0; i < 4; ++i) x[i] = swap32_add(x[i], x[i + 4]);   // index i + 4 b5
#pragma unroll
    for (int i = 0; i < 2; ++i) x[i] = swap16_add(x[i], x[i + 2]);   // + 2 b4
    return dpp_half_add<0x140>(x[0], x[1], lane & 8);                // row mirror: + b3
}

constexpr int ANV_NW = 4;   // wavefronts per analysis work group (vector path)
constexpr int ANV_CH = 64;  // degrees x transforms per chunk of the vector analysis

// Work group = one m and J transforms from blockIdx.y J; the m's active tiles
// are dealt K per wavefront, NW K per pass, and every pass after the first
// adds into the m's a_lm row.
template <int J, int K>
__global__ __launch_bounds__(64 * ANV_NW) void k_legendre_anal_valu(LegView v, const int *__restrict__ mlist,
                                                                   const double *__restrict__ phase,
                                                                   double *__restrict__ alm, int mode)
{
    constexpr int LC = ANV_CH / J;       // degrees per chunk (one barrier and output round each)
    constexpr int NV = LC * J * 2;       // output values of a chunk
    constexpr int GD = 4 / J;            // degrees per reduction group: 8 values
    static_assert(GD * J * 2 == 8 && LC % GD == 0 && LC <= 64, "value layout");
    constexpr int OPT = (NV + 63) / 64;  // output values per thread (at least one wavefront)
    constexpr int NWM = J == 1 ? 2 : ANV_NW;   // wavefronts per work group at most (launcher)
    // per wavefront, value and octet lane: the octet's 8 partial sums of the value
    __shared__ double part[2][NWM][NV * 8];
    __shared__ double4 stq[2][LC];
    const int m = mlist[blockIdx.x];
    const int t0 = (int)blockIdx.y * J;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int nw = (int)(blockDim.x >> 6);
    const int lmax = v.lmax, l0 = m;
    const double4 *coef = v.coef + v.coef_ofs[m];
    const double *flm = v.fl + v.coef_ofs[m];
    const int64_t mbase = (int64_t)m * (2 * (int64_t)lmax + 1 - m) / 2;
    const double thr = ldexp(1.0, v.thresh_bits), down = ldexp(1.0, -v.rescale_bits);
    const bool grad = mode & ANA_MODE_GRAD;
    const double2 *G = reinterpret_cast<const double2 *>(phase);
    double2 *out = reinterpret_cast<double2 *>(alm);
    // output elements e = tid + j blockDim of a chunk: value index e = (t J + tr) 2 + re/im
    const double fac = (grad && m > 0) ? 2.0 : 1.0;   // fac_m of the real-field gradient
    auto orow = [&](int e) {   // element e of degree lc + t lives at orow(e)[2 (lc + t)]
        const int tr = (e >> 1) % J;
        return reinterpret_cast<double *>(out + (int64_t)(t0 + tr) * v.nalm + mbase) + (e & 1);
    };
    auto o_valid = [&](int e) { return e < NV && t0 + (e >> 1) % J < v.ntrans; };

    int ntiles_act = 0;
    for (int t = 0; t < v.ntiles; ++t) ntiles_act += v.tile_mlim[t] >= m;
    int tscan = 0, tcount = 0, cidx = 0;
    bool first = true;
    while (tcount < ntiles_act || first) {
        // this pass's tiles of this wavefront (the m's active tiles in order, K each)
        int tile[K];
#pragma unroll
        for (int k = 0; k < K; ++k) tile[k] = -1;
        {
            int n = 0;
            for (; tscan < v.ntiles && n < nw * K; ++tscan) {
                if (v.tile_mlim[tscan] < m) continue;
#pragma unroll
                for (int k = 0; k < K; ++k)
                    if (n == wave * K + k) tile[k] = tscan;
                ++n;
            }
            tcount += n;
        }
        const bool active = tile[0] >= 0;   // tiles are dealt to k = 0 first
        Chain cs[K];
        bool diff, slow;
        chains_init<K>(v, m, tile, lane, cs, diff, slow);
        // stationary phases G_t +- G_(pi-t) of the lane's slots (zero for missing
        // rings and slots, absent transforms)
        double2 g[K][2][J];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int slot = tile[k] >= 0 ? tile[k] * 64 + lane : v.nslots;
            const bool ok = slot < v.nslots;
            const int yn = ok ? v.slot_yn[slot] : -1, ys = ok ? v.slot_ys[slot] : -1;
#pragma unroll
            for (int tr = 0; tr < J; ++tr) {
                const bool tok = t0 + tr < v.ntrans;
                const int64_t rowbase = (int64_t)(tok ? t0 + tr : 0) * v.nrings;
                const double2 gn0 = G[(rowbase + (yn >= 0 ? yn : 0)) * (v.mmax + 1) + m];
                const double2 gs0 = G[(rowbase + (ys >= 0 ? ys : 0)) * (v.mmax + 1) + m];
                const double2 gn = (tok && yn >= 0) ? gn0 : make_double2(0.0, 0.0);
                const double2 gs = (tok && ys >= 0) ? gs0 : make_double2(0.0, 0.0);
                g[k][0][tr] = make_double2(gn.x + gs.x, gn.y + gs.y);
                g[k][1][tr] = make_double2(gn.x - gs.x, gn.y - gs.y);
            }
        }
        // staged step coefficients (alpha, beta, alpha + beta - 2, f_l) of a
        // chunk, shared by the wavefronts: thread t < LC of wavefront 0 fetches
        // degree lc + t one chunk ahead and stages it after its own products
        double4 nq = double4{0, 0, 0, 0};
        double nf = 0.0;
        auto fetch = [&](int lc) {
            if (wave == 0) {
                const int l = lc + (lane % LC);
                const int lcl = l > lmax ? lmax : l;
                nq = coef[lcl];
                nf = flm[lcl];
            }
        };
        auto stage = [&](int buf, int lc) {
            if (wave == 0 && lane < LC) {
                const int l = lc + lane;
                stq[buf][lane] = l < lmax ? double4{nq.x, nq.y, nq.z, nf} : double4{0, 0, 0, l <= lmax ? nf : 0.0};
            }
        };
        fetch(l0);
        stage(cidx & 1, l0);
        __syncthreads();
        for (int lc = l0; lc <= lmax; lc += LC, ++cidx) {
            const int buf = cidx & 1;
            const bool more = lc + LC <= lmax;
            if (more) fetch(lc + LC);
            // the earlier passes' sums of this thread's output elements, in flight
            // during the chunk's arithmetic
            double prev[OPT];
#pragma unroll
            for (int j = 0; j < OPT; ++j) {
                const int e = tid + j * (int)blockDim.x;
                const int ol = lc + (e >> 1) / J;
                prev[j] = (!first && o_valid(e) && ol <= lmax) ? orow(e)[2 * (int64_t)ol] : 0.0;
            }
            // value index within a group: (u J + tr) 2 + re/im; over the chunk:
            // that + 8 (group offset / GD), i.e. (t J + tr) 2 + re/im
            double x[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) x[i] = 0.0;
            struct AnaD {
                double4 q;
            };
            auto load = [&](int t) { return AnaD{stq[buf][t]}; };
            auto emit = [&](int u, int k, double mu, const AnaD &) {
#pragma unroll
                for (int tr = 0; tr < J; ++tr) {
                    const double2 gv = g[k][u & 1][tr];   // GD even: class of the degree = u & 1
                    x[(u * J + tr) * 2] = fma(mu, gv.x, x[(u * J + tr) * 2]);
                    x[(u * J + tr) * 2 + 1] = fma(mu, gv.y, x[(u * J + tr) * 2 + 1]);
                }
            };
            auto gend = [&](int g0) {
                // lane L: partial sum of value (g0 / GD) 8 + (L >> 3), slot L & 7
                part[buf][wave][(g0 / GD) * 64 + lane] = wave_reduce8_octet(x, lane);
#pragma unroll
                for (int i = 0; i < 8; ++i) x[i] = 0.0;
            };
            if (active) {
                if (diff) chains_chunk<LC, GD, K, true, 1>(cs, slow, l0, lc, lmax, thr, down, load, emit, gend);
                else chains_chunk<LC, GD, K, false, 1>(cs, slow, l0, lc, lmax, thr, down, load, emit, gend);
            } else {
                for (int e = lane; e < NV * 8; e += 64) part[buf][wave][e] = 0.0;
            }
            if (more) stage(buf ^ 1, lc + LC);
            __syncthreads();
#pragma unroll
            for (int j = 0; j < OPT; ++j) {
                const int e = tid + j * (int)blockDim.x;
                const int t = (e >> 1) / J, ol = lc + t;
                if (!o_valid(e) || ol > lmax) continue;
                double sum = 0.0;   // wavefronts and octet slots in a fixed order
                for (int w = 0; w < nw; ++w) {
                    const double *pw = &part[buf][w][e * 8];
#pragma unroll
                    for (int q = 0; q < 8; ++q) sum += pw[q];
                }
                double val = sum * stq[buf][t].w * fac;
                if (m == 0 && (e & 1)) val = 0.0;
                orow(e)[2 * (int64_t)ol] = first ? val : prev[j] + val;
            }
            // part[buf] and stq[buf] are written again in the next chunk but one,
            // after the next barrier
        }
        first = false;
    }
}

// Spin s > 0 analysis (transposed column maps of the spin synthesis): per
// degree and slot W = -(mu_+ + mu_-), X = mu_+ - mu_-, and per transform
//   E_re += W GW_Qre + X GX_Uim,   E_im += W GW_Qim - X GX_Ure,
//   B_re += W GW_Ure - X GX_Qim,   B_im += W GW_Uim + X GX_Qre,
// with GW the stationary phases of the degree's class (G_t + (-1)^s G_(pi-t) at
// l + m even, G_t - (-1)^s G_(pi-t) at odd) and GX those of the other class;
// the sums times c f_l (c = 1/2).  Work groups, passes and the butterfly as in
// the spin-0 kernel (4 values per degree and transform), the slots dealt in
// units of 64 (two 32-slot tiles).  Adjoint of the derivative synthesis: E
// alone, times sqrt(l (l + 1)), one output component per transform.
template <int J, int K>
__global__ __launch_bounds__(64 * ANV_NW) void k_legendre_anal_valu_s(LegView v, const int *__restrict__ mlist,
                                                                     const double *__restrict__ phase,
                                                                     double *__restrict__ alm, int mode)
{
    constexpr int LC = ANV_CH / (2 * J);   // degrees per chunk
    constexpr int NV = LC * J * 4;         // output values of a chunk: (E, B) x (re, im) per transform
    constexpr int GD = 2;                  // degrees per reduction group: 8 values (one transform)
    static_assert(J == 1 && LC % GD == 0 && LC <= 64, "value layout");
    constexpr int OPT = (NV + 63) / 64;
    constexpr int NWM = 2;   // wavefronts per work group at most (launcher)
    __shared__ double part[2][NWM][NV * 8];   // octet partial sums per value
    __shared__ double4 stq[2][LC];
    __shared__ double stf[2][LC];
    const int m = mlist[blockIdx.x];
    const int t0 = (int)blockIdx.y * J;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int nw = (int)(blockDim.x >> 6);
    const int lmax = v.lmax;
    const int l0 = v.spin > m ? v.spin : m;
    const int lstart = l0 - ((l0 + m) & 1);   // l + m even at every chunk start
    const double sig = (v.spin & 1) ? -1.0 : 1.0;
    const double4 *coef = v.coef + v.coef_ofs[m];
    const double *flm = v.fl + v.coef_ofs[m];
    const int64_t mbase = (int64_t)m * (2 * (int64_t)lmax + 1 - m) / 2;
    const double thr = ldexp(1.0, v.thresh_bits), down = ldexp(1.0, -v.rescale_bits);
    const bool grad = mode & ANA_MODE_GRAD;
    const bool deriv = mode & ANA_MODE_DERIV;
    const double2 *G = reinterpret_cast<const double2 *>(phase);
    double2 *out = reinterpret_cast<double2 *>(alm);
    const double fac = (grad && m > 0) ? 2.0 : 1.0;   // fac_m of the real-field gradient
    // output element e: value index ((t J + tr) 2 + comp) 2 + re/im, comp 0 = E, 1 = B
    const int ncout = deriv ? 1 : 2;
    auto orow = [&](int e) {
        const int tr = (e >> 2) % J, comp = (e >> 1) & 1;
        return reinterpret_cast<double *>(out + ((int64_t)(t0 + tr) * ncout + comp) * v.nalm + mbase) + (e & 1);
    };
    auto o_valid = [&](int e) {
        return e < NV && t0 + (e >> 2) % J < v.ntrans && !(deriv && ((e >> 1) & 1));
    };

    // degrees m .. l0 - 1 (spin s > m) are zero by convention
    for (int e = tid; e < (l0 - m) * J * 4; e += (int)blockDim.x) {
        const int l = m + e / (J * 4), r = e % (J * 4);
        if (o_valid(r)) orow(r)[2 * (int64_t)l] = 0.0;
    }

    // units of 64 slots: active when one of their two tiles is
    const int nunits = (v.nslots + 63) / 64;
    auto unit_act = [&](int u) {
        return v.tile_mlim[2 * u] >= m || (2 * u + 1 < v.ntiles && v.tile_mlim[2 * u + 1] >= m);
    };
    int ntiles_act = 0;
    for (int u = 0; u < nunits; ++u) ntiles_act += unit_act(u);
    int tscan = 0, tcount = 0, cidx = 0;
    bool first = true;
    while (tcount < ntiles_act || first) {
        int tile[K];
#pragma unroll
        for (int k = 0; k < K; ++k) tile[k] = -1;
        {
            int n = 0;
            for (; tscan < nunits && n < nw * K; ++tscan) {
                if (!unit_act(tscan)) continue;
#pragma unroll
                for (int k = 0; k < K; ++k)
                    if (n == wave * K + k) tile[k] = tscan;
                ++n;
            }
            tcount += n;
        }
        const bool active = tile[0] >= 0;
        Chain cs[2 * K];
        bool diff, slow;
        chains_init<K, 2>(v, m, tile, lane, cs, diff, slow);
        // stationary phases (Q_re, Q_im, U_re, U_im) of the lane's slots per class
        double4 g[K][2][J];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int slot = tile[k] >= 0 ? tile[k] * 64 + lane : v.nslots;
            const bool ok = slot < v.nslots;
            const int yn = ok ? v.slot_yn[slot] : -1, ys = ok ? v.slot_ys[slot] : -1;
#pragma unroll
            for (int tr = 0; tr < J; ++tr) {
                const bool tok = t0 + tr < v.ntrans;
                const int64_t rq = (int64_t)(tok ? t0 + tr : 0) * 2 * v.nrings, ru = rq + v.nrings;
                const int yn0 = yn >= 0 ? yn : 0, ys0 = ys >= 0 ? ys : 0;
                const double2 qn0 = G[(rq + yn0) * (v.mmax + 1) + m], un0 = G[(ru + yn0) * (v.mmax + 1) + m];
                const double2 qs0 = G[(rq + ys0) * (v.mmax + 1) + m], us0 = G[(ru + ys0) * (v.mmax + 1) + m];
                const bool nok = tok && yn >= 0, sok = tok && ys >= 0;
                const double2 qn = nok ? qn0 : make_double2(0.0, 0.0), un = nok ? un0 : make_double2(0.0, 0.0);
                const double2 qs = sok ? make_double2(sig * qs0.x, sig * qs0.y) : make_double2(0.0, 0.0);
                const double2 us = sok ? make_double2(sig * us0.x, sig * us0.y) : make_double2(0.0, 0.0);
                g[k][0][tr] = double4{qn.x + qs.x, qn.y + qs.y, un.x + us.x, un.y + us.y};
                g[k][1][tr] = double4{qn.x - qs.x, qn.y - qs.y, un.x - us.x, un.y - us.y};
            }
        }
        double4 nq = double4{0, 0, 0, 0};
        double nf = 0.0;
        auto fetch = [&](int lc) {
            if (wave == 0) {
                const int l = lc + (lane % LC);
                const int lcl = l < l0 ? l0 : (l > lmax ? lmax : l);
                nq = coef[lcl];
                nf = flm[lcl] * (deriv ? v.dfac[lcl] : 1.0);
            }
        };
        auto stage = [&](int buf, int lc) {
            if (wave == 0 && lane < LC) {
                const int l = lc + lane;
                stq[buf][lane] = (l >= l0 && l < lmax) ? nq : double4{0, 0, 0, 0};
                stf[buf][lane] = (l >= l0 && l <= lmax) ? 0.5 * nf : 0.0;
            }
        };
        fetch(lstart);
        stage(cidx & 1, lstart);
        __syncthreads();
        for (int lc = lstart; lc <= lmax; lc += LC, ++cidx) {
            const int buf = cidx & 1;
            const bool more = lc + LC <= lmax;
            if (more) fetch(lc + LC);
            double prev[OPT];
#pragma unroll
            for (int j = 0; j < OPT; ++j) {
                const int e = tid + j * (int)blockDim.x;
                const int ol = lc + (e >> 2) / J;
                prev[j] = (!first && o_valid(e) && ol <= lmax) ? orow(e)[2 * (int64_t)ol] : 0.0;
            }
            // value index within a group: ((u J + tr) 2 + comp) 2 + re/im
            double x[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) x[i] = 0.0;
            double mu_p[K];
            struct AnaD {
                double4 q;
            };
            auto load = [&](int t) { return AnaD{stq[buf][t]}; };
            auto emit = [&](int u, int kc, double mu, const AnaD &) {
                const int k = kc >> 1;
                if (!(kc & 1)) {
                    mu_p[k] = mu;
                    return;
                }
                const double w = -(mu_p[k] + mu), xx = mu_p[k] - mu;
                const int cw = u & 1, cx = cw ^ 1;   // groups of two degrees from an even offset
#pragma unroll
                for (int tr = 0; tr < J; ++tr) {
                    const double4 gw = g[k][cw][tr], gx = g[k][cx][tr];
                    double *o = x + (u * J + tr) * 4;
                    o[0] = fma(w, gw.x, fma(xx, gx.w, o[0]));    // E_re
                    o[1] = fma(w, gw.y, fma(-xx, gx.z, o[1]));   // E_im
                    o[2] = fma(w, gw.z, fma(-xx, gx.y, o[2]));   // B_re
                    o[3] = fma(w, gw.w, fma(xx, gx.x, o[3]));    // B_im
                }
            };
            auto gend = [&](int g0) {
                // lane L: partial sum of value (g0 / GD) 8 + (L >> 3), slot L & 7
                part[buf][wave][(g0 / GD) * 64 + lane] = wave_reduce8_octet(x, lane);
#pragma unroll
                for (int i = 0; i < 8; ++i) x[i] = 0.0;
            };
            if (active) {
                if (diff) chains_chunk<LC, GD, 2 * K, true, 2>(cs, slow, l0, lc, lmax, thr, down, load, emit, gend);
                else chains_chunk<LC, GD, 2 * K, false, 2>(cs, slow, l0, lc, lmax, thr, down, load, emit, gend);
            } else {
                for (int e = lane; e < NV * 8; e += 64) part[buf][wave][e] = 0.0;
            }
            if (more) stage(buf ^ 1, lc + LC);
            __syncthreads();
#pragma unroll
            for (int j = 0; j < OPT; ++j) {
                const int e = tid + j * (int)blockDim.x;
                const int t = (e >> 2) / J, ol = lc + t;
                if (!o_valid(e) || ol > lmax || ol < m) continue;
                double sum = 0.0;   // wavefronts and octet slots in a fixed order
                for (int w = 0; w < nw; ++w) {
                    const double *pw = &part[buf][w][e * 8];
#pragma unroll
                    for (int q = 0; q < 8; ++q) sum += pw[q];
                }
                double val = sum * stf[buf][t] * fac;
                if (m == 0 && (e & 1)) val = 0.0;
                orow(e)[2 * (int64_t)ol] = first ? val : prev[j] + val;
            }
        }
        first = false;
    }
}

__global__ void k_reset_counter(unsigned *counter)

{
    if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0u;
}

// n counters `stride` apart (one work group of at least n threads)
__global__ void k_reset_counters(unsigned *counter, int n, int stride)
{
    if ((int)threadIdx.x < n) counter[threadIdx.x * stride] = 0u;
}

// ---------------------------------------------------------------- launchers

// column blocks (16 columns each) per analysis work group: bounded so that
// the stationary phases stay in registers at two wavefronts per SIMD
int anal_ncb(int spin, int ntrans)
{
    const int cols = ntrans * (spin ? 4 : 2);
    int ncb = (cols + 15) / 16;
    return ncb > 2 ? 2 : ncb;
}

int anal_tpw_built(int spin, int ncb) { return spin ? ana_tpw<2, 1>() : (ncb == 2 ? ana_tpw<0, 2>() : ana_tpw<0, 1>()); }

// default column blocks per synthesis wavefront (the autotuner may change it)
int synth_ncb_default(int spin, int ntrans, int precision)
{
    (void)precision;
    if (spin == 0) return 1;      // 64-slot tiles: two column blocks would need 1 wavefront/SIMD
    const int cols = ntrans * 4;
    return cols > 16 ? 2 : 1;
}

template <int SPIN, int NCB, bool F32>
static void launch_synth_t(const Plan &p, const LegView &v, const double *alm, double *phase,
                           int deriv, hipStream_t s)
{
    hipLaunchKernelGGL((k_legendre_synth<SPIN, NCB, F32>), dim3((unsigned)p.synth_items.size()), dim3(64),
                       0, s, v, p.d_synth_items, alm, phase, p.flush_chunks, deriv);
}

template <int SPIN, int NCB, bool F32>
static void launch_anal_t(const Plan &p, const LegView &v, const double *phase, double *alm,
                          int mode, hipStream_t s)
{
    const int jpg = NCB * 16 / (SPIN ? 4 : 2);
    dim3 grid((unsigned)(p.mmax + 1), (unsigned)((p.ntrans + jpg - 1) / jpg));
    hipLaunchKernelGGL((k_legendre_anal<SPIN, NCB, F32>), grid, dim3(64 * ana_nw(F32, SPIN != 0)), 0, s, v,
                       p.d_anal_ms, phase, alm, jpg, mode);
}

template <bool F32>
static int dispatch_synth(const Plan &p, const LegView &v, const double *alm, double *phase,
                          int deriv, hipStream_t s)
{
    const int ncb = p.tune.synth_ncb;
    if (p.spin == 0) {
        if (ncb == 1) launch_synth_t<0, 1, F32>(p, v, alm, phase, 0, s);
        else if (ncb == 2) launch_synth_t<0, 2, F32>(p, v, alm, phase, 0, s);
        else return SHT_EINVAL;
    } else {
        if (ncb == 1) launch_synth_t<2, 1, F32>(p, v, alm, phase, deriv, s);
        else if (ncb == 2) launch_synth_t<2, 2, F32>(p, v, alm, phase, deriv, s);
        else return SHT_EINVAL;
    }
    return SHT_OK;
}

template <bool F32>
static void dispatch_anal(const Plan &p, const LegView &v, const double *phase, double *alm,
                          int mode, hipStream_t s)
{
    const int ncb = p.tune.anal_ncb;
    if (p.spin == 0) {
        if (ncb == 1) launch_anal_t<0, 1, F32>(p, v, phase, alm, mode, s);
        else launch_anal_t<0, 2, F32>(p, v, phase, alm, mode, s);
    } else {
        if (ncb == 1) launch_anal_t<2, 1, F32>(p, v, phase, alm, mode, s);
        else launch_anal_t<2, 2, F32>(p, v, phase, alm, mode, s);
    }
}

// transforms per work item of the vector kernels: two for spin 0, one for spin > 0
int valu_jpg(const Plan &p) { return (p.spin == 0 && p.ntrans >= 2) ? 2 : 1; }

// slot tiles per lane group of the vector kernels (K slots per lane) where the
// plan has tiles enough to keep the waves busy, fewer for small grids:
// synthesis two, analysis four for one transform and two for two (measured at
// HEALPix N_side 1024, lmax 2047: synthesis 1.07 ms with two, 1.16 with four;
// analysis 1.43 ms with four, 1.49 with two)
int valu_k(const Plan &p, bool anal)
{
    // analysis, spin 0: four slots per lane (registers 208 for one transform,
    // 239 for two; six would leave one wavefront per SIMD); otherwise two
    const int kmax = (anal && p.spin == 0) ? 4 : 2;
    const int units = (p.nslots + 63) / 64;   // 64-slot units (spin plans: two tiles each)
    const int k = units >= 8 ? 4 : (units >= 2 ? 2 : 1);
    return k < kmax ? k : kmax;
}

template <int J, int K>
static void launch_synth_valu_t(const Plan &p, const LegView &v, const double *alm, double *phase, hipStream_t s)
{
    hipLaunchKernelGGL((k_legendre_synth_valu<J, K>), dim3((unsigned)p.synth_items.size()), dim3(64), 0, s, v,
                       p.d_synth_items, alm, phase);
}

template <int J, int K>
static void launch_anal_valu_t(const Plan &p, const LegView &v, const double *phase, double *alm, int mode,
                               hipStream_t s)
{
    // wavefronts per work group: two for one transform, four for two (measured
    // at HEALPix N_side 1024, lmax 2047: one transform 1.39 ms with two, 1.47 with
    // four, 1.56 with eight; two transforms 2.51 ms with four, 3.42 with two)
    const int groups = (p.ntiles + K - 1) / K;
    const int nwmax = J == 1 ? 2 : ANV_NW;
    const int nw = groups < nwmax ? (groups > 0 ? groups : 1) : nwmax;
    const dim3 grid((unsigned)(p.mmax + 1), (unsigned)((p.ntrans + J - 1) / J));
    hipLaunchKernelGGL((k_legendre_anal_valu<J, K>), grid, dim3(64 * nw), 0, s, v, p.d_anal_ms, phase, alm, mode);
}

template <int K>
static void launch_synth_valu_s_t(const Plan &p, const LegView &v, const double *alm, double *phase, int deriv,
                                  hipStream_t s)
{
    hipLaunchKernelGGL((k_legendre_synth_valu_s<1, K>), dim3((unsigned)p.synth_items.size()), dim3(64), 0, s, v,
                       p.d_synth_items, alm, phase, deriv);
}

template <int K>
static void launch_anal_valu_s_t(const Plan &p, const LegView &v, const double *phase, double *alm, int mode,
                                 hipStream_t s)
{
    const int groups = ((p.nslots + 63) / 64 + K - 1) / K;
    const int nw = groups < 2 ? (groups > 0 ? groups : 1) : 2;
    const dim3 grid((unsigned)(p.mmax + 1), (unsigned)p.ntrans);
    hipLaunchKernelGGL((k_legendre_anal_valu_s<1, K>), grid, dim3(64 * nw), 0, s, v, p.d_anal_ms, phase, alm, mode);
}

template <int J>
static void synth_valu_k(const Plan &p, const LegView &v, const double *alm, double *phase, hipStream_t s)
{
    switch (valu_k(p, false)) {
    case 2: launch_synth_valu_t<J, 2>(p, v, alm, phase, s); break;
    default: launch_synth_valu_t<J, 1>(p, v, alm, phase, s); break;
    }
}

template <int J>
static void anal_valu_k(const Plan &p, const LegView &v, const double *phase, double *alm, int mode, hipStream_t s)
{
    switch (valu_k(p, true)) {
    case 4: launch_anal_valu_t<J, 4>(p, v, phase, alm, mode, s); break;
    case 2: launch_anal_valu_t<J, 2>(p, v, phase, alm, mode, s); break;
    default: launch_anal_valu_t<J, 1>(p, v, phase, alm, mode, s); break;
    }
}

int launch_legendre_synth(const Plan &p, const double *alm, double *phase, bool deriv, hipStream_t s)
{
    if (p.synth_items.empty()) return SHT_OK;
    const LegView v = make_leg_view(p);
    log_msg(3, "launch Legendre synthesis plan %llu: %zu items, %s kernels%s, stream %p",
            (unsigned long long)p.serial, p.synth_items.size(), p.tune.valu ? "vector-unit" : "matrix-core",
            deriv ? " (derivative maps)" : "", (void *)s);
    if (p.tune.valu && p.spin == 0) {
        if (valu_jpg(p) == 1) synth_valu_k<1>(p, v, alm, phase, s);
        else synth_valu_k<2>(p, v, alm, phase, s);
        return check_hip(hipGetLastError(), "legendre synthesis launch");
    }
    if (p.tune.valu) {   // spin > 0
        if (valu_k(p, false) == 2) launch_synth_valu_s_t<2>(p, v, alm, phase, deriv ? 1 : 0, s);
        else launch_synth_valu_s_t<1>(p, v, alm, phase, deriv ? 1 : 0, s);
        return check_hip(hipGetLastError(), "legendre synthesis launch");
    }
    const int d = deriv ? 1 : 0;
    const int rc = p.precision == SHT_FP32_MFMA ? dispatch_synth<true>(p, v, alm, phase, d, s)
                                                : dispatch_synth<false>(p, v, alm, phase, d, s);
    if (rc) {
        set_error("synthesis column blocks %d not available", p.tune.synth_ncb);
        return rc;
    }
    return check_hip(hipGetLastError(), "legendre synthesis launch");
}

int launch_legendre_anal(const Plan &p, const double *phase, double *alm, int mode, hipStream_t s)
{
    const LegView v = make_leg_view(p);
    log_msg(3, "launch Legendre analysis plan %llu: %d m values x %d transforms, %s kernels, mode %d, stream %p",
            (unsigned long long)p.serial, p.mmax + 1, p.ntrans, p.tune.valu ? "vector-unit" : "matrix-core", mode,
            (void *)s);
    if (p.tune.valu && p.spin == 0) {
        if (valu_jpg(p) == 1) anal_valu_k<1>(p, v, phase, alm, mode, s);
        else anal_valu_k<2>(p, v, phase, alm, mode, s);
        return check_hip(hipGetLastError(), "legendre analysis launch");
    }
    if (p.tune.valu) {   // spin > 0
        if (valu_k(p, true) == 2) launch_anal_valu_s_t<2>(p, v, phase, alm, mode, s);
        else launch_anal_valu_s_t<1>(p, v, phase, alm, mode, s);
        return check_hip(hipGetLastError(), "legendre analysis launch");
    }
    if (p.precision == SHT_FP32_MFMA) dispatch_anal<true>(p, v, phase, alm, mode, s);
    else dispatch_anal<false>(p, v, phase, alm, mode, s);
    return check_hip(hipGetLastError(), "legendre analysis launch");
}

// ---------------------------------------------------------------- batches

// work groups of a persistent launch on a device: every CU filled to the
// kernel's occupancy
template <typename K>
static int persistent_groups(K kernel, int threads, int dev)
{
    int ncu = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)kernel, threads, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 1024;
    }
    const int g = ncu * (per_cu > 0 ? per_cu : 1);
    return g > 0 ? g : 1024;
}

template <int SPIN, int NCB, bool F32>
static int anal_batch_groups_t(int dev)
{
    return persistent_groups(k_legendre_anal_batch<SPIN, NCB, F32>, 64 * ana_nw(F32, SPIN != 0), dev);
}

int anal_batch_groups(int spin, int ncb, bool f32, int dev)
{
    const int key = (spin ? 4 : 0) + (ncb == 2 ? 2 : 0) + (f32 ? 1 : 0);
    switch (key) {
    case 0: return anal_batch_groups_t<0, 1, false>(dev);
    case 1: return anal_batch_groups_t<0, 1, true>(dev);
    case 2: return anal_batch_groups_t<0, 2, false>(dev);
    case 3: return anal_batch_groups_t<0, 2, true>(dev);
    case 4: return anal_batch_groups_t<2, 1, false>(dev);
    case 5: return anal_batch_groups_t<2, 1, true>(dev);
    case 6: return anal_batch_groups_t<2, 2, false>(dev);
    default: return anal_batch_groups_t<2, 2, true>(dev);
    }
}

template <int SPIN, int NCB, bool F32>
static int synth_batch_groups_t(int dev)
{
    return persistent_groups(k_legendre_synth_batch<SPIN, NCB, F32>, 64, dev);
}

int synth_batch_groups(int spin, int ncb, bool f32, int dev)
{
    const int key = (spin ? 4 : 0) + (ncb == 2 ? 2 : 0) + (f32 ? 1 : 0);
    switch (key) {
    case 0: return synth_batch_groups_t<0, 1, false>(dev);
    case 1: return synth_batch_groups_t<0, 1, true>(dev);
    case 2: return synth_batch_groups_t<0, 2, false>(dev);
    case 3: return synth_batch_groups_t<0, 2, true>(dev);
    case 4: return synth_batch_groups_t<2, 1, false>(dev);
    case 5: return synth_batch_groups_t<2, 1, true>(dev);
    case 6: return synth_batch_groups_t<2, 2, false>(dev);
    default: return synth_batch_groups_t<2, 2, true>(dev);
    }
}

template <int SPIN, int NCB, bool F32>
static void launch_synth_batch_t(const Batch &b, const BatchPtrs &ptrs, int deriv, hipStream_t s)
{
    unsigned *counters = b.d_counter + 16;
    SynQueues q;
    for (int d = 0; d <= NUM_XCD; ++d) q.ofs[d] = b.syn_ofs[d];
    hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(64), 0, s, counters, NUM_XCD, 16);
    hipLaunchKernelGGL((k_legendre_synth_batch<SPIN, NCB, F32>), dim3((unsigned)b.syn_groups), dim3(64), 0, s,
                       b.d_views, b.d_syn, q, ptrs, b.syn_flush, deriv, counters);
}

int launch_legendre_synth_batch(const Batch &b, const BatchPtrs &ptrs, bool deriv, hipStream_t s)
{
    if (b.nsyn == 0) return SHT_OK;
    log_msg(3, "launch persistent batch Legendre synthesis: %d items, %d wavefronts%s, stream %p", b.nsyn,
            b.syn_groups, deriv ? " (derivative maps)" : "", (void *)s);
    const bool f32 = b.precision == SHT_FP32_MFMA;
    const int d = deriv ? 1 : 0;
    const int key = (b.spin ? 4 : 0) + (b.syn_ncb == 2 ? 2 : 0) + (f32 ? 1 : 0);
    switch (key) {
    case 0: launch_synth_batch_t<0, 1, false>(b, ptrs, 0, s); break;
    case 1: launch_synth_batch_t<0, 1, true>(b, ptrs, 0, s); break;
    case 2: launch_synth_batch_t<0, 2, false>(b, ptrs, 0, s); break;
    case 3: launch_synth_batch_t<0, 2, true>(b, ptrs, 0, s); break;
    case 4: launch_synth_batch_t<2, 1, false>(b, ptrs, d, s); break;
    case 5: launch_synth_batch_t<2, 1, true>(b, ptrs, d, s); break;
    case 6: launch_synth_batch_t<2, 2, false>(b, ptrs, d, s); break;
    default: launch_synth_batch_t<2, 2, true>(b, ptrs, d, s); break;
    }
    return check_hip(hipGetLastError(), "batch legendre synthesis launch");
}

template <int SPIN, int NCB, bool F32>
static void launch_anal_batch_t(const Batch &b, const BatchPtrs &ptrs, int mode, hipStream_t s)
{
    auto k = k_legendre_anal_batch<SPIN, NCB, F32>;
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, s, b.d_counter);
    hipLaunchKernelGGL(k, dim3((unsigned)b.ana_groups), dim3(64 * ana_nw(F32, SPIN != 0)), 0, s, b.d_views, b.d_ana,
                       b.nana, ptrs, mode, b.d_counter);
}

int launch_legendre_anal_batch(const Batch &b, const BatchPtrs &ptrs, int mode, hipStream_t s)
{
    if (b.nana == 0) return SHT_OK;
    log_msg(3, "launch persistent batch Legendre analysis: %d items, %d work groups, mode %d, stream %p", b.nana,
            b.ana_groups, mode, (void *)s);
    const bool f32 = b.precision == SHT_FP32_MFMA;
    const int key = (b.spin ? 4 : 0) + (b.ana_ncb == 2 ? 2 : 0) + (f32 ? 1 : 0);
    switch (key) {
    case 0: launch_anal_batch_t<0, 1, false>(b, ptrs, mode, s); break;
    case 1: launch_anal_batch_t<0, 1, true>(b, ptrs, mode, s); break;
    case 2: launch_anal_batch_t<0, 2, false>(b, ptrs, mode, s); break;
    case 3: launch_anal_batch_t<0, 2, true>(b, ptrs, mode, s); break;
    case 4: launch_anal_batch_t<2, 1, false>(b, ptrs, mode, s); break;
    case 5: launch_anal_batch_t<2, 1, true>(b, ptrs, mode, s); break;
    case 6: launch_anal_batch_t<2, 2, false>(b, ptrs, mode, s); break;
    default: launch_anal_batch_t<2, 2, true>(b, ptrs, mode, s); break;
    }
    return check_hip(hipGetLastError(), "batch legendre analysis launch");
}

}  // namespace sht
