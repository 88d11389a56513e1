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
// k runs over degrees (spin 0) or (degree, W/X) pairs (spin 2) of one parity
// class, col over (transform, component, re/im).  With
// lambda(pi-t) = (-1)^(l+m) lambda(t) (spin 0), resp. W(pi-t) = (-1)^(l+m) W(t),
// X(pi-t) = -(-1)^(l+m) X(t) for W, X = (2lambda +- -2lambda)/2 (spin 2), two
// class accumulators A0, A1 give both rings: t: A0 + A1, pi - t: A0 - A1.
// Spin-2 column maps (HEALPix convention -+2 a = -(E +- iB)):
//   Q_re = -E_re W + B_im X,  Q_im = -E_im W - B_re X,
//   U_re = -B_re W - E_im X,  U_im = -B_im W + E_re X.
//
// Analysis (Eq. 5), per m: out[l][col] = sum_slot Lambda[l][slot] G[slot][col]
// with the ring pair folded into G_t +- G_(pi-t); a work group of LEG_NW
// wavefronts walks the active tiles LEG_NW at a time, reduces the wavefronts'
// partial sums in LDS and accumulates them into the output in a fixed order
// (deterministic, no atomics).
#include <hip/hip_runtime.h>

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

// Per-chain step coefficients of one chunk, staged in LDS:
// (alpha_l, +-beta_l, alpha_l +- beta_l - 2, 0) for the chain's sign.
__device__ inline double4 chain_coef(const double4 c, bool minus)
{
    return minus ? double4{c.x, -c.y, c.w, 0.0} : double4{c.x, c.y, c.z, 0.0};
}

// Run the recursion over the degrees lc .. lc+LC-1, writing lambda (true value
// or 0 while the lane's scale k < 0) to out[t * stride].
template <typename T, int LC>
__device__ inline void chain_chunk(Chain &c, const double4 *__restrict__ cf, bool diff, bool slow,
                                   int l0, int lc, int lmax, T *out, int stride, double thr,
                                   double down)
{
    if (!slow) {
#pragma unroll 4
        for (int t = 0; t < LC; ++t) {
            const int l = lc + t;
            out[t * stride] = (l >= l0 && l <= lmax) ? (T)c.mu : (T)0;
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
            out[t * stride] = (l >= l0 && l <= lmax && c.k == 0) ? (T)c.mu : (T)0;
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
template <typename T, int LC>
__device__ __forceinline__ void chain_chunk_fast(Chain &c, const double4 *__restrict__ cf, bool diff,
                                                 T *out, int stride)
{
    if (diff) {
#pragma unroll
        for (int t = 0; t < LC; ++t) {
            out[t * stride] = (T)c.mu;
            const double4 q = cf[t];
            const double eps = fma(q.x, c.ms2, q.z);
            c.aux = fma(eps, c.mu, c.aux);
            c.mu += c.aux;
        }
    } else {
#pragma unroll
        for (int t = 0; t < LC; ++t) {
            out[t * stride] = (T)c.mu;
            const double4 q = cf[t];
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

// Recursion role of a wavefront within a work group of LEG_NW = 4 wavefronts
// covering 4 slot tiles.  Spin 0: wavefront w runs tile w (64 slots).  Spin 2:
// wavefronts 2g and 2g+1 run the +2 and -2 chains of tiles 2g, 2g+1 (32 slots
// each), so that every wavefront's chains share one sign.
template <int SPIN>
struct RecRole {
    int tile_local;    // tile (0..3) of this lane's chain
    int slot_local;    // slot within that tile
    int chain;         // 0: +s, 1: -s
    __device__ RecRole(int wave, int lane)
    {
        if (SPIN) {
            tile_local = 2 * (wave >> 1) + (lane >> 5);
            slot_local = lane & 31;
            chain = wave & 1;
        } else {
            tile_local = wave;
            slot_local = lane;
            chain = 0;
        }
    }
};

// ---------------------------------------------------------------- synthesis

constexpr int SYN_LC = 16;   // degrees per chunk

// B-operand layout of a synthesis chunk (16 degrees lc .. lc+15, lc + m even).
// Element e = ((p * KS + ks) * NCB + cb) * 64 + lane, lane = j + 16 kk, column
// col = j + 16 cb.  Spin 0: class p, k-step ks holds the degrees
// lc + p + 2 kk + 8 ks.  Spin 2: each k-step holds rows of one kind, so that
// the A operand is built with the same operation in every lane:
//   class 0: ks 0,1: W rows at lc + 8 ks + 2 kk;  ks 2,3: X rows at lc + 8 (ks-2) + 2 kk + 1
//   class 1: ks 0,1: W rows at lc + 8 ks + 2 kk + 1;  ks 2,3: X rows at lc + 8 (ks-2) + 2 kk
// (W rows have the parity class of l + m, X rows the opposite one).
template <int SPIN, int NCB>
struct SynLayout {
    static constexpr int KS = SPIN ? 4 : 2;
    static constexpr int NB = 2 * KS * NCB * 64;
    // degree offset, a_lm component / re-im and sign-scale of element e; scale 0: zero
    __device__ static inline void element(int e, int m, int t0, int ntrans, int &loff,
                                          int &tcomp, int &reim, double &scale)
    {
        const int ln = e & 63;
        const int cb = (e >> 6) % NCB;
        const int ks = (e >> 6) / NCB % KS;
        const int p = (e >> 6) / NCB / KS;
        const int j = ln & 15, kk = ln >> 4;
        const int col = j + 16 * cb;
        if constexpr (SPIN == 0) {
            loff = p + 2 * kk + 8 * ks;
            const int t = t0 + (col >> 1);
            reim = col & 1;
            tcomp = t;
            scale = (t < ntrans && !(m == 0 && reim)) ? 1.0 : 0.0;
        } else {
            const bool wrow = ks < 2;
            const int par = (p == 0) ? (wrow ? 0 : 1) : (wrow ? 1 : 0);
            loff = 8 * (ks & 1) + 2 * kk + par;
            const int t = t0 + (col >> 2);
            const int o = col & 3;
            int comp;
            // W row: -(E_re, E_im, B_re, B_im); X row: (B_im, -B_re, -E_im, E_re); times 1/2
            if (wrow) {
                comp = o >> 1;
                reim = o & 1;
                scale = -0.5;
            } else {
                comp = (o == 0 || o == 1) ? 1 : 0;
                reim = (o == 0 || o == 2) ? 1 : 0;
                scale = (o == 0 || o == 3) ? 0.5 : -0.5;
            }
            tcomp = 2 * t + comp;
            if (t >= ntrans || (m == 0 && reim)) scale = 0.0;
        }
    }
};

template <int SPIN, int NCB, bool F32>
__global__ __launch_bounds__(64 * LEG_NW, 2) void k_legendre_synth(LegView v,
                                                                   const LegItem *__restrict__ items,
                                                                   const double *__restrict__ alm,
                                                                   double *__restrict__ phase,
                                                                   int jobs_per_group, int flush_chunks)
{
    using T = typename MT<F32>::T;
    using V = typename MT<F32>::V;
    using LY = SynLayout<SPIN, NCB>;
    constexpr int SPT = SPIN ? 32 : 64;          // slots per tile
    constexpr int NSB = SPT / 16;                // 16-slot row blocks
    constexpr int LC = SYN_LC;
    constexpr int KS = LY::KS;
    constexpr int NB = LY::NB;
    constexpr int NT = 64 * LEG_NW;
    constexpr int BPT = NB / NT;                 // fragment elements per thread
    static_assert(NB % NT == 0, "fragment staging");
    constexpr int NCH = SPIN ? 2 : 1;
    constexpr int NCOMP = SPIN ? 2 : 1;
    __shared__ T bst[2][NB];
    __shared__ double4 cfs[2][NCH][LC];
    __shared__ T lam[LEG_NW][LC][NCH][SPT];

    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int i16 = lane & 15, kk = lane >> 4;
    const LegItem *it = items + blockIdx.x;
    const int m = it->m;
    const int t0 = blockIdx.y * jobs_per_group;
    const int lmax = v.lmax;
    const int l0 = m > SPIN ? m : SPIN;
    const int lstart = l0 - ((l0 + m) & 1);
    const double4 *coef = v.coef + v.coef_ofs[m];
    const double *flm = v.fl + v.coef_ofs[m];
    const int64_t mbase = (int64_t)m * (2 * (int64_t)lmax + 1 - m) / 2;
    const double thr = ldexp(1.0, v.thresh_bits), down = ldexp(1.0, -v.rescale_bits);

    // recursion role
    const RecRole<SPIN> rr(wave, lane);
    const int rtile = it->tile[rr.tile_local];
    Chain cs = chain_init(v, m, rtile >= 0 ? rtile * SPT + rr.slot_local : v.nslots, rr.chain);
    const bool diff = wave_any(cs.x > DIFF_FORM_COS);
    if (diff) cs.aux = cs.mu;
    bool slow = wave_any(cs.k < 0);
    T *lam_out = &lam[rr.tile_local][0][rr.chain][rr.slot_local];
    // product role
    const int mtile = it->tile[wave];
    const bool active = mtile >= 0;
    const int slot0 = active ? mtile * SPT : 0;

    // this thread's staging elements: fixed source column, degree offset, scale
    const double *ebase[BPT];
    int eloff[BPT];
    double escale[BPT];
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
        int loff, tcomp, reim;
        double sc;
        LY::element(tid + j * NT, m, t0, v.ntrans, loff, tcomp, reim, sc);
        eloff[j] = loff;
        escale[j] = sc;
        ebase[j] = (sc != 0.0) ? alm + ((int64_t)tcomp * v.nalm + mbase) * 2 + reim : alm;
    }
    double pv[BPT];
    double4 pc = double4{0, 0, 0, 0};
    auto prefetch = [&](int lc) {
#pragma unroll
        for (int j = 0; j < BPT; ++j) {
            const int l = lc + eloff[j];
            const bool ok = escale[j] != 0.0 && l >= l0 && l <= lmax;
            pv[j] = ok ? ebase[j][2 * (int64_t)l] * (escale[j] * flm[l]) : 0.0;
        }
        if (tid < NCH * LC) {
            const int l = lc + (tid % LC);
            const double4 c = (l >= l0 && l < lmax) ? coef[l] : double4{0, 0, 0, 0};
            pc = chain_coef(c, tid >= LC);
        }
    };
    auto commit = [&](int buf) {
#pragma unroll
        for (int j = 0; j < BPT; ++j) bst[buf][tid + j * NT] = (T)pv[j];
        if (tid < NCH * LC) cfs[buf][tid / LC][tid % LC] = pc;
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

    prefetch(lstart);
    commit(0);
    __syncthreads();
    int chunk = 0;
    for (int lc = lstart; lc <= lmax; lc += LC, ++chunk) {
        const int buf = chunk & 1;
        const bool more = lc + LC <= lmax;
        if (more) prefetch(lc + LC);
        if (rtile >= 0 || !SPIN) {
            if (!slow && lc >= l0 && lc + LC <= lmax) {
                chain_chunk_fast<T, LC>(cs, cfs[buf][rr.chain], diff, lam_out, NCH * SPT);
            } else {
                chain_chunk<T, LC>(cs, cfs[buf][rr.chain], diff, slow, l0, lc, lmax, lam_out,
                                   NCH * SPT, thr, down);
                slow = wave_any(cs.k < 0);
            }
        }
        __syncthreads();
        if (active) {
            const T *bb = bst[buf];
            if constexpr (SPIN == 0) {
#pragma unroll
                for (int ks = 0; ks < KS; ++ks)
#pragma unroll
                    for (int sb = 0; sb < NSB; ++sb) {
                        const T a0 = lam[wave][0 + 2 * kk + 8 * ks][0][sb * 16 + i16];
                        const T a1 = lam[wave][1 + 2 * kk + 8 * ks][0][sb * 16 + i16];
#pragma unroll
                        for (int cb = 0; cb < NCB; ++cb) {
                            acc[0][sb][cb] = mfma(a0, bb[((0 * KS + ks) * NCB + cb) * 64 + lane], acc[0][sb][cb]);
                            acc[1][sb][cb] = mfma(a1, bb[((1 * KS + ks) * NCB + cb) * 64 + lane], acc[1][sb][cb]);
                        }
                    }
            } else {
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int sb = 0; sb < NSB; ++sb) {
                        const int te = 8 * h + 2 * kk;
                        const T upe = lam[wave][te][0][sb * 16 + i16];
                        const T ume = lam[wave][te][1][sb * 16 + i16];
                        const T upo = lam[wave][te + 1][0][sb * 16 + i16];
                        const T umo = lam[wave][te + 1][1][sb * 16 + i16];
                        const T we = upe + ume, xe = upe - ume;
                        const T wo = upo + umo, xo = upo - umo;
#pragma unroll
                        for (int cb = 0; cb < NCB; ++cb) {
                            acc[0][sb][cb] = mfma(we, bb[((0 * KS + h) * NCB + cb) * 64 + lane], acc[0][sb][cb]);
                            acc[0][sb][cb] = mfma(xo, bb[((0 * KS + 2 + h) * NCB + cb) * 64 + lane], acc[0][sb][cb]);
                            acc[1][sb][cb] = mfma(wo, bb[((1 * KS + h) * NCB + cb) * 64 + lane], acc[1][sb][cb]);
                            acc[1][sb][cb] = mfma(xe, bb[((1 * KS + 2 + h) * NCB + cb) * 64 + lane], acc[1][sb][cb]);
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
        }
        if (more) commit(buf ^ 1);
        __syncthreads();
    }
    if (!active) return;

    // epilogue: ring t = A0 + A1, ring pi - t = A0 - A1
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
                const int slot = slot0 + sb * 16 + row;
                if (slot >= v.nslots) continue;
                const int col = i16 + 16 * cb;
                int t, comp, reim;
                if constexpr (SPIN == 0) {
                    t = t0 + (col >> 1);
                    comp = 0;
                    reim = col & 1;
                } else {
                    t = t0 + (col >> 2);
                    comp = (col & 3) >> 1;
                    reim = col & 1;
                }
                if (t >= v.ntrans) continue;
                const int yn = v.slot_yn[slot], ys = v.slot_ys[slot];
                const int64_t rowbase = ((int64_t)t * NCOMP + comp) * v.nrings;
                if (yn >= 0) phase[((rowbase + yn) * (v.mmax + 1) + m) * 2 + reim] = c0 + c1;
                if (ys >= 0) phase[((rowbase + ys) * (v.mmax + 1) + m) * 2 + reim] = c0 - c1;
            }
}

// ---------------------------------------------------------------- analysis

constexpr int ANA_LC = 32;   // degrees per chunk (16 per parity class)

template <int SPIN, int NCB, bool F32>
__global__ __launch_bounds__(64 * LEG_NW, 2) void k_legendre_anal(LegView v, const int *__restrict__ mlist,
                                                                  const double *__restrict__ phase,
                                                                  double *__restrict__ alm,
                                                                  int jobs_per_group, int grad)
{
    using T = typename MT<F32>::T;
    using V = typename MT<F32>::V;
    constexpr int SPT = SPIN ? 32 : 64;
    constexpr int LC = ANA_LC;
    constexpr int KSA = SPT / 4;       // k-steps (4 slots each) per tile
    constexpr int NCH = SPIN ? 2 : 1;
    constexpr int NCOMP = SPIN ? 2 : 1;
    constexpr int LDP = SPT + 1;       // padded LDS row
    constexpr int NT = 64 * LEG_NW;
    constexpr int CPJ = SPIN ? 4 : 2;  // columns per transform
    constexpr int NCOL = NCB * 16;
    constexpr int NOUT = LC * NCOL;    // output elements per chunk
    constexpr int OPT = (NOUT + NT - 1) / NT;
    constexpr int LAMW = NCH * LC * LDP;   // lambda elements per tile
    // lambda tiles and, once the products are done, the partial sums share LDS
    constexpr int LAM_BYTES = LEG_NW * LAMW * (int)sizeof(T);
    constexpr int PART_BYTES = LEG_NW * NOUT * (int)sizeof(double);
    constexpr int SMEM_D = ((LAM_BYTES > PART_BYTES ? LAM_BYTES : PART_BYTES) + 7) / 8;
    __shared__ double smem[SMEM_D];
    __shared__ double4 cfs[NCH][LC];
    __shared__ double fls[LC];

    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int i16 = lane & 15, kk = lane >> 4;
    const int m = mlist[blockIdx.x];
    const int t0 = blockIdx.y * jobs_per_group;
    const int lmax = v.lmax;
    const int l0 = m > SPIN ? m : SPIN;
    const int lstart = l0 - ((l0 + m) & 1);
    const double4 *coef = v.coef + v.coef_ofs[m];
    const double *flm = v.fl + v.coef_ofs[m];
    const int64_t mbase = (int64_t)m * (2 * (int64_t)lmax + 1 - m) / 2;
    const double thr = ldexp(1.0, v.thresh_bits), down = ldexp(1.0, -v.rescale_bits);
    T *lamb = reinterpret_cast<T *>(smem);          // [tile][chain][LC][LDP]
    double *part = smem;                            // [LEG_NW][NOUT] after the products
    const RecRole<SPIN> rr(wave, lane);
    T *lam_out = lamb + (rr.tile_local * NCH + rr.chain) * LC * LDP + rr.slot_local;
    const T *lam_mine = lamb + wave * LAMW;

    // this thread's output elements of a chunk: element e -> (transform, component,
    // degree offset, re/im), consecutive e consecutive in memory
    double *obase[OPT];
    int oloff[OPT], oreim[OPT];
#pragma unroll
    for (int j = 0; j < OPT; ++j) {
        const int e = tid + j * NT;
        const int reim = e & 1;
        const int loff = (e >> 1) % LC;
        const int tc = (e >> 1) / LC;
        const int t = t0 + tc / NCOMP, comp = tc % NCOMP;
        oreim[j] = reim;
        oloff[j] = (e < NOUT && t < v.ntrans) ? loff : -1000000;
        obase[j] = alm + (((int64_t)(t < v.ntrans ? t : 0) * NCOMP + comp) * v.nalm + mbase) * 2 + reim;
    }

    // degrees below l0 (spin 2 with m < 2) are zero by convention
    for (int e = tid; e < 2 * NCOMP * (NCOL / CPJ) * 2; e += NT) {
        const int l = m + (e & 1);
        const int rest = e >> 1;
        const int reim = rest & 1, tc = rest >> 1;
        const int t = t0 + tc / NCOMP, comp = tc % NCOMP;
        if (l < l0 && t < v.ntrans)
            alm[(((int64_t)t * NCOMP + comp) * v.nalm + mbase + l) * 2 + reim] = 0.0;
    }

    int ntiles_act = 0;
    for (int t = 0; t < v.ntiles; ++t) ntiles_act += v.tile_mlim[t] >= m;
    int tcount = 0, tscan = 0;
    bool first = true;
    while (tcount < ntiles_act || first) {
        int ptile_r = -1, ptile_m = -1;    // tiles of this wave's recursion and product roles
        {
            int k = 0;
            for (; tscan < v.ntiles && k < LEG_NW; ++tscan) {
                if (v.tile_mlim[tscan] < m) continue;
                if (k == rr.tile_local) ptile_r = tscan;
                if (k == wave) ptile_m = tscan;
                ++k;
            }
            tcount += k;
        }
        const bool active = ptile_m >= 0;
        const int slot0 = active ? ptile_m * SPT : 0;
        // stationary phase fragments B[kk][j] for slot 4 ks + kk and column j + 16 cb:
        // gw[q] multiplies W (spin 2) or lambda (spin 0) rows, gx[q] the X rows;
        // q = 0: G_t + G_(pi-t), q = 1: G_t - G_(pi-t).  For output o the X part
        // is sigma_o times the W operand of column 3 - o, sigma = (-, +, +, -).
        T gw[2][KSA][NCB], gx[SPIN ? 2 : 1][SPIN ? KSA : 1][SPIN ? NCB : 1];
#pragma unroll
        for (int ks = 0; ks < KSA; ++ks) {
            const int slot = slot0 + 4 * ks + kk;
            int yn = -1, ys = -1;
            if (active && slot < v.nslots) {
                yn = v.slot_yn[slot];
                ys = v.slot_ys[slot];
            }
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                const int col = i16 + 16 * cb;
                const int tl = col / CPJ, o = col % CPJ;
                const int t = t0 + tl;
                auto gval = [&](int oo, double &gsum, double &gdif) {
                    const int comp = SPIN ? (oo >> 1) : 0, reim = oo & 1;
                    double gn = 0.0, gs = 0.0;
                    if (t < v.ntrans) {
                        const int64_t rowbase = ((int64_t)t * NCOMP + comp) * v.nrings;
                        if (yn >= 0) gn = phase[((rowbase + yn) * (v.mmax + 1) + m) * 2 + reim];
                        if (ys >= 0) gs = phase[((rowbase + ys) * (v.mmax + 1) + m) * 2 + reim];
                    }
                    gsum = gn + gs;
                    gdif = gn - gs;
                };
                double a, b;
                gval(o, a, b);
                const double sg = SPIN ? -1.0 : 1.0;
                gw[0][ks][cb] = (T)(sg * a);
                gw[1][ks][cb] = (T)(sg * b);
                if constexpr (SPIN) {
                    double c, d;
                    gval(3 - o, c, d);
                    const double sx = (o == 0 || o == 3) ? 1.0 : -1.0;   // sigma_o * (-1)
                    gx[0][ks][cb] = (T)(sx * c);
                    gx[1][ks][cb] = (T)(sx * d);
                }
            }
        }
        Chain cs = chain_init(v, m, ptile_r >= 0 ? ptile_r * SPT + rr.slot_local : v.nslots, rr.chain);
        const bool diff = wave_any(cs.x > DIFF_FORM_COS);
        if (diff) cs.aux = cs.mu;
        bool slow = wave_any(cs.k < 0);
        for (int lc = lstart; lc <= lmax; lc += LC) {
            double pold[OPT];
            if (tid < NCH * LC) {
                const int l = lc + (tid % LC);
                const double4 c = (l >= l0 && l < lmax) ? coef[l] : double4{0, 0, 0, 0};
                cfs[tid / LC][tid % LC] = chain_coef(c, tid >= LC);
            }
            if (tid < LC) {
                const int l = lc + tid;
                fls[tid] = (l >= l0 && l <= lmax) ? flm[l] : 0.0;
            }
            if (!first) {
#pragma unroll
                for (int j = 0; j < OPT; ++j) {
                    const int l = lc + oloff[j];
                    pold[j] = (l >= l0 && l <= lmax) ? obase[j][2 * (int64_t)l] : 0.0;
                }
            }
            __syncthreads();
            if (ptile_r >= 0 || !SPIN) {
                if (!slow && lc >= l0 && lc + LC <= lmax) {
                    chain_chunk_fast<T, LC>(cs, cfs[rr.chain], diff, lam_out, LDP);
                } else {
                    chain_chunk<T, LC>(cs, cfs[rr.chain], diff, slow, l0, lc, lmax, lam_out, LDP, thr, down);
                    slow = wave_any(cs.k < 0);
                }
            }
            __syncthreads();
            V acc[2][NCB];   // [class][column block]
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb) acc[p][cb] = V{0, 0, 0, 0};
            if (active) {
#pragma unroll
                for (int p = 0; p < 2; ++p) {
#pragma unroll
                    for (int ks = 0; ks < KSA; ++ks) {
                        // A[i][kk] = Lambda[degree lc + p + 2 i][slot 4 ks + kk]
                        if constexpr (SPIN == 0) {
                            const T a = lam_mine[(p + 2 * i16) * LDP + 4 * ks + kk];
#pragma unroll
                            for (int cb = 0; cb < NCB; ++cb) acc[p][cb] = mfma(a, gw[p][ks][cb], acc[p][cb]);
                        } else {
                            const T up = lam_mine[(0 * LC + p + 2 * i16) * LDP + 4 * ks + kk];
                            const T um = lam_mine[(1 * LC + p + 2 * i16) * LDP + 4 * ks + kk];
                            const T aw = up + um, ax = up - um;
#pragma unroll
                            for (int cb = 0; cb < NCB; ++cb) {
                                acc[p][cb] = mfma(aw, gw[p][ks][cb], acc[p][cb]);
                                acc[p][cb] = mfma(ax, gx[1 - p][ks][cb], acc[p][cb]);
                            }
                        }
                    }
                }
            }
            __syncthreads();   // lambda no longer needed: its LDS holds the partials
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
                        part[wave * NOUT + e] = active ? (double)acc[p][cb][r] : 0.0;
                    }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < OPT; ++j) {
                const int e = tid + j * NT;
                const int l = lc + oloff[j];
                if (e >= NOUT || l < l0 || l > lmax) continue;
                double s = 0.0;
#pragma unroll
                for (int w = 0; w < LEG_NW; ++w) s += part[w * NOUT + e];
                s *= SPIN ? 0.5 * fls[oloff[j]] : fls[oloff[j]];
                if (grad && m > 0) s *= 2.0;   // fac_m of the real-field gradient
                if (m == 0 && oreim[j]) s = 0.0;
                obase[j][2 * (int64_t)l] = first ? s : pold[j] + s;
            }
            __syncthreads();
        }
        first = false;
    }
}

// ---------------------------------------------------------------- launchers

// column blocks (16 columns each) per work group: bounded so that the
// accumulators (synthesis) or the stationary phases (analysis) stay in
// registers at two wavefronts per SIMD
static int ncb_for(int spin, int ntrans, bool f32, bool anal)
{
    const int cols = ntrans * (spin ? 4 : 2);
    int ncb = (cols + 15) / 16;
    (void)f32;
    (void)anal;
    return ncb > 2 ? 2 : ncb;
}

template <int SPIN, int NCB, bool F32>
static void launch_synth_t(const Plan &p, const LegView &v, const double *alm, double *phase,
                           hipStream_t s)
{
    const int jpg = NCB * 16 / (SPIN ? 4 : 2);
    dim3 grid((unsigned)p.synth_items.size(), (unsigned)((p.ntrans + jpg - 1) / jpg));
    hipLaunchKernelGGL((k_legendre_synth<SPIN, NCB, F32>), grid, dim3(64 * LEG_NW), 0, s, v,
                       p.d_synth_items, alm, phase, jpg, p.flush_chunks);
}

template <int SPIN, int NCB, bool F32>
static void launch_anal_t(const Plan &p, const LegView &v, const double *phase, double *alm,
                          int grad, hipStream_t s)
{
    const int jpg = NCB * 16 / (SPIN ? 4 : 2);
    dim3 grid((unsigned)(p.mmax + 1), (unsigned)((p.ntrans + jpg - 1) / jpg));
    hipLaunchKernelGGL((k_legendre_anal<SPIN, NCB, F32>), grid, dim3(64 * LEG_NW), 0, s, v,
                       p.d_anal_ms, phase, alm, jpg, grad);
}

template <bool F32>
static void dispatch_synth(const Plan &p, const LegView &v, const double *alm, double *phase,
                           hipStream_t s)
{
    const int ncb = ncb_for(p.spin, p.ntrans, F32, false);
    if (p.spin == 0) {
        if (ncb == 1) launch_synth_t<0, 1, F32>(p, v, alm, phase, s);
        else launch_synth_t<0, 2, F32>(p, v, alm, phase, s);
    } else {
        if (ncb == 1) launch_synth_t<2, 1, F32>(p, v, alm, phase, s);
        else launch_synth_t<2, 2, F32>(p, v, alm, phase, s);
    }
}

template <bool F32>
static void dispatch_anal(const Plan &p, const LegView &v, const double *phase, double *alm,
                          int grad, hipStream_t s)
{
    const int ncb = ncb_for(p.spin, p.ntrans, F32, true);
    if (p.spin == 0) {
        if (ncb == 1) launch_anal_t<0, 1, F32>(p, v, phase, alm, grad, s);
        else launch_anal_t<0, 2, F32>(p, v, phase, alm, grad, s);
    } else {
        if (ncb == 1) launch_anal_t<2, 1, F32>(p, v, phase, alm, grad, s);
        else launch_anal_t<2, 2, F32>(p, v, phase, alm, grad, s);
    }
}

int launch_legendre_synth(const Plan &p, const double *alm, double *phase, hipStream_t s)
{
    if (p.synth_items.empty()) return SHT_OK;
    const LegView v = make_leg_view(p);
    if (p.precision == SHT_FP32_MFMA) dispatch_synth<true>(p, v, alm, phase, s);
    else dispatch_synth<false>(p, v, alm, phase, s);
    return check_hip(hipGetLastError(), "legendre synthesis launch");
}

int launch_legendre_anal(const Plan &p, const double *phase, double *alm, bool grad, hipStream_t s)
{
    const LegView v = make_leg_view(p);
    if (p.precision == SHT_FP32_MFMA) dispatch_anal<true>(p, v, phase, alm, grad ? 1 : 0, s);
    else dispatch_anal<false>(p, v, phase, alm, grad ? 1 : 0, s);
    return check_hip(hipGetLastError(), "legendre analysis launch");
}

}  // namespace sht
