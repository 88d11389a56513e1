// Legendre step on gfx950 matrix cores (Eqs. 4 and 5 of the paper).
//
// For each m and each slot (a ring and its mirror ring), lambda_lm is produced
// by the three-term recursion in l (Sect. 4.1, Eq. 11) in the rescaled form
//   mu_{l+1} = (alpha_l x +- beta_l) mu_l - mu_{l-1},   lambda_l = f_l mu_l,
// one chain per wavefront lane, with an extended exponent: a lane carries an
// integer scale k (true value = mu 2^(S k)) and contributes nothing while
// k < 0 (|lambda| < 2^-(S/2)); see Sect. 4.1 on the enhanced exponent range.
// lambda never leaves the chip (Sect. 3.2: applied as soon as it is computed):
// each 16- or 32-degree chunk is staged in LDS and consumed by MFMA tiles.
//
// Synthesis (Eq. 4) for a tile of slots:
//   C[slot][col] += sum_k Lambda[slot][k] * Coef[k][col]
// where k runs over degrees (spin 0) or (degree, W/X) pairs (spin 2) of one
// parity class, and col over (transform, component, re/im).  Because
// lambda(pi - theta) = (-1)^(l+m) lambda(theta) (spin 0), resp.
// W(pi-t) = (-1)^(l+m) W(t), X(pi-t) = -(-1)^(l+m) X(t) with
// W = (2lambda + -2lambda)/2, X = (2lambda - -2lambda)/2 (spin 2), two
// class accumulators A0, A1 give both rings: north = A0 + A1, south = A0 - A1.
//
// Analysis (Eq. 5) for one m: out[l][col] = sum_slot Lambda[l][slot] G[slot][col]
// with the ring pair folded into G_N +- G_S per class; one wavefront owns an m,
// walks the active slot tiles, and accumulates each 32-degree chunk into the
// output (deterministic order, no atomics).
//
// Spin-2 conventions: -+2 a = -(E +- iB);  with W, X as above
//   Q = sum [-E W + i(-B) X]... written out per real part in the column maps:
//   Q_re = -E_re W + B_im X,  Q_im = -E_im W - B_re X,
//   U_re = -B_re W - E_im X,  U_im = -B_im W + E_re X,
// and the analysis uses the transposed map (E from G^Q, G^U likewise).
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

// Row of the 16x16 result held in register r of this lane (column = lane & 15).
// The two instructions use different result layouts.
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

struct ChainState {
    double x;     // cos theta of the slot's north ring
    double sig;   // +1: chain +s, -1: chain -s
    double mu0;   // mu_{l-1}
    double mu1;   // mu_l
    int k;        // scale index (value = mu * 2^(S k)), k <= 0
};

// Initial state at l = l0 for one lane.
__device__ inline ChainState chain_init(const LegView &v, int m, int slot, int chain)
{
    ChainState c;
    c.sig = chain ? -1.0 : 1.0;
    c.mu0 = 0.0;
    c.mu1 = 0.0;
    c.k = 0;
    c.x = 0.0;
    if (slot >= v.nslots) return c;
    const double x = v.slot_cos[slot], st = v.slot_sin[slot];
    c.x = x;
    if (v.polar_T >= 0.0) {
        const double s = (double)v.spin, mm = (double)m;
        double q = mm * mm + s * s - 2.0 * mm * s * fabs(x);
        double crit = sqrt(q > 0.0 ? q : 0.0) - (double)v.lmax * st;
        if (crit > v.polar_T) return c;   // skipped term (Sect. 3.3)
    }
    const StartCoef sc = v.start[2 * m + chain];
    double mc, ms;
    int ec, es;
    xpow(v.slot_chalf[slot], sc.p, mc, ec);
    xpow(v.slot_shalf[slot], sc.q, ms, es);
    int d;
    double mant = frexp(sc.kmant * mc * ms, &d);
    if (mant == 0.0) return c;
    const int e = sc.kexp + ec + es + d;
    const int S = v.rescale_bits, T = v.thresh_bits;
    int kk = 0;
    if (e < T) kk = (T - e) / S;
    c.k = -kk;
    c.mu1 = (double)sc.sign * ldexp(mant, e + S * kk);
    return c;
}

// One recursion step from l to l+1 (coefficients of degree l).
__device__ __forceinline__ void chain_step(ChainState &c, double alpha, double beta)
{
    const double t = fma(alpha, c.x, c.sig * beta);
    const double mu2 = fma(t, c.mu1, -c.mu0);
    c.mu0 = c.mu1;
    c.mu1 = mu2;
}

__device__ __forceinline__ void chain_rescale(ChainState &c, double thr, double down)
{
    if (c.k < 0 && fabs(c.mu1) >= thr) {
        c.mu1 *= down;
        c.mu0 *= down;
        c.k += 1;
    }
}

__device__ __forceinline__ bool wave_any(bool p)
{
    return __builtin_amdgcn_ballot_w64(p) != 0;
}

// ---------------------------------------------------------------- synthesis

constexpr int SYN_LC = 16;   // degrees per chunk

template <int SPIN, int NCB, bool F32>
__global__ __launch_bounds__(64) void k_legendre_synth(LegView v, const LegItem *__restrict__ items,
                                                       const double *__restrict__ alm,
                                                       double *__restrict__ phase, int jobs_per_group,
                                                       int flush_chunks)
{
    using T = typename MT<F32>::T;
    using V = typename MT<F32>::V;
    constexpr int SPT = SPIN ? 32 : 64;          // slots per tile
    constexpr int NSB = SPT / 16;                // 16-slot row blocks
    constexpr int LC = SYN_LC;
    constexpr int KS = SPIN ? LC / 4 : LC / 8;   // k-steps of 4 per class per chunk
    constexpr int NCH = SPIN ? 2 : 1;
    constexpr int NCOMP = SPIN ? 2 : 1;
    __shared__ T lam[LC][NCH][SPT];
    __shared__ T bst[2][KS][NCB][64];

    const int lane = threadIdx.x;
    const int i16 = lane & 15, kk = lane >> 4;
    const LegItem it = items[blockIdx.x];
    const int m = it.m, tile = it.tile;
    const int t0 = blockIdx.y * jobs_per_group;
    const int lmax = v.lmax;
    const int l0 = m > SPIN ? m : SPIN;
    const int lstart = l0 - ((l0 + m) & 1);
    const int slot_local = SPIN ? (lane & 31) : lane;
    const int chain = SPIN ? (lane >> 5) : 0;
    const int slot0 = tile * SPT;
    const double4 *coef = v.coef + v.coef_ofs[m];
    const int64_t mbase = (int64_t)m * (2 * (int64_t)lmax + 1 - m) / 2;
    const double thr = ldexp(1.0, v.thresh_bits), down = ldexp(1.0, -v.rescale_bits);

    ChainState cs = chain_init(v, m, slot0 + slot_local, chain);
    bool slow = wave_any(cs.k < 0);

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

    int chunk = 0;
    for (int lc = lstart; lc <= lmax; lc += LC, ++chunk) {
        // (1) coefficient fragments of this chunk: B[kk][j] at lane j + 16 kk
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb) {
                    const int col = i16 + 16 * cb;
                    double val = 0.0;
                    if constexpr (SPIN == 0) {
                        const int l = lc + p + 2 * (4 * ks + kk);
                        const int t = t0 + (col >> 1), reim = col & 1;
                        if (l >= l0 && l <= lmax && t < v.ntrans && !(m == 0 && reim)) {
                            val = alm[(((int64_t)t * v.nalm) + mbase + l) * 2 + reim] * coef[l].z;
                        }
                    } else {
                        const int l = lc + 4 * ks + kk;
                        const int t = t0 + (col >> 2), o = col & 3;
                        if (l >= l0 && l <= lmax && t < v.ntrans) {
                            const double *aE = alm + (((int64_t)t * 2 + 0) * v.nalm + mbase + l) * 2;
                            const double *aB = alm + (((int64_t)t * 2 + 1) * v.nalm + mbase + l) * 2;
                            const bool wrow = ((kk + p) & 1) == 0;
                            double e;
                            if (wrow) {
                                // -(E_re, E_im, B_re, B_im)
                                e = (o == 0) ? -aE[0] : (o == 1) ? -aE[1] : (o == 2) ? -aB[0] : -aB[1];
                                if (m == 0 && (o & 1)) e = 0.0;
                            } else {
                                // (B_im, -B_re, -E_im, E_re)
                                e = (o == 0) ? aB[1] : (o == 1) ? -aB[0] : (o == 2) ? -aE[1] : aE[0];
                                if (m == 0 && (o == 0 || o == 2)) e = 0.0;
                            }
                            val = e * (0.5 * coef[l].z);
                        }
                    }
                    bst[p][ks][cb][lane] = (T)val;
                }
        // (2) recursion over the chunk; lambda (masked by k == 0) into LDS
        for (int t = 0; t < LC; ++t) {
            const int l = lc + t;
            T val = 0;
            if (l >= l0 && l <= lmax && cs.k == 0) val = (T)cs.mu1;
            lam[t][chain][slot_local] = val;
            if (l >= l0 && l < lmax) {
                const double4 cf = coef[l];
                chain_step(cs, cf.x, cf.y);
                if (slow) chain_rescale(cs, thr, down);
            }
        }
        slow = wave_any(cs.k < 0);
        __syncthreads();
        // (3) matrix-core products
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
#pragma unroll
            for (int sb = 0; sb < NSB; ++sb) {
                T a0, a1;
                if constexpr (SPIN == 0) {
                    a0 = lam[0 + 2 * (4 * ks + kk)][0][sb * 16 + i16];
                    a1 = lam[1 + 2 * (4 * ks + kk)][0][sb * 16 + i16];
                } else {
                    const T up = lam[4 * ks + kk][0][sb * 16 + i16];
                    const T um = lam[4 * ks + kk][1][sb * 16 + i16];
                    if (kk & 1) {
                        a0 = up - um;
                        a1 = up + um;
                    } else {
                        a0 = up + um;
                        a1 = up - um;
                    }
                }
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb) {
                    acc[0][sb][cb] = mfma(a0, bst[0][ks][cb][lane], acc[0][sb][cb]);
                    acc[1][sb][cb] = mfma(a1, bst[1][ks][cb][lane], acc[1][sb][cb]);
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
        __syncthreads();
    }

    // epilogue: north = A0 + A1, south = A0 - A1
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
                phase[((rowbase + yn) * (v.mmax + 1) + m) * 2 + reim] = c0 + c1;
                if (ys >= 0) phase[((rowbase + ys) * (v.mmax + 1) + m) * 2 + reim] = c0 - c1;
            }
}

// ---------------------------------------------------------------- analysis

constexpr int ANA_LC = 32;   // degrees per chunk (16 per parity class)

template <int SPIN, int NCB, bool F32>
__global__ __launch_bounds__(64) void k_legendre_anal(LegView v, const int *__restrict__ mlist,
                                                      const double *__restrict__ phase,
                                                      double *__restrict__ alm, int jobs_per_group)
{
    using T = typename MT<F32>::T;
    using V = typename MT<F32>::V;
    constexpr int SPT = SPIN ? 32 : 64;
    constexpr int LC = ANA_LC;
    constexpr int KSA = SPT / 4;       // k-steps (4 slots each) per tile
    constexpr int NCH = SPIN ? 2 : 1;
    constexpr int NCOMP = SPIN ? 2 : 1;
    constexpr int LDP = SPT + 1;       // padded LDS row
    __shared__ T lam[NCH][LC][LDP];

    const int lane = threadIdx.x;
    const int i16 = lane & 15, kk = lane >> 4;
    const int m = mlist[blockIdx.x];
    const int t0 = blockIdx.y * jobs_per_group;
    const int lmax = v.lmax;
    const int l0 = m > SPIN ? m : SPIN;
    const int lstart = l0 - ((l0 + m) & 1);
    const int slot_local = SPIN ? (lane & 31) : lane;
    const int chain = SPIN ? (lane >> 5) : 0;
    const double4 *coef = v.coef + v.coef_ofs[m];
    const int64_t mbase = (int64_t)m * (2 * (int64_t)lmax + 1 - m) / 2;
    const double thr = ldexp(1.0, v.thresh_bits), down = ldexp(1.0, -v.rescale_bits);
    const int ncols = jobs_per_group * (SPIN ? 4 : 2);

    // degrees below l0 (spin 2 with m < 2) are zero by convention
    for (int l = m + lane / ncols; l < l0 && l <= lmax; l += 64 / ncols) {
        const int col = lane % ncols;
        int t, comp, reim;
        if constexpr (SPIN == 0) { t = t0 + (col >> 1); comp = 0; reim = col & 1; }
        else { t = t0 + (col >> 2); comp = (col & 3) >> 1; reim = col & 1; }
        if (t < v.ntrans && lane < (64 / ncols) * ncols)
            alm[(((int64_t)t * NCOMP + comp) * v.nalm + mbase + l) * 2 + reim] = 0.0;
    }

    bool first = true;
    for (int tile = 0; tile < v.ntiles; ++tile) {
        if (v.tile_mlim[tile] < m) continue;
        const int slot0 = tile * SPT;
        // stationary phase fragments: B[kk][j] = Gop[slot 4 ks + kk][col j + 16 cb]
        T gf[2][KSA][NCB];
#pragma unroll
        for (int ks = 0; ks < KSA; ++ks) {
            const int slot = slot0 + 4 * ks + kk;
            int yn = -1, ys = -1;
            if (slot < v.nslots) { yn = v.slot_yn[slot]; ys = v.slot_ys[slot]; }
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                const int col = i16 + 16 * cb;
                int t, comp, reim;
                if constexpr (SPIN == 0) { t = t0 + (col >> 1); comp = 0; reim = col & 1; }
                else { t = t0 + (col >> 2); comp = (col & 3) >> 1; reim = col & 1; }
                double gn = 0.0, gs = 0.0;
                if (yn >= 0 && t < v.ntrans) {
                    const int64_t rowbase = ((int64_t)t * NCOMP + comp) * v.nrings;
                    gn = phase[((rowbase + yn) * (v.mmax + 1) + m) * 2 + reim];
                    if (ys >= 0) gs = phase[((rowbase + ys) * (v.mmax + 1) + m) * 2 + reim];
                }
                const double sgn = SPIN ? -1.0 : 1.0;
                gf[0][ks][cb] = (T)(sgn * (gn + gs));
                gf[1][ks][cb] = (T)(sgn * (gn - gs));
            }
        }
        ChainState cs = chain_init(v, m, slot0 + slot_local, chain);
        bool slow = wave_any(cs.k < 0);
        for (int lc = lstart; lc <= lmax; lc += LC) {
            for (int t = 0; t < LC; ++t) {
                const int l = lc + t;
                T val = 0;
                if (l >= l0 && l <= lmax && cs.k == 0) val = (T)cs.mu1;
                lam[chain][t][slot_local] = val;
                if (l >= l0 && l < lmax) {
                    const double4 cf = coef[l];
                    chain_step(cs, cf.x, cf.y);
                    if (slow) chain_rescale(cs, thr, down);
                }
            }
            slow = wave_any(cs.k < 0);
            __syncthreads();
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                V accW[NCB], accX[SPIN ? NCB : 1];
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb) accW[cb] = V{0, 0, 0, 0};
                if constexpr (SPIN) {
#pragma unroll
                    for (int cb = 0; cb < NCB; ++cb) accX[cb] = V{0, 0, 0, 0};
                }
#pragma unroll
                for (int ks = 0; ks < KSA; ++ks) {
                    // A[i][kk] = Lambda[degree lc + p + 2 i][slot 4 ks + kk]
                    if constexpr (SPIN == 0) {
                        const T a = lam[0][p + 2 * i16][4 * ks + kk];
#pragma unroll
                        for (int cb = 0; cb < NCB; ++cb) accW[cb] = mfma(a, gf[p][ks][cb], accW[cb]);
                    } else {
                        const T up = lam[0][p + 2 * i16][4 * ks + kk];
                        const T um = lam[1][p + 2 * i16][4 * ks + kk];
                        const T aw = up + um, ax = up - um;
#pragma unroll
                        for (int cb = 0; cb < NCB; ++cb) {
                            accW[cb] = mfma(aw, gf[p][ks][cb], accW[cb]);
                            accX[cb] = mfma(ax, gf[1 - p][ks][cb], accX[cb]);
                        }
                    }
                }
                // epilogue of class p: rows are degrees lc + p + 2 i
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = c_row<F32>(lane, r);
                        const int l = lc + p + 2 * row;
                        const int col = i16 + 16 * cb;
                        double val = (double)accW[cb][r];
                        int t, comp, reim;
                        if constexpr (SPIN == 0) {
                            t = t0 + (col >> 1);
                            comp = 0;
                            reim = col & 1;
                        } else {
                            const int o = col & 3;
                            // X part of output o is sigma_o * Xacc[3 - o], sigma = (-,+,+,-)
                            const double xo = (double)__shfl_xor((T)accX[cb][r], 3, 64);
                            val += (o == 0 || o == 3) ? -xo : xo;
                            t = t0 + (col >> 2);
                            comp = o >> 1;
                            reim = o & 1;
                        }
                        if (l < l0 || l > lmax || t >= v.ntrans) continue;
                        val *= SPIN ? 0.5 * coef[l].z : coef[l].z;
                        if (m == 0 && reim) val = 0.0;
                        double *dst = alm + (((int64_t)t * NCOMP + comp) * v.nalm + mbase + l) * 2 + reim;
                        if (first) *dst = val;
                        else *dst += val;
                    }
            }
            __syncthreads();
        }
        first = false;
    }
    if (first) {
        // no active slot for this m: every degree is zero
        for (int l = l0 + lane / ncols; l <= lmax; l += 64 / ncols) {
            const int col = lane % ncols;
            int t, comp, reim;
            if constexpr (SPIN == 0) { t = t0 + (col >> 1); comp = 0; reim = col & 1; }
            else { t = t0 + (col >> 2); comp = (col & 3) >> 1; reim = col & 1; }
            if (t < v.ntrans && lane < (64 / ncols) * ncols)
                alm[(((int64_t)t * NCOMP + comp) * v.nalm + mbase + l) * 2 + reim] = 0.0;
        }
    }
}

// ---------------------------------------------------------------- launchers

static int ncb_for(int spin, int ntrans, bool anal)
{
    const int cols = ntrans * (spin ? 4 : 2);
    int ncb = (cols + 15) / 16;
    const int cap = spin ? 4 : 2;
    (void)anal;
    return ncb > cap ? cap : ncb;
}

template <int SPIN, int NCB, bool F32>
static void launch_synth_t(const Plan &p, const LegView &v, const double *alm, double *phase,
                           hipStream_t s)
{
    const int jpg = NCB * 16 / (SPIN ? 4 : 2);
    dim3 grid((unsigned)p.synth_items.size(), (unsigned)((p.ntrans + jpg - 1) / jpg));
    hipLaunchKernelGGL((k_legendre_synth<SPIN, NCB, F32>), grid, dim3(64), 0, s, v,
                       p.d_synth_items, alm, phase, jpg, p.flush_chunks);
}

template <int SPIN, int NCB, bool F32>
static void launch_anal_t(const Plan &p, const LegView &v, const double *phase, double *alm,
                          hipStream_t s)
{
    const int jpg = NCB * 16 / (SPIN ? 4 : 2);
    dim3 grid((unsigned)(p.mmax + 1), (unsigned)((p.ntrans + jpg - 1) / jpg));
    hipLaunchKernelGGL((k_legendre_anal<SPIN, NCB, F32>), grid, dim3(64), 0, s, v, p.d_anal_ms,
                       phase, alm, jpg);
}

template <bool F32>
static void dispatch_synth(const Plan &p, const LegView &v, const double *alm, double *phase,
                           hipStream_t s)
{
    const int ncb = ncb_for(p.spin, p.ntrans, false);
    if (p.spin == 0) {
        if (ncb == 1) launch_synth_t<0, 1, F32>(p, v, alm, phase, s);
        else launch_synth_t<0, 2, F32>(p, v, alm, phase, s);
    } else {
        if (ncb == 1) launch_synth_t<2, 1, F32>(p, v, alm, phase, s);
        else if (ncb == 2) launch_synth_t<2, 2, F32>(p, v, alm, phase, s);
        else launch_synth_t<2, 4, F32>(p, v, alm, phase, s);
    }
}

template <bool F32>
static void dispatch_anal(const Plan &p, const LegView &v, const double *phase, double *alm,
                          hipStream_t s)
{
    const int ncb = ncb_for(p.spin, p.ntrans, true);
    if (p.spin == 0) {
        if (ncb == 1) launch_anal_t<0, 1, F32>(p, v, phase, alm, s);
        else launch_anal_t<0, 2, F32>(p, v, phase, alm, s);
    } else {
        if (ncb == 1) launch_anal_t<2, 1, F32>(p, v, phase, alm, s);
        else if (ncb == 2) launch_anal_t<2, 2, F32>(p, v, phase, alm, s);
        else launch_anal_t<2, 4, F32>(p, v, phase, alm, s);
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

int launch_legendre_anal(const Plan &p, const double *phase, double *alm, hipStream_t s)
{
    const LegView v = make_leg_view(p);
    if (p.precision == SHT_FP32_MFMA) dispatch_anal<true>(p, v, phase, alm, s);
    else dispatch_anal<false>(p, v, phase, alm, s);
    return check_hip(hipGetLastError(), "legendre analysis launch");
}

}  // namespace sht
