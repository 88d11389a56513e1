/*
 * Plain, slow, CPU reference for spherical harmonic transforms (test
 * infrastructure only: nothing in the product library may link, import or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline use it).
 *
 * What it computes is the plain definition of the transforms of
 * Reinecke & Seljebotn (2013), Sect. 2:
 *   synthesis  p_xy  = sum_{m=-mmax}^{mmax} sum_{l>=|m|} a_lm lambda_lm(theta_y)
 *                      exp(i m phi0_y + 2 pi i m x / Nphi_y)            (Eq. 1)
 *   analysis   a_lm  = sum_y sum_x p_xy w_y lambda_lm(theta_y)
 *                      exp(-i m phi0_y - 2 pi i m x / Nphi_y)           (Eq. 2)
 * split into the Fourier phases F_{m,y} (Eq. 4) and G_{m,y} (Eq. 6), which
 * it can also export.  There is no FFT, no hemisphere symmetry and no polar
 * skipping here: every sum is evaluated term by term.
 *
 * lambda is evaluated as in Sect. 4.1:
 *   s_lambda_lm(theta) = (-1)^m sqrt((2l+1)/(4 pi)) d^l_{-m,s}(theta)   (Eq. 10)
 * with d^l at the lowest degree l0 = max(|m|,|s|) taken from Wigner's
 * explicit sum formula, and all higher degrees from the three-term recursion
 * in l of Eq. 11, run upwards.  As Sect. 4.1 requires, the recursion runs in a
 * number format with an extended exponent: here an x87 long double mantissa
 * (64-bit significand) and a separate 64-bit binary exponent, so that values
 * as small as 2^-50000 are carried exactly and nothing underflows.
 * Accumulations are done in long double as well.
 *
 * Conventions (where the paper is silent, these are the readings used):
 *   - real fields: a_{l,-m} = (-1)^m conj(a_lm); the imaginary part of a_l0
 *     is ignored, and coefficients with l < |s| are ignored (set to zero);
 *   - spin s > 0 uses E/B input and Q/U maps with
 *     +-s_a_lm = -(E_lm +- i B_lm) and Q + iU = sum s_a_lm s_Y_lm; since
 *     -s_Y_lm = (-1)^(s+m) conj(s_Y_l,-m) (from Eq. 10 and the symmetries of
 *     d^l), real Q and U give Q - iU = (-1)^s sum -s_a_lm -s_Y_lm, so the
 *     analysis takes -s_a from Q - iU with the factor (-1)^s (1 for even s);
 *   - Eq. 2's weights w_y include the 2 pi / Nphi_y factor.
 *
 * Layouts (all double precision, complex numbers as (re, im) pairs):
 *   alm  [ntrans][ncomp][nalm][2], index(l,m) = m(2 lmax + 1 - m)/2 + l
 *   map  [ntrans][ncomp][...], pixel x of ring y at ofs[y] + x*stride
 *   phases F or G  [ntrans][ncomp][nrings][mmax+1][2]
 * ncomp is 1 for spin 0 and 2 for spin s > 0 (E,B resp. Q,U).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef long double ld;

/* ------------------------------------------------------------------ */
/* extended-exponent real: value = v * 2^e                               */
/* ------------------------------------------------------------------ */
typedef struct { ld v; int64_t e; } xr;

static xr xr_norm(ld v, int64_t e)
{
    xr r;
    if (v == 0.0L) { r.v = 0.0L; r.e = 0; return r; }
    int d;
    r.v = frexpl(v, &d);
    r.e = e + d;
    return r;
}

static xr xr_from(ld v) { return xr_norm(v, 0); }

static xr xr_mul(xr a, xr b) { return xr_norm(a.v * b.v, a.e + b.e); }

static xr xr_div(xr a, xr b) { return xr_norm(a.v / b.v, a.e - b.e); }

static xr xr_add(xr a, xr b)
{
    if (a.v == 0.0L) return b;
    if (b.v == 0.0L) return a;
    if (a.e < b.e) { xr t = a; a = b; b = t; }
    int64_t d = a.e - b.e;
    ld bv = (d > 20000) ? 0.0L : ldexpl(b.v, (int)-d);
    return xr_norm(a.v + bv, a.e);
}

static xr xr_sqrt(xr a)
{
    if (a.v == 0.0L) return a;
    if (a.e & 1) return xr_norm(sqrtl(a.v * 2.0L), (a.e - 1) / 2);
    return xr_norm(sqrtl(a.v), a.e / 2);
}

/* base^p for a long double base >= 0 and integer p >= 0 (0^0 = 1) */
static xr xr_pow(ld base, int64_t p)
{
    xr r = xr_from(1.0L);
    if (p == 0) return r;
    xr b = xr_from(base);
    if (b.v == 0.0L) return b;
    while (p) {
        if (p & 1) r = xr_mul(r, b);
        p >>= 1;
        if (p) b = xr_mul(b, b);
    }
    return r;
}

static ld xr_to_ld(xr a)
{
    if (a.v == 0.0L) return 0.0L;
    if (a.e < -17000) return 0.0L;
    return ldexpl(a.v, (int)a.e);
}

/* factorials n! for n = 0..nmax, as extended-exponent numbers */
static xr *fact_table(int nmax)
{
    xr *f = (xr *)malloc(sizeof(xr) * (size_t)(nmax + 1));
    if (!f) return NULL;
    f[0] = xr_from(1.0L);
    for (int n = 1; n <= nmax; ++n) f[n] = xr_mul(f[n - 1], xr_from((ld)n));
    return f;
}

/*
 * Wigner small-d element d^j_{mp,mm}(beta) from Wigner's explicit sum:
 *   d^j_{m'm} = sum_k (-1)^(k-m+m') sqrt((j+m')!(j-m')!(j+m)!(j-m)!)
 *               / ((j+m-k)! k! (j-k-m')! (k-m+m')!)
 *               cos(beta/2)^(2j-2k+m-m') sin(beta/2)^(2k-m+m')
 * over all k for which every factorial argument is non-negative.
 * Requires |mp|,|mm| <= j; fact must hold at least 2j+1 entries.
 */
static xr wigner_d_explicit(int j, int mp, int mm, double beta, const xr *fact)
{
    ld c = cosl(0.5L * (ld)beta), s = sinl(0.5L * (ld)beta);
    if (c < 0.0L) c = 0.0L;  /* beta in [0, pi] */
    if (s < 0.0L) s = 0.0L;
    int kmin = 0;
    if (mm - mp > kmin) kmin = mm - mp;
    int kmax = j + mm;
    if (j - mp < kmax) kmax = j - mp;
    xr pre = xr_sqrt(xr_mul(xr_mul(fact[j + mp], fact[j - mp]),
                            xr_mul(fact[j + mm], fact[j - mm])));
    xr sum = xr_from(0.0L);
    for (int k = kmin; k <= kmax; ++k) {
        xr den = xr_mul(xr_mul(fact[j + mm - k], fact[k]),
                        xr_mul(fact[j - k - mp], fact[k - mm + mp]));
        xr t = xr_div(pre, den);
        t = xr_mul(t, xr_pow(c, 2 * j - 2 * k + mm - mp));
        t = xr_mul(t, xr_pow(s, 2 * k - mm + mp));
        if (((k - mm + mp) & 1) != 0) t.v = -t.v;
        sum = xr_add(sum, t);
    }
    return sum;
}

/*
 * s_lambda_lm(theta) for l = 0..lmax (entries with l < max(|m|,|s|) are 0).
 * Eq. 10 with d from Eq. 11 (Kostelec & Rockmore recursion) in the direction
 * of increasing l.  With d indices (m_d, m'_d) = (-m, s), Eq. 11 reads
 *   [cos t - m_d m'_d/(l(l+1))] d^l = A_l d^{l-1} + B_l d^{l+1},
 *   A_l = sqrt((l^2-m_d^2)(l^2-m'_d^2)) / (l(2l+1)),
 *   B_l = sqrt(((l+1)^2-m_d^2)((l+1)^2-m'_d^2)) / ((l+1)(2l+1)).
 * out must hold lmax+1 doubles.  Returns 0, or -1 on bad arguments.
 */
static int lambda_column(int lmax, int m, int s, double theta, const xr *fact,
                         double *out)
{
    int am = m < 0 ? -m : m, as = s < 0 ? -s : s;
    int l0 = am > as ? am : as;
    for (int l = 0; l <= lmax; ++l) out[l] = 0.0;
    if (l0 > lmax) return 0;
    const int md = -m, mpd = s;
    const ld x = cosl((ld)theta);
    xr dprev = xr_from(0.0L);
    xr dcur = wigner_d_explicit(l0, md, mpd, theta, fact);
    const ld sgn = (am & 1) ? -1.0L : 1.0L;     /* (-1)^m */
    const ld inv4pi = 1.0L / (4.0L * 3.14159265358979323846264338327950288L);
    for (int l = l0; l <= lmax; ++l) {
        ld norm = sgn * sqrtl((2.0L * l + 1.0L) * inv4pi);
        out[l] = (double)(norm * xr_to_ld(dcur));
        if (l == lmax) break;
        ld ll = (ld)l, l1 = (ld)(l + 1);
        ld cfac = x;
        if (l > 0) cfac -= (ld)md * (ld)mpd / (ll * l1);
        ld A = 0.0L;
        if (l > 0) {
            ld p = (ll * ll - (ld)md * md) * (ll * ll - (ld)mpd * mpd);
            A = (p > 0.0L) ? sqrtl(p) / (ll * (2.0L * ll + 1.0L)) : 0.0L;
        }
        ld B = sqrtl((l1 * l1 - (ld)md * md) * (l1 * l1 - (ld)mpd * mpd))
               / (l1 * (2.0L * ll + 1.0L));
        xr t = xr_mul(dcur, xr_from(cfac));
        xr u = xr_mul(dprev, xr_from(-A));
        xr dnext = xr_div(xr_add(t, u), xr_from(B));
        dprev = dcur;
        dcur = dnext;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* public helpers                                                        */
/* ------------------------------------------------------------------ */

int64_t oracle_alm_index(int lmax, int l, int m)
{
    return (int64_t)m * (2 * (int64_t)lmax + 1 - m) / 2 + l;
}

int64_t oracle_nalm(int lmax, int mmax)
{
    /* index of the (non-existent) first entry l = m = mmax + 1 */
    return oracle_alm_index(lmax, mmax + 1, mmax + 1);
}

/* s_lambda_lm(theta) for l = 0..lmax into out[lmax+1]; any m, s. */
int oracle_lambda(int lmax, int m, int s, double theta, double *out)
{
    int am = m < 0 ? -m : m, as = s < 0 ? -s : s;
    if (lmax < 0 || am > lmax + 1000000 || as > lmax) return -1;
    int l0 = am > as ? am : as;
    xr *fact = fact_table(2 * (l0 > lmax ? l0 : lmax) + 2);
    if (!fact) return -2;
    int rc = lambda_column(lmax, m, s, theta, fact, out);
    free(fact);
    return rc;
}

/* Wigner d^j_{mp,mm}(beta) (explicit sum), as a double; for tests. */
double oracle_wigner_d(int j, int mp, int mm, double beta)
{
    if (j < 0 || mp > j || -mp > j || mm > j || -mm > j) return NAN;
    xr *fact = fact_table(2 * j + 2);
    if (!fact) return NAN;
    xr d = wigner_d_explicit(j, mp, mm, beta, fact);
    free(fact);
    return (double)xr_to_ld(d);
}

/* complex long double helpers (kept explicit for readability) */
typedef struct { ld re, im; } cld;

static cld cmul(cld a, cld b)
{
    cld r = { a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re };
    return r;
}

/* The (conjugate-symmetric) coefficient of a real field at (l, m), m may be
   negative: a_{l,-m} = (-1)^m conj(a_lm); Im(a_l0) is dropped. */
static cld coef_real_field(const double *a, int lmax, int l, int m)
{
    int am = m < 0 ? -m : m;
    const double *p = a + 2 * oracle_alm_index(lmax, l, am);
    cld c = { (ld)p[0], (ld)p[1] };
    if (am == 0) c.im = 0.0L;
    if (m < 0) {
        c.im = -c.im;
        if (am & 1) { c.re = -c.re; c.im = -c.im; }
    }
    return c;
}

/*
 * Synthesis (Eq. 1 via Eqs. 3-4), evaluated directly.
 * nsel/sel: ring subset to evaluate (sel == NULL: all rings).  Only the map
 * pixels of those rings (and only those F rows) are written.
 * F (optional, may be NULL) receives the per-component real-field phases
 *   F^c_{m,y}, m = 0..mmax, such that map_c(x,y) = sum_{m=-mmax}^{mmax}
 *   F^c_{m,y} e^{i m (phi0 + 2 pi x / Nphi)} with F^c_{-m} = conj(F^c_m)
 * (for spin 0 this is exactly Eq. 4; for spin 2 it is the split of the
 * complex Q+iU phase into its Q and U parts).
 */
int oracle_synthesis(int nrings, const double *theta, const int64_t *nphi,
                     const double *phi0, const int64_t *ofs, int64_t stride,
                     int lmax, int mmax, int spin, int ntrans,
                     const double *alm, double *map, int nsel, const int *sel,
                     double *F)
{
    if (lmax < 0 || mmax < 0 || mmax > lmax || spin < 0 || spin > lmax || ntrans < 1 || nrings < 1)
        return -1;
    const int ncomp = spin ? 2 : 1;
    const int64_t nalm = oracle_nalm(lmax, mmax);
    const int nr = sel ? nsel : nrings;
    int64_t npix_max = 0;
    for (int y = 0; y < nrings; ++y) if (nphi[y] > npix_max) npix_max = nphi[y];
    int64_t map_size = 0;  /* per (trans, comp): max pixel index + 1 */
    for (int y = 0; y < nrings; ++y) {
        int64_t last = ofs[y] + (nphi[y] - 1) * stride + 1;
        if (last > map_size) map_size = last;
    }
    xr *fact = fact_table(2 * lmax + 4);
    if (!fact) return -2;
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int iy = 0; iy < nr; ++iy) {
        int y = sel ? sel[iy] : iy;
        const int64_t N = nphi[y];
        double *lam = (double *)malloc(sizeof(double) * (size_t)(lmax + 1));
        /* ph[t][c][m + mmax]: the Eq. 4 phase of the field (complex) */
        cld *ph = (cld *)calloc((size_t)ntrans * ncomp * (2 * mmax + 1), sizeof(cld));
        ld *ctab = (ld *)malloc(sizeof(ld) * (size_t)N);
        ld *stab = (ld *)malloc(sizeof(ld) * (size_t)N);
        if (!lam || !ph || !ctab || !stab) {
#pragma omp atomic write
            err = -2;
            free(lam); free(ph); free(ctab); free(stab);
            continue;
        }
        for (int m = -mmax; m <= mmax; ++m) {
            if (spin == 0) {
                lambda_column(lmax, m, 0, theta[y], fact, lam);
                for (int t = 0; t < ntrans; ++t) {
                    const double *a = alm + (size_t)t * nalm * 2;
                    cld acc = { 0.0L, 0.0L };
                    int am = m < 0 ? -m : m;
                    for (int l = am; l <= lmax; ++l) {
                        cld c = coef_real_field(a, lmax, l, m);
                        acc.re += c.re * lam[l];
                        acc.im += c.im * lam[l];
                    }
                    ph[(size_t)t * (2 * mmax + 1) + (m + mmax)] = acc;
                }
            } else {
                /* Q + iU = sum_m sum_l s_a_lm s_lambda_lm e^{i m phi},
                   s_a_lm = -(E_lm + i B_lm) */
                lambda_column(lmax, m, spin, theta[y], fact, lam);
                for (int t = 0; t < ntrans; ++t) {
                    const double *aE = alm + ((size_t)t * 2 + 0) * nalm * 2;
                    const double *aB = alm + ((size_t)t * 2 + 1) * nalm * 2;
                    cld acc = { 0.0L, 0.0L };
                    int am = m < 0 ? -m : m;
                    int lstart = am > spin ? am : spin;
                    for (int l = lstart; l <= lmax; ++l) {
                        cld e = coef_real_field(aE, lmax, l, m);
                        cld b = coef_real_field(aB, lmax, l, m);
                        /* -(e + i b) */
                        ld re = -(e.re - b.im), im = -(e.im + b.re);
                        acc.re += re * lam[l];
                        acc.im += im * lam[l];
                    }
                    /* stored in component slot 0 as the complex Q+iU phase */
                    ph[((size_t)t * ncomp) * (2 * mmax + 1) + (m + mmax)] = acc;
                }
            }
        }
        /* optional export of real-field phases per component, m >= 0 */
        if (F) {
            for (int t = 0; t < ntrans; ++t) {
                for (int m = 0; m <= mmax; ++m) {
                    if (spin == 0) {
                        cld p = ph[(size_t)t * (2 * mmax + 1) + (m + mmax)];
                        double *o = F + ((((size_t)t * nrings) + y) * (mmax + 1) + m) * 2;
                        o[0] = (double)p.re; o[1] = (double)p.im;
                    } else {
                        const cld *P = ph + ((size_t)t * ncomp) * (2 * mmax + 1);
                        cld pp = P[m + mmax], pm = P[-m + mmax];
                        /* F^Q_m = (P_m + conj(P_-m))/2, F^U_m = (P_m - conj(P_-m))/(2i) */
                        cld fq = { 0.5L * (pp.re + pm.re), 0.5L * (pp.im - pm.im) };
                        cld d = { 0.5L * (pp.re - pm.re), 0.5L * (pp.im + pm.im) };
                        cld fu = { d.im, -d.re };
                        double *oq = F + (((((size_t)t * 2 + 0) * nrings) + y) * (mmax + 1) + m) * 2;
                        double *ou = F + (((((size_t)t * 2 + 1) * nrings) + y) * (mmax + 1) + m) * 2;
                        oq[0] = (double)fq.re; oq[1] = (double)fq.im;
                        ou[0] = (double)fu.re; ou[1] = (double)fu.im;
                    }
                }
            }
        }
        /* direct DFT of Eq. 3 with integer-reduced twiddles:
           p_x = sum_m (P_m e^{i m phi0}) e^{2 pi i ((m x) mod N) / N} */
        const ld twopi = 2.0L * 3.14159265358979323846264338327950288L;
        for (int64_t k = 0; k < N; ++k) {
            ctab[k] = cosl(twopi * (ld)k / (ld)N);
            stab[k] = sinl(twopi * (ld)k / (ld)N);
        }
        cld *pr = (cld *)malloc(sizeof(cld) * (size_t)(2 * mmax + 1));
        for (int t = 0; t < ntrans; ++t) {
            const cld *P = ph + ((size_t)t * ncomp) * (2 * mmax + 1);
            for (int m = -mmax; m <= mmax; ++m) {
                ld ang = (ld)m * (ld)phi0[y];
                cld e0 = { cosl(ang), sinl(ang) };
                pr[m + mmax] = cmul(P[m + mmax], e0);
            }
            for (int64_t x = 0; x < N; ++x) {
                cld acc = { 0.0L, 0.0L };
                for (int m = -mmax; m <= mmax; ++m) {
                    int64_t k = ((int64_t)m * x) % N;
                    if (k < 0) k += N;
                    const cld c = pr[m + mmax];
                    acc.re += c.re * ctab[k] - c.im * stab[k];
                    acc.im += c.re * stab[k] + c.im * ctab[k];
                }
                int64_t pix = ofs[y] + x * stride;
                if (spin == 0) {
                    map[(size_t)t * map_size + pix] = (double)acc.re;
                } else {
                    map[((size_t)t * 2 + 0) * map_size + pix] = (double)acc.re;
                    map[((size_t)t * 2 + 1) * map_size + pix] = (double)acc.im;
                }
            }
        }
        free(pr);
        free(lam); free(ph); free(ctab); free(stab);
    }
    free(fact);
    (void)npix_max;
    return err;
}

/*
 * Analysis (Eq. 2 via Eqs. 5-6), evaluated directly, for the m values in
 * msel (NULL: all m = 0..mmax).  Only those a_lm are written.
 * wgt: ring weights w_y (pass all ones for the adjoint synthesis Y^T).
 * G (optional) receives G^c_{m,y} = w_y sum_x p^c_xy e^{-i m phi} for each
 * map component c (all rings, the selected m only).
 * For spin s > 0: s_a_lm = sum_y sum_x w_y (Q + iU) s_lambda_lm e^{-i m phi},
 * -s_a_lm = (-1)^s sum_y sum_x w_y (Q - iU) -s_lambda_lm e^{-i m phi},
 * E = -(s_a + -s_a)/2, B = i (s_a - -s_a)/2.
 */
int oracle_analysis(int nrings, const double *theta, const int64_t *nphi,
                    const double *phi0, const double *wgt, const int64_t *ofs,
                    int64_t stride, int lmax, int mmax, int spin, int ntrans,
                    const double *map, double *alm, int nsel, const int *msel,
                    double *G)
{
    if (lmax < 0 || mmax < 0 || mmax > lmax || spin < 0 || spin > lmax || ntrans < 1 || nrings < 1)
        return -1;
    const int ncomp = spin ? 2 : 1;
    const int64_t nalm = oracle_nalm(lmax, mmax);
    const int nm = msel ? nsel : mmax + 1;
    int64_t map_size = 0;
    for (int y = 0; y < nrings; ++y) {
        int64_t last = ofs[y] + (nphi[y] - 1) * stride + 1;
        if (last > map_size) map_size = last;
    }
    xr *fact = fact_table(2 * lmax + 4);
    if (!fact) return -2;
    int err = 0;
    const ld twopi = 2.0L * 3.14159265358979323846264338327950288L;
#pragma omp parallel for schedule(dynamic, 1)
    for (int im = 0; im < nm; ++im) {
        int m = msel ? msel[im] : im;
        /* g[t][c][y]: Eq. 6 phase of map component c at this m */
        cld *g = (cld *)calloc((size_t)ntrans * ncomp * nrings, sizeof(cld));
        double *lam = (double *)malloc(sizeof(double) * (size_t)(lmax + 1));
        if (!g || !lam) {
#pragma omp atomic write
            err = -2;
            free(g); free(lam);
            continue;
        }
        for (int y = 0; y < nrings; ++y) {
            const int64_t N = nphi[y];
            ld ang0 = -(ld)m * (ld)phi0[y];
            cld e0 = { cosl(ang0), sinl(ang0) };
            /* e^{-2 pi i m x / N} for x = 0..N-1, by the integer-reduced angle */
            ld *cx = (ld *)malloc(sizeof(ld) * (size_t)N);
            ld *sx = (ld *)malloc(sizeof(ld) * (size_t)N);
            for (int64_t x = 0; x < N; ++x) {
                int64_t k = ((int64_t)m * x) % N;
                ld a = -twopi * (ld)k / (ld)N;
                cx[x] = cosl(a);
                sx[x] = sinl(a);
            }
            for (int t = 0; t < ntrans; ++t) {
                for (int c = 0; c < ncomp; ++c) {
                    const double *mp = map + ((size_t)t * ncomp + c) * map_size;
                    cld acc = { 0.0L, 0.0L };
                    for (int64_t x = 0; x < N; ++x) {
                        ld v = (ld)mp[ofs[y] + x * stride];
                        acc.re += v * cx[x];
                        acc.im += v * sx[x];
                    }
                    acc = cmul(acc, e0);
                    acc.re *= (ld)wgt[y];
                    acc.im *= (ld)wgt[y];
                    g[((size_t)t * ncomp + c) * nrings + y] = acc;
                    if (G) {
                        double *o = G + (((((size_t)t * ncomp + c) * nrings) + y) * (mmax + 1) + m) * 2;
                        o[0] = (double)acc.re; o[1] = (double)acc.im;
                    }
                }
            }
            free(cx);
            free(sx);
        }
        if (spin == 0) {
            cld *acc = (cld *)calloc((size_t)ntrans * (lmax + 1), sizeof(cld));
            for (int y = 0; y < nrings; ++y) {
                lambda_column(lmax, m, 0, theta[y], fact, lam);
                for (int t = 0; t < ntrans; ++t) {
                    cld gv = g[(size_t)t * nrings + y];
                    for (int l = m; l <= lmax; ++l) {
                        acc[(size_t)t * (lmax + 1) + l].re += gv.re * lam[l];
                        acc[(size_t)t * (lmax + 1) + l].im += gv.im * lam[l];
                    }
                }
            }
            for (int t = 0; t < ntrans; ++t)
                for (int l = m; l <= lmax; ++l) {
                    double *o = alm + ((size_t)t * nalm + oracle_alm_index(lmax, l, m)) * 2;
                    o[0] = (double)acc[(size_t)t * (lmax + 1) + l].re;
                    o[1] = (m == 0) ? 0.0 : (double)acc[(size_t)t * (lmax + 1) + l].im;
                }
            free(acc);
        } else {
            /* sp[t][l] = s_a_lm, sm[t][l] = -s_a_lm */
            cld *sp = (cld *)calloc((size_t)ntrans * (lmax + 1), sizeof(cld));
            cld *sm = (cld *)calloc((size_t)ntrans * (lmax + 1), sizeof(cld));
            int lstart = m > spin ? m : spin;
            const ld sfac = (spin & 1) ? -1.0L : 1.0L;   /* (-1)^s for the -s part */
            for (int sg = -1; sg <= 1; sg += 2) {
                cld *dst = sg > 0 ? sp : sm;
                for (int y = 0; y < nrings; ++y) {
                    lambda_column(lmax, m, spin * sg, theta[y], fact, lam);
                    if (sg < 0)
                        for (int l = 0; l <= lmax; ++l) lam[l] = (double)(sfac * lam[l]);
                    for (int t = 0; t < ntrans; ++t) {
                        cld q = g[((size_t)t * 2 + 0) * nrings + y];
                        cld u = g[((size_t)t * 2 + 1) * nrings + y];
                        /* phase of Q + i sg U */
                        cld v = { q.re - sg * u.im, q.im + sg * u.re };
                        for (int l = lstart; l <= lmax; ++l) {
                            dst[(size_t)t * (lmax + 1) + l].re += v.re * lam[l];
                            dst[(size_t)t * (lmax + 1) + l].im += v.im * lam[l];
                        }
                    }
                }
            }
            for (int t = 0; t < ntrans; ++t)
                for (int l = m; l <= lmax; ++l) {
                    double *oE = alm + (((size_t)t * 2 + 0) * nalm + oracle_alm_index(lmax, l, m)) * 2;
                    double *oB = alm + (((size_t)t * 2 + 1) * nalm + oracle_alm_index(lmax, l, m)) * 2;
                    if (l < spin) { oE[0] = oE[1] = oB[0] = oB[1] = 0.0; continue; }
                    cld p = sp[(size_t)t * (lmax + 1) + l], q = sm[(size_t)t * (lmax + 1) + l];
                    /* E = -(p + q)/2 ; B = i (p - q)/2 */
                    ld Ere = -0.5L * (p.re + q.re), Eim = -0.5L * (p.im + q.im);
                    ld Bre = -0.5L * (p.im - q.im), Bim = 0.5L * (p.re - q.re);
                    oE[0] = (double)Ere; oE[1] = (m == 0) ? 0.0 : (double)Eim;
                    oB[0] = (double)Bre; oB[1] = (m == 0) ? 0.0 : (double)Bim;
                }
            free(sp); free(sm);
        }
        free(g); free(lam);
    }
    free(fact);
    return err;
}
