// libsht C ABI: error handling, geometries, plans and the transform drivers.
//
// The transform is computed in two stages (Sect. 2, Eqs. 3-6): the Legendre
// step between a_lm and the per-ring Fourier phases F/G (legendre.hip), and
// per-ring FFTs between the phases and the map pixels (ringfft.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>

#include "sht_internal.h"

namespace sht {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

int check_hip(hipError_t e, const char *what)
{
    if (e == hipSuccess) return SHT_OK;
    set_error("%s: %s", what, hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? SHT_ENOMEM : SHT_EDEVICE;
}

static bool fault_inject_alloc()
{
    const char *v = getenv("SHT_FAULT_INJECT");
    return v && strcmp(v, "alloc") == 0;
}

int dev_alloc(void **ptr, size_t bytes, const char *what)
{
    *ptr = nullptr;
    if (bytes == 0) return SHT_OK;
    if (fault_inject_alloc()) {
        set_error("%s: injected allocation failure (%zu bytes)", what, bytes);
        return SHT_ENOMEM;
    }
    hipError_t e = hipMalloc(ptr, bytes);
    if (e != hipSuccess) {
        *ptr = nullptr;
        (void)hipGetLastError();
        set_error("%s: hipMalloc(%zu) failed: %s", what, bytes, hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? SHT_ENOMEM : SHT_EDEVICE;
    }
    return SHT_OK;
}

void dev_free(void *ptr)
{
    if (ptr) (void)hipFree(ptr);
}

int dev_upload(void *dst, const void *src, size_t bytes, const char *what)
{
    if (bytes == 0) return SHT_OK;
    return check_hip(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice), what);
}

// ------------------------------------------------------------------ geometry

static int validate_rings(int nrings, const double *theta, const int64_t *nphi,
                          const double *phi0, int64_t stride)
{
    if (nrings < 1) { set_error("nrings must be >= 1 (got %d)", nrings); return SHT_EINVAL; }
    if (!theta || !nphi || !phi0) { set_error("theta, nphi and phi0 are required"); return SHT_EINVAL; }
    if (stride < 1) { set_error("stride must be >= 1"); return SHT_EINVAL; }
    for (int i = 0; i < nrings; ++i) {
        if (!(theta[i] >= 0.0 && theta[i] <= M_PI)) {
            set_error("theta[%d] = %g outside [0, pi]", i, theta[i]);
            return SHT_EINVAL;
        }
        if (nphi[i] < 1 || nphi[i] > (int64_t(1) << 24)) {
            set_error("nphi[%d] = %lld outside [1, 2^24]", i, (long long)nphi[i]);
            return SHT_EINVAL;
        }
        if (!std::isfinite(phi0[i])) { set_error("phi0[%d] not finite", i); return SHT_EINVAL; }
    }
    return SHT_OK;
}

static Geom *geom_from(int nrings, const double *theta, const int64_t *nphi, const double *phi0,
                       const double *weight, const int64_t *ofs, int64_t stride)
{
    Geom *g = new (std::nothrow) Geom();
    if (!g) return nullptr;
    g->nrings = nrings;
    g->theta.assign(theta, theta + nrings);
    g->nphi.assign(nphi, nphi + nrings);
    g->phi0.assign(phi0, phi0 + nrings);
    g->has_weight = weight != nullptr;
    if (weight) g->weight.assign(weight, weight + nrings);
    else g->weight.assign(nrings, 0.0);
    g->stride = stride;
    g->ofs.resize(nrings);
    int64_t acc = 0;
    for (int i = 0; i < nrings; ++i) {
        if (ofs) g->ofs[i] = ofs[i];
        else { g->ofs[i] = acc; acc += nphi[i] * stride; }
    }
    int64_t np = 0;
    for (int i = 0; i < nrings; ++i)
        np = std::max(np, g->ofs[i] + (g->nphi[i] - 1) * stride + 1);
    g->npix = np;
    return g;
}

// Gauss-Legendre nodes as colatitudes by Newton's method on P_n(cos t) in
// long double, with weights 2 / ((1 - x^2) P_n'(x)^2).
static void gauss_legendre(int n, std::vector<double> &theta, std::vector<double> &w)
{
    theta.resize(n);
    w.resize(n);
    const long double pi = 3.14159265358979323846264338327950288L;
    int nh = (n + 1) / 2;
    for (int k = 1; k <= nh; ++k) {
        long double t = pi * (4.0L * k - 1.0L) / (4.0L * n + 2.0L);
        long double dp = 0;
        for (int it = 0; it < 100; ++it) {
            long double c = cosl(t);
            long double p0 = 1.0L, p1 = c;
            for (int j = 2; j <= n; ++j) {
                long double p2 = ((2.0L * j - 1.0L) * c * p1 - (j - 1.0L) * p0) / j;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p0 = 1.0L; p1 = c; }
            dp = n * (c * p1 - p0) / (c * c - 1.0L);
            long double step = p1 / (-sinl(t) * dp);
            t -= step;
            if (fabsl(step) < 1e-18L) {
                c = cosl(t);
                p0 = 1.0L; p1 = c;
                for (int j = 2; j <= n; ++j) {
                    long double p2 = ((2.0L * j - 1.0L) * c * p1 - (j - 1.0L) * p0) / j;
                    p0 = p1;
                    p1 = p2;
                }
                if (n == 1) { p0 = 1.0L; p1 = c; }
                dp = n * (c * p1 - p0) / (c * c - 1.0L);
                break;
            }
        }
        long double c = cosl(t);
        long double wk = 2.0L / ((1.0L - c * c) * dp * dp);
        theta[k - 1] = (double)t;
        w[k - 1] = (double)wk;
        theta[n - k] = M_PI - (double)t;
        w[n - k] = (double)wk;
    }
    if (n % 2 == 1) theta[n / 2] = 0.5 * M_PI;
}

}  // namespace sht

using namespace sht;

extern "C" {

const char *sht_last_error(void) { return g_err; }

const char *sht_strerror(int status)
{
    switch (status) {
    case SHT_OK: return "ok";
    case SHT_EINVAL: return "invalid argument";
    case SHT_ENOMEM: return "out of memory";
    case SHT_EDEVICE: return "device error";
    case SHT_EUNSUPPORTED: return "unsupported";
    case SHT_ESTATE: return "invalid object state";
    default: return "unknown status";
    }
}

int64_t sht_alm_index(int lmax, int l, int m)
{
    return (int64_t)m * (2 * (int64_t)lmax + 1 - m) / 2 + l;
}

int64_t sht_nalm(int lmax, int mmax)
{
    if (lmax < 0 || mmax < 0 || mmax > lmax) return 0;
    return (int64_t)(mmax + 1) * (lmax + 1) - (int64_t)mmax * (mmax + 1) / 2;
}

int sht_geom_create(int nrings, const double *theta, const int64_t *nphi, const double *phi0,
                    const double *weight, const int64_t *ofs, int64_t stride, sht_geom **out)
{
    if (!out) { set_error("out is NULL"); return SHT_EINVAL; }
    *out = nullptr;
    int rc = validate_rings(nrings, theta, nphi, phi0, stride);
    if (rc) return rc;
    if (ofs)
        for (int i = 0; i < nrings; ++i)
            if (ofs[i] < 0) { set_error("ofs[%d] < 0", i); return SHT_EINVAL; }
    if (weight)
        for (int i = 0; i < nrings; ++i)
            if (!std::isfinite(weight[i])) { set_error("weight[%d] not finite", i); return SHT_EINVAL; }
    Geom *g = geom_from(nrings, theta, nphi, phi0, weight, ofs, stride);
    if (!g) { set_error("host allocation failed"); return SHT_ENOMEM; }
    *out = reinterpret_cast<sht_geom *>(g);
    return SHT_OK;
}

int sht_geom_gauss(int nrings, int64_t nphi, double phi0, sht_geom **out)
{
    if (!out) { set_error("out is NULL"); return SHT_EINVAL; }
    *out = nullptr;
    if (nrings < 1 || nrings > 65536) { set_error("nrings %d outside [1, 65536]", nrings); return SHT_EINVAL; }
    if (nphi < 1) { set_error("nphi must be >= 1"); return SHT_EINVAL; }
    std::vector<double> th, w;
    gauss_legendre(nrings, th, w);
    std::vector<int64_t> np(nrings, nphi);
    std::vector<double> p0(nrings, phi0), wt(nrings);
    for (int i = 0; i < nrings; ++i) wt[i] = w[i] * (2.0 * M_PI / (double)nphi);
    return sht_geom_create(nrings, th.data(), np.data(), p0.data(), wt.data(), nullptr, 1, out);
}

// Weights of the rules of sht_geom_ecp on [-1, 1] in x = cos theta, from the
// closed-form cosine and sine sums of the interpolatory rules (the sums that
// Waldvogel's FFT method evaluates), in long double.
static void ecp_rule(int n, int kind, std::vector<double> &th, std::vector<double> &w)
{
    const long double pi = 3.14159265358979323846264338327950288L;
    th.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int k = 0; k < n; ++k) {
        long double t = 0.0L, s = 0.0L;
        if (kind == SHT_ECP_FEJER1) {
            t = pi * ((long double)k + 0.5L) / n;
            long double sum = 0.0L;
            for (int j = 1; j <= n / 2; ++j) sum += cosl(2.0L * j * t) / (4.0L * j * j - 1.0L);
            s = (2.0L / n) * (1.0L - 2.0L * sum);
        } else if (kind == SHT_ECP_FEJER2) {
            t = pi * (long double)(k + 1) / (n + 1);
            long double sum = 0.0L;
            for (int j = 1; j <= (n + 1) / 2; ++j) sum += sinl((2.0L * j - 1.0L) * t) / (2.0L * j - 1.0L);
            s = 4.0L * sinl(t) / (n + 1) * sum;
        } else {
            const int N = n - 1;
            t = pi * (long double)k / N;
            long double sum = 0.0L;
            for (int j = 1; j <= N / 2; ++j) {
                const long double b = (2 * j == N) ? 1.0L : 2.0L;
                sum += b * cosl(2.0L * j * t) / (4.0L * j * j - 1.0L);
            }
            const long double c = (k == 0 || k == N) ? 1.0L : 2.0L;
            s = c / N * (1.0L - sum);
        }
        th[k] = (double)t;
        w[k] = (double)s;
    }
}

int sht_geom_ecp(int nrings, int64_t nphi, int kind, double phi0, sht_geom **out)
{
    if (!out) { set_error("out is NULL"); return SHT_EINVAL; }
    *out = nullptr;
    if (kind != SHT_ECP_FEJER1 && kind != SHT_ECP_FEJER2 && kind != SHT_ECP_CC) {
        set_error("unknown ECP kind %d", kind);
        return SHT_EINVAL;
    }
    const int nmin = kind == SHT_ECP_CC ? 2 : 1;
    if (nrings < nmin || nrings > 65536) { set_error("nrings %d outside [%d, 65536]", nrings, nmin); return SHT_EINVAL; }
    if (nphi < 1) { set_error("nphi must be >= 1"); return SHT_EINVAL; }
    std::vector<double> th, w;
    ecp_rule(nrings, kind, th, w);
    std::vector<int64_t> np(nrings, nphi);
    std::vector<double> p0(nrings, phi0), wt(nrings);
    for (int i = 0; i < nrings; ++i) wt[i] = w[i] * (2.0 * M_PI / (double)nphi);
    return sht_geom_create(nrings, th.data(), np.data(), p0.data(), wt.data(), nullptr, 1, out);
}

static bool smooth235(int64_t n)
{
    for (int p : {2, 3, 5})
        while (n % p == 0) n /= p;
    return n == 1;
}

int sht_geom_reduced_gauss(int nrings, int64_t nphi_max, int lmax, int mmax, int spin, double phi0,
                           sht_geom **out)
{
    if (!out) { set_error("out is NULL"); return SHT_EINVAL; }
    *out = nullptr;
    if (nrings < 1 || nrings > 65536) { set_error("nrings %d outside [1, 65536]", nrings); return SHT_EINVAL; }
    if (lmax < 0 || mmax < 0 || mmax > lmax || spin < 0 || spin > lmax) {
        set_error("need 0 <= mmax <= lmax and 0 <= spin <= lmax");
        return SHT_EINVAL;
    }
    if (nphi_max < 1) { set_error("nphi_max must be >= 1"); return SHT_EINVAL; }
    std::vector<double> th, w;
    gauss_legendre(nrings, th, w);
    const double T = std::max(100.0, 0.01 * lmax), sp = (double)spin;
    std::vector<int64_t> np(nrings);
    std::vector<double> p0(nrings, phi0), wt(nrings);
    for (int i = 0; i < nrings; ++i) {
        const double c = fabs(cos(th[i])), st = sin(th[i]);
        int mlim = mmax;
        while (mlim > 0 && sqrt(std::max(0.0, (double)mlim * mlim + sp * sp - 2.0 * mlim * sp * c)) - lmax * st > T)
            --mlim;
        int64_t n = 2 * (int64_t)mlim + 1;
        while (!smooth235(n)) ++n;
        np[i] = std::min(n, nphi_max);
        wt[i] = w[i] * (2.0 * M_PI / (double)np[i]);
    }
    return sht_geom_create(nrings, th.data(), np.data(), p0.data(), wt.data(), nullptr, 1, out);
}

int sht_geom_healpix(int nside, sht_geom **out)
{
    if (!out) { set_error("out is NULL"); return SHT_EINVAL; }
    *out = nullptr;
    if (nside < 1 || nside > 8192) { set_error("nside %d outside [1, 8192]", nside); return SHT_EINVAL; }
    int nr = 4 * nside - 1;
    std::vector<double> th(nr), p0(nr), wt(nr);
    std::vector<int64_t> np(nr);
    for (int i = 1; i <= 2 * nside; ++i) {
        int y = i - 1;
        if (i < nside) {
            th[y] = 2.0 * asin(i / (sqrt(6.0) * nside));
            np[y] = 4 * (int64_t)i;
            p0[y] = M_PI / (4.0 * i);
        } else {
            double z = 4.0 / 3.0 - 2.0 * i / (3.0 * nside);
            th[y] = acos(z);
            np[y] = 4 * (int64_t)nside;
            int s = (i - nside + 1) % 2;
            p0[y] = (M_PI / (2.0 * nside)) * (1.0 - 0.5 * s);
        }
    }
    for (int y = 2 * nside; y < nr; ++y) {
        int yn = nr - 1 - y;
        th[y] = M_PI - th[yn];
        np[y] = np[yn];
        p0[y] = p0[yn];
    }
    th[2 * nside - 1] = 0.5 * M_PI;
    double npix = 12.0 * nside * (double)nside;
    for (int y = 0; y < nr; ++y) wt[y] = 4.0 * M_PI / npix;
    return sht_geom_create(nr, th.data(), np.data(), p0.data(), wt.data(), nullptr, 1, out);
}

static Geom *as_geom(const sht_geom *g)
{
    Geom *G = reinterpret_cast<Geom *>(const_cast<sht_geom *>(g));
    if (!G || G->magic != kGeomMagic) return nullptr;
    return G;
}

int sht_geom_info(const sht_geom *g, int *nrings, int64_t *npix)
{
    Geom *G = as_geom(g);
    if (!G) { set_error("invalid geometry handle"); return SHT_ESTATE; }
    if (nrings) *nrings = G->nrings;
    if (npix) *npix = G->npix;
    return SHT_OK;
}

int sht_geom_rings(const sht_geom *g, double *theta, int64_t *nphi, double *phi0, double *weight,
                   int64_t *ofs)
{
    Geom *G = as_geom(g);
    if (!G) { set_error("invalid geometry handle"); return SHT_ESTATE; }
    size_t n = (size_t)G->nrings;
    if (theta) memcpy(theta, G->theta.data(), n * sizeof(double));
    if (nphi) memcpy(nphi, G->nphi.data(), n * sizeof(int64_t));
    if (phi0) memcpy(phi0, G->phi0.data(), n * sizeof(double));
    if (weight) memcpy(weight, G->weight.data(), n * sizeof(double));
    if (ofs) memcpy(ofs, G->ofs.data(), n * sizeof(int64_t));
    return SHT_OK;
}

void sht_geom_destroy(sht_geom *g)
{
    Geom *G = as_geom(g);
    if (!G) return;
    G->magic = kDeadMagic;
    delete G;
}

}  // extern "C"

// ------------------------------------------------------------------ plans

namespace sht {

static void plan_free_device(Plan *p)
{
    dev_free(p->d_slot_cos); dev_free(p->d_slot_sin);
    dev_free(p->d_slot_chalf); dev_free(p->d_slot_shalf);
    dev_free(p->d_slot_yn); dev_free(p->d_slot_ys);
    dev_free(p->d_coef); dev_free(p->d_fl); dev_free(p->d_coef_ofs); dev_free(p->d_start);
    dev_free(p->d_tile_mlim); dev_free(p->d_synth_items); dev_free(p->d_anal_ms);
    dev_free(p->d_zeros);
    dev_free(p->d_dfac);
    dev_free(p->d_rh);
    dev_free(p->d_phase);
    fft_plan_free(p->fft);
    p->d_slot_cos = p->d_slot_sin = p->d_slot_chalf = p->d_slot_shalf = nullptr;
    p->d_slot_yn = p->d_slot_ys = nullptr;
    p->d_coef = nullptr; p->d_fl = nullptr; p->d_coef_ofs = nullptr; p->d_start = nullptr;
    p->d_tile_mlim = nullptr; p->d_synth_items = nullptr; p->d_anal_ms = nullptr;
    p->d_zeros = nullptr;
    p->d_dfac = nullptr;
    p->d_rh = nullptr;
    p->d_phase = nullptr;
}

// Pair every ring with its mirror at pi - theta (Sect. 4.2 "counterparts on the
// other hemisphere"); unmatched rings form single-ring slots.  Slots are
// ordered from the poles towards the equator (ascending sin theta), so the
// polar-skip boundary of Sect. 3.3 moves monotonically through the tiles.
static void build_slots(Plan &p)
{
    const Geom &g = p.geom;
    std::vector<int> idx(g.nrings);
    for (int i = 0; i < g.nrings; ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(),
                     [&](int a, int b) { return g.theta[a] < g.theta[b]; });
    const double tol = 8.0 * M_PI * 2.220446049250313e-16;
    p.slots.clear();
    auto make = [&](int yn, int ys, double t) {
        SlotHost s;
        s.yn = yn;
        s.ys = ys;
        s.cth = cos(t);
        s.sth = sin(t);
        s.chalf = cos(0.5 * t);
        s.shalf = sin(0.5 * t);
        p.slots.push_back(s);
    };
    // a ring beyond the equator is represented by its mirror colatitude
    auto single = [&](int y) {
        double t = g.theta[y];
        if (t <= 0.5 * M_PI) make(y, -1, t);
        else make(-1, y, M_PI - t);
    };
    int i = 0, j = g.nrings - 1;
    while (i <= j) {
        if (i == j) { single(idx[i]); break; }
        double ti = g.theta[idx[i]], tj = g.theta[idx[j]];
        double d = ti + tj - M_PI;
        if (fabs(d) <= tol && ti <= 0.5 * M_PI) {
            make(idx[i], idx[j], ti);
            ++i;
            --j;
        } else if (d < 0) {
            single(idx[i]);
            ++i;
        } else {
            single(idx[j]);
            --j;
        }
    }
    std::stable_sort(p.slots.begin(), p.slots.end(),
                     [](const SlotHost &a, const SlotHost &b) { return a.sth < b.sth; });
    p.nslots = (int)p.slots.size();
}

// Polar optimisation (Sect. 3.3, Eqs. 7-8): the term (m, ring) is skipped when
// sqrt(m^2 + s^2 - 2 m s cos t) - lmax sin t > T.  For a ring pair the more
// conservative of the two hemispheres and of +-s is used (|cos t|).
static int slot_mlim(const Plan &p, const SlotHost &s)
{
    if (p.polar_T < 0) return p.mmax;
    const double sp = (double)p.spin;
    for (int m = p.mmax; m >= 0; --m) {
        double v = sqrt(std::max(0.0, (double)m * m + sp * sp - 2.0 * m * sp * fabs(s.cth)))
                   - (double)p.lmax * s.sth;
        if (!(v > p.polar_T)) return m;
    }
    return -1;
}

// Per-m recursion coefficients for the rescaled recursion used on the GPU.
//
// With lambda_l = (-1)^m sqrt((2l+1)/4pi) d^l_{-m,s} (Eq. 10) and the
// three-term relation of Eq. 11 (d indices -m and s), lambda obeys
//   lambda_{l+1} = P_l (x + c_l) lambda_l - Q_l lambda_{l-1},
//   P_l = sqrt((2l+3)/(2l+1)) / B_l,  Q_l = sqrt((2l+3)/(2l-1)) A_l / B_l,
//   A_l = sqrt((l^2-m^2)(l^2-s^2)) / (l(2l+1)),
//   B_l = sqrt(((l+1)^2-m^2)((l+1)^2-s^2)) / ((l+1)(2l+1)),
//   c_l = m s / (l(l+1))  (-c_l for the -s chain).
// Writing lambda_l = f_l mu_l with f_{l0} = f_{l0+1} = 1, f_{l+1} = Q_l f_{l-1}
// turns it into mu_{l+1} = (alpha_l x +- beta_l) mu_l - mu_{l-1}, two fused
// multiply-adds per step, alpha_l = P_l f_l / f_{l+1}, beta_l = alpha_l c_l.
// All l-only factors are computed once per m and reused for every ring
// (Sect. 4.1: "re-used for different colatitudes").
static void build_coef(Plan &p, std::vector<double4> &coef, std::vector<double> &fl,
                       std::vector<int64_t> &ofs)
{
    const int s = p.spin;
    ofs.assign(p.mmax + 1, 0);
    int64_t total = 0;
    for (int m = 0; m <= p.mmax; ++m) total += p.lmax + 1 - std::max(m, s);
    coef.assign((size_t)std::max<int64_t>(total, 1), double4{0, 0, 0, 0});
    fl.assign((size_t)std::max<int64_t>(total, 1), 0.0);
    int64_t base = 0;
    for (int m = 0; m <= p.mmax; ++m) {
        const int l0 = std::max(m, s);
        ofs[m] = base - l0;
        const long double mm = m, ss = s;
        long double f_prev = 1.0L, f_cur = 1.0L;   // f_{l-1}, f_l  (l = l0: f_{l0-1} unused)
        for (int l = l0; l <= p.lmax; ++l) {
            const long double L = l, L1 = l + 1;
            long double B = sqrtl((L1 * L1 - mm * mm) * (L1 * L1 - ss * ss)) / (L1 * (2 * L + 1));
            long double P = sqrtl((2 * L + 3) / (2 * L + 1)) / B;
            long double Q = 0.0L;
            if (l > l0) {
                long double A = sqrtl((L * L - mm * mm) * (L * L - ss * ss)) / (L * (2 * L + 1));
                Q = sqrtl((2 * L + 3) / (2 * L - 1)) * A / B;
            }
            long double c = (l > 0) ? mm * ss / (L * L1) : 0.0L;
            long double f_next = (l == l0) ? 1.0L : Q * f_prev;
            long double alpha = P * f_cur / f_next;
            if (l == p.lmax) alpha = 0.0L;
            const long double beta = alpha * c;
            double4 e;
            e.x = (double)alpha;
            e.y = (double)beta;
            // t - 2 = (alpha +- beta - 2) - 2 alpha sin^2(t/2): the small part
            // is formed here in long double, so that near the poles the
            // recursion sees 1 - cos t at full relative precision
            e.z = (double)(alpha + beta - 2.0L);
            e.w = (double)(alpha - beta - 2.0L);
            coef[(size_t)(base + (l - l0))] = e;
            fl[(size_t)(base + (l - l0))] = (double)f_cur;
            f_prev = f_cur;
            f_cur = f_next;
        }
        base += p.lmax + 1 - l0;
    }
}

// Start values lambda_{l0}, l0 = max(m, |s|), from Wigner's formula for the
// extreme index (a single term): for chain sigma in {+s, -s}
//   m >= s:  d^m_{-m,sigma} = sqrt(C(2m, m+sigma)) cos(t/2)^(m-sigma) sin(t/2)^(m+sigma)
//   m <  s:  d^s_{-m, s}  = sqrt(C(2s, s+m)) cos(t/2)^(s-m) sin(t/2)^(s+m)
//            d^s_{-m,-s}  = (-1)^(s-m) sqrt(C(2s, s+m)) cos(t/2)^(s+m) sin(t/2)^(s-m)
// times (-1)^m sqrt((2 l0 + 1)/4pi) (Eq. 10).  K is kept as mantissa/exponent.
// The -s chain carries an extra (-1)^s, so that W = (s_lambda + (-1)^s
// -s_lambda)/2 and X = (s_lambda - (-1)^s -s_lambda)/2 give Q and U with the
// same column maps for every spin (real Q, U: Q - iU = (-1)^s sum -s_a -s_Y).
static void build_start(Plan &p, std::vector<StartCoef> &st)
{
    const int s = p.spin;
    st.assign((size_t)(p.mmax + 1) * 2, StartCoef{});
    const long double inv4pi = 1.0L / (4.0L * 3.14159265358979323846264338327950288L);
    for (int m = 0; m <= p.mmax; ++m) {
        const int l0 = std::max(m, s);
        for (int ch = 0; ch < 2; ++ch) {
            const int sig = (ch == 0) ? s : -s;
            int top, p_, q_, sign = (m & 1) ? -1 : 1;
            if (m >= s) {
                top = m + sig;            // C(2m, m+sigma)
                p_ = m - sig;
                q_ = m + sig;
            } else {
                top = s + m;              // C(2s, s+m)
                if (sig > 0) { p_ = s - m; q_ = s + m; }
                else { p_ = s + m; q_ = s - m; if ((s - m) & 1) sign = -sign; }
            }
            if (ch == 1 && (s & 1)) sign = -sign;
            // C(2 l0, top) as mantissa/exponent, via a product of ratios
            long double mant = 1.0L;
            long e = 0;
            int n = 2 * l0, k = top;
            if (k > n - k) k = n - k;
            for (int i = 1; i <= k; ++i) {
                mant *= (long double)(n - k + i) / (long double)i;
                int d;
                mant = frexpl(mant, &d);
                e += d;
            }
            // K = sqrt((2 l0 + 1)/4pi * C)
            mant *= (2.0L * l0 + 1.0L) * inv4pi;
            {
                int d;
                mant = frexpl(mant, &d);
                e += d;
            }
            if (e & 1) { mant *= 2.0L; e -= 1; }
            mant = sqrtl(mant);
            e /= 2;
            int d;
            mant = frexpl(mant, &d);
            e += d;
            StartCoef sc;
            sc.kmant = (double)mant;
            sc.kexp = (int)e;
            sc.p = p_;
            sc.q = q_;
            sc.sign = sign;
            sc.pad = 0;
            st[(size_t)m * 2 + ch] = sc;
        }
    }
}

// Algorithmic work of the Legendre step (see sht.h): per kept (m, slot, l)
// triple the recursion (4 flops for spin 0: two FMAs; 8 for spin s > 0: two
// chains) plus per transform and ring of the slot 4 (spin 0) / 16 (spin s > 0)
// flops of products; HBM: a_lm + 2 x phases + maps.
static void count_work(Plan &p)
{
    double triples = 0.0;
    for (int t = 0; t < p.ntiles; ++t) {
        int s0 = t * p.slots_per_tile, s1 = std::min(p.nslots, s0 + p.slots_per_tile);
        for (int sl = s0; sl < s1; ++sl) {
            int ml = slot_mlim(p, p.slots[sl]);
            for (int m = 0; m <= ml; ++m) triples += (double)(p.lmax + 1 - std::max(m, p.spin));
        }
    }
    const double r = p.spin ? 10.0 : 4.0, c = p.spin ? 16.0 : 4.0;
    p.flops_synth = triples * (r + c * p.ntrans);
    p.flops_anal = p.flops_synth;
    double alm_b = (double)p.ntrans * p.ncomp * p.nalm * 16.0;
    double ph_b = (double)p.ntrans * p.ncomp * p.geom.nrings * (p.mmax + 1) * 16.0;
    double map_b = (double)p.ntrans * p.ncomp * p.geom.npix * 8.0;
    p.hbm_bytes = alm_b + 2.0 * ph_b + map_b;
}

// Synthesis work items (one wavefront each): (m, active slot tile, transform
// group).  Blocks of four consecutive m go to one accelerator die (work group
// i runs on die i mod NUM_XCD), so that the a_lm of an m and the cache lines
// of its phases stay in one L2; blocks are dealt to the dies greedily by
// cost, and each die's list runs from the longest degree range down.
int build_synth_items(Plan &p)
{
    const int cpj = p.spin ? 4 : 2;
    const int jpg = p.synth_ncb * 16 / cpj;
    const int ngroups = (p.ntrans + jpg - 1) / jpg;
    constexpr int MB = 4;
    std::vector<std::vector<WaveItem>> die(NUM_XCD);
    std::vector<double> load(NUM_XCD, 0.0);
    for (int mb = 0; mb <= p.mmax; mb += MB) {
        std::vector<WaveItem> blk;
        double cost = 0.0;
        for (int m = mb; m < std::min(p.mmax + 1, mb + MB); ++m) {
            const double lrange = (double)(p.lmax + 1 - std::max(m, p.spin));
            for (int t = 0; t < p.ntiles; ++t) {
                if (p.tile_mlim[t] < m) continue;
                for (int gI = 0; gI < ngroups; ++gI) {
                    blk.push_back(WaveItem{m, t, gI * jpg, 0});
                    cost += lrange;
                }
            }
        }
        if (blk.empty()) continue;
        const int d = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[d] += cost;
        die[d].insert(die[d].end(), blk.begin(), blk.end());
    }
    size_t longest = 0;
    for (auto &l : die) longest = std::max(longest, l.size());
    p.synth_items.assign(longest * NUM_XCD, WaveItem{-1, 0, 0, 0});
    for (int d = 0; d < NUM_XCD; ++d)
        for (size_t i = 0; i < die[d].size(); ++i) p.synth_items[i * NUM_XCD + d] = die[d][i];
    p.n_items = (int64_t)p.synth_items.size();
    dev_free(p.d_synth_items);
    p.d_synth_items = nullptr;
    if (p.synth_items.empty()) return SHT_OK;
    int rc;
    if ((rc = dev_alloc((void **)&p.d_synth_items, p.synth_items.size() * sizeof(WaveItem), "item list")))
        return rc;
    return dev_upload(p.d_synth_items, p.synth_items.data(), p.synth_items.size() * sizeof(WaveItem),
                      "upload");
}

static int plan_build(Plan &p)
{
    int rc;
    build_slots(p);
    p.slots_per_tile = p.spin ? 32 : 64;
    p.ntiles = (p.nslots + p.slots_per_tile - 1) / p.slots_per_tile;
    p.tile_mlim.assign(p.ntiles, -1);
    for (int sl = 0; sl < p.nslots; ++sl) {
        int t = sl / p.slots_per_tile;
        p.tile_mlim[t] = std::max(p.tile_mlim[t], slot_mlim(p, p.slots[sl]));
    }
    // slot tables (padded to whole tiles)
    const int ns = p.ntiles * p.slots_per_tile;
    std::vector<double> sc(ns, 0.0), ss(ns, 0.0), sch(ns, 1.0), ssh(ns, 0.0);
    std::vector<int> yn(ns, -1), ys(ns, -1);
    for (int i = 0; i < p.nslots; ++i) {
        sc[i] = p.slots[i].cth; ss[i] = p.slots[i].sth;
        sch[i] = p.slots[i].chalf; ssh[i] = p.slots[i].shalf;
        yn[i] = p.slots[i].yn; ys[i] = p.slots[i].ys;
    }
    if ((rc = dev_alloc((void **)&p.d_slot_cos, ns * sizeof(double), "slot tables"))) return rc;
    if ((rc = dev_alloc((void **)&p.d_slot_sin, ns * sizeof(double), "slot tables"))) return rc;
    if ((rc = dev_alloc((void **)&p.d_slot_chalf, ns * sizeof(double), "slot tables"))) return rc;
    if ((rc = dev_alloc((void **)&p.d_slot_shalf, ns * sizeof(double), "slot tables"))) return rc;
    if ((rc = dev_alloc((void **)&p.d_slot_yn, ns * sizeof(int), "slot tables"))) return rc;
    if ((rc = dev_alloc((void **)&p.d_slot_ys, ns * sizeof(int), "slot tables"))) return rc;
    if ((rc = dev_upload(p.d_slot_cos, sc.data(), ns * sizeof(double), "upload"))) return rc;
    if ((rc = dev_upload(p.d_slot_sin, ss.data(), ns * sizeof(double), "upload"))) return rc;
    if ((rc = dev_upload(p.d_slot_chalf, sch.data(), ns * sizeof(double), "upload"))) return rc;
    if ((rc = dev_upload(p.d_slot_shalf, ssh.data(), ns * sizeof(double), "upload"))) return rc;
    if ((rc = dev_upload(p.d_slot_yn, yn.data(), ns * sizeof(int), "upload"))) return rc;
    if ((rc = dev_upload(p.d_slot_ys, ys.data(), ns * sizeof(int), "upload"))) return rc;

    std::vector<double4> coef;
    std::vector<double> fl;
    std::vector<int64_t> cofs;
    build_coef(p, coef, fl, cofs);
    if ((rc = dev_alloc((void **)&p.d_coef, coef.size() * sizeof(double4), "coefficient table"))) return rc;
    if ((rc = dev_upload(p.d_coef, coef.data(), coef.size() * sizeof(double4), "upload"))) return rc;
    if ((rc = dev_alloc((void **)&p.d_fl, fl.size() * sizeof(double), "coefficient table"))) return rc;
    if ((rc = dev_upload(p.d_fl, fl.data(), fl.size() * sizeof(double), "upload"))) return rc;
    if ((rc = dev_alloc((void **)&p.d_coef_ofs, cofs.size() * sizeof(int64_t), "coefficient table"))) return rc;
    if ((rc = dev_upload(p.d_coef_ofs, cofs.data(), cofs.size() * sizeof(int64_t), "upload"))) return rc;

    std::vector<StartCoef> st;
    build_start(p, st);
    if ((rc = dev_alloc((void **)&p.d_start, st.size() * sizeof(StartCoef), "start table"))) return rc;
    if ((rc = dev_upload(p.d_start, st.data(), st.size() * sizeof(StartCoef), "upload"))) return rc;

    if ((rc = dev_alloc((void **)&p.d_tile_mlim, p.ntiles * sizeof(int), "tile table"))) return rc;
    if ((rc = dev_upload(p.d_tile_mlim, p.tile_mlim.data(), p.ntiles * sizeof(int), "upload"))) return rc;

    {
        const size_t zb = (size_t)2 * (p.lmax + 2) * sizeof(double);
        if ((rc = dev_alloc((void **)&p.d_zeros, zb, "zero operands"))) return rc;
        if ((rc = check_hip(hipMemset(p.d_zeros, 0, zb), "zero operands"))) return rc;
        std::vector<double> df(p.lmax + 2);
        for (int l = 0; l <= p.lmax + 1; ++l) df[l] = (double)sqrtl((long double)l * (long double)(l + 1));
        if ((rc = dev_alloc((void **)&p.d_dfac, df.size() * sizeof(double), "derivative factors"))) return rc;
        if ((rc = dev_upload(p.d_dfac, df.data(), df.size() * sizeof(double), "upload"))) return rc;
    }
    p.synth_ncb = synth_ncb_default(p.spin, p.ntrans, p.precision);
    if ((rc = build_synth_items(p))) return rc;
    p.anal_ms.resize(p.mmax + 1);
    for (int m = 0; m <= p.mmax; ++m) p.anal_ms[m] = m;
    if ((rc = dev_alloc((void **)&p.d_anal_ms, p.anal_ms.size() * sizeof(int), "m list"))) return rc;
    if ((rc = dev_upload(p.d_anal_ms, p.anal_ms.data(), p.anal_ms.size() * sizeof(int), "upload"))) return rc;

    p.phase_elems = (int64_t)p.ntrans * p.ncomp * p.geom.nrings * (p.mmax + 1);
    if ((rc = dev_alloc((void **)&p.d_phase, (size_t)p.phase_elems * 16, "phase workspace"))) return rc;
    if (p.real_h &&
        (rc = dev_alloc((void **)&p.d_rh, (size_t)p.ntrans * p.ncomp * p.nalm * 16, "real harmonics workspace")))
        return rc;

    if ((rc = fft_plan_build(p))) return rc;
    count_work(p);
    return SHT_OK;
}

LegView make_leg_view(const Plan &p)
{
    LegView v;
    v.lmax = p.lmax; v.mmax = p.mmax; v.spin = p.spin; v.ntrans = p.ntrans;
    v.nrings = p.geom.nrings; v.nslots = p.nslots; v.ntiles = p.ntiles;
    v.rescale_bits = p.rescale_bits;
    v.thresh_bits = p.rescale_bits / 2;
    v.polar_T = p.polar_T;
    v.slot_cos = p.d_slot_cos; v.slot_sin = p.d_slot_sin;
    v.slot_chalf = p.d_slot_chalf; v.slot_shalf = p.d_slot_shalf;
    v.slot_yn = p.d_slot_yn; v.slot_ys = p.d_slot_ys;
    v.coef = p.d_coef; v.fl = p.d_fl; v.coef_ofs = p.d_coef_ofs; v.start = p.d_start;
    v.tile_mlim = p.d_tile_mlim;
    v.zeros = p.d_zeros;
    v.dfac = p.d_dfac;
    v.nalm = p.nalm;
    return v;
}

static Plan *as_plan(sht_plan *h)
{
    Plan *p = reinterpret_cast<Plan *>(h);
    if (!p || p->magic != kPlanMagic) return nullptr;
    return p;
}

static bool ranges_overlap(const void *a, size_t na, const void *b, size_t nb)
{
    uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    return a0 < b0 + nb && b0 < a0 + na;
}

int check_exec_args(const Plan *p, int direction, const void *in, const void *out, bool stage_fft,
                    bool stage_leg)
{
    if (direction < 0 || direction >= NUM_DIRECTIONS) {
        set_error("unknown direction %d", direction);
        return SHT_EINVAL;
    }
    if (!in || !out) { set_error("in and out must be device pointers"); return SHT_EINVAL; }
    if (weighted_direction(direction) && !p->geom.has_weight && !stage_leg) {
        set_error("geometry has no ring weights: analysis and its adjoint unavailable");
        return SHT_EINVAL;
    }
    if (deriv_direction(direction) && p->spin != 1) {
        set_error("first-derivative directions need a plan of spin 1 (plan spin %d)", p->spin);
        return SHT_EINVAL;
    }
    const int alm_comp = deriv_direction(direction) ? 1 : p->ncomp;
    const size_t alm_b = (size_t)p->ntrans * alm_comp * p->nalm * 16;
    const size_t map_b = (size_t)p->ntrans * p->ncomp * p->geom.npix * 8;
    const size_t ph_b = (size_t)p->phase_elems * 16;
    size_t in_b, out_b;
    if (synth_direction(direction)) {
        in_b = stage_fft ? ph_b : alm_b;
        out_b = stage_leg ? ph_b : map_b;
    } else {
        in_b = stage_leg ? ph_b : map_b;
        out_b = stage_fft ? ph_b : alm_b;
    }
    if (ranges_overlap(in, in_b, out, out_b)) { set_error("input and output buffers overlap"); return SHT_EINVAL; }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != p->device) {
        (void)hipGetLastError();
        set_error("current device differs from the plan's device %d", p->device);
        return SHT_EDEVICE;
    }
    return SHT_OK;
}

int finish_launch(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return check_hip(e, what);
    return SHT_OK;
}

}  // namespace sht

extern "C" {

int sht_plan_create(const sht_geom *g, int lmax, int mmax, int spin, int ntrans, int precision,
                    const sht_plan_opts *opts, sht_plan **out)
{
    if (!out) { set_error("out is NULL"); return SHT_EINVAL; }
    *out = nullptr;
    Geom *G = as_geom(g);
    if (!G) { set_error("invalid geometry handle"); return SHT_ESTATE; }
    if (lmax < 0 || lmax > 16383) { set_error("lmax %d outside [0, 16383]", lmax); return SHT_EINVAL; }
    if (mmax < 0 || mmax > lmax) { set_error("mmax %d outside [0, lmax=%d]", mmax, lmax); return SHT_EINVAL; }
    if (spin < 0) { set_error("spin must be >= 0"); return SHT_EINVAL; }
    if (spin > lmax) { set_error("spin %d exceeds lmax %d", spin, lmax); return SHT_EINVAL; }
    if (ntrans < 1 || ntrans > 4096) { set_error("ntrans %d outside [1, 4096]", ntrans); return SHT_EINVAL; }
    if (precision != SHT_FP64 && precision != SHT_FP32_MFMA) { set_error("unknown precision %d", precision); return SHT_EINVAL; }
    sht_plan_opts o{};
    if (opts) o = *opts;
    if (o.rescale_bits != 0 && (o.rescale_bits < 64 || o.rescale_bits > 700)) {
        set_error("rescale_bits %d outside [64, 700]", o.rescale_bits);
        return SHT_EINVAL;
    }
    if (o.flush_chunks < 0 || o.flush_chunks > 64) { set_error("flush_chunks outside [0, 64]"); return SHT_EINVAL; }
    if (o.polar_T < 0 || !std::isfinite(o.polar_T)) { set_error("polar_T must be finite and >= 0"); return SHT_EINVAL; }

    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) { (void)hipGetLastError(); set_error("no HIP device"); return SHT_EDEVICE; }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) { (void)hipGetLastError(); set_error("hipGetDeviceProperties failed"); return SHT_EDEVICE; }
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        set_error("device %d is %s; this library is built for gfx950", dev, prop.gcnArchName);
        return SHT_EDEVICE;
    }

    Plan *p = new (std::nothrow) Plan();
    if (!p) { set_error("host allocation failed"); return SHT_ENOMEM; }
    p->device = dev;
    p->lmax = lmax; p->mmax = mmax; p->spin = spin; p->ntrans = ntrans;
    p->precision = precision; p->ncomp = spin ? 2 : 1;
    p->geom = *G;
    p->opts = o;
    p->polar_T = o.no_polar_skip ? -1.0 : (o.polar_T > 0 ? o.polar_T : std::max(100.0, 0.01 * lmax));
    p->rescale_bits = o.rescale_bits ? o.rescale_bits : 256;
    p->flush_chunks = o.flush_chunks ? o.flush_chunks : 4;
    p->real_h = o.real_harmonics != 0;
    p->nalm = sht_nalm(lmax, mmax);
    int rc = plan_build(*p);
    if (rc) {
        plan_free_device(p);
        p->magic = kDeadMagic;
        delete p;
        return rc;
    }
    *out = reinterpret_cast<sht_plan *>(p);
    return SHT_OK;
}

void sht_plan_destroy(sht_plan *h)
{
    Plan *p = as_plan(h);
    if (!p) return;
    (void)hipDeviceSynchronize();
    plan_free_device(p);
    p->magic = kDeadMagic;
    delete p;
}

int sht_execute(sht_plan *h, int direction, const double *in, double *out, void *hip_stream)
{
    Plan *p = as_plan(h);
    if (!p) { set_error("invalid plan handle"); return SHT_ESTATE; }
    int rc = check_exec_args(p, direction, in, out, false, false);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)hip_stream;
    const int acomp = deriv_direction(direction) ? 1 : p->ncomp;
    if (synth_direction(direction)) {
        const double *a = in;
        if (p->real_h) {
            if ((rc = launch_real_harm(*p, in, p->d_rh, acomp, true, s))) return rc;
            a = p->d_rh;
        }
        if ((rc = launch_legendre_synth(*p, a, p->d_phase, deriv_direction(direction), s))) return rc;
        if ((rc = launch_ring_synth(*p, p->d_phase, out, weighted_direction(direction), s))) return rc;
    } else {
        if ((rc = launch_ring_anal(*p, in, p->d_phase, weighted_direction(direction), s))) return rc;
        if ((rc = launch_legendre_anal(*p, p->d_phase, out, anal_mode(direction, p->real_h), s))) return rc;
        if (p->real_h && (rc = launch_real_harm(*p, out, out, acomp, false, s))) return rc;
    }
    return finish_launch("sht_execute");
}

int sht_legendre(sht_plan *h, int direction, const double *in, double *out, void *hip_stream)
{
    Plan *p = as_plan(h);
    if (!p) { set_error("invalid plan handle"); return SHT_ESTATE; }
    int rc = check_exec_args(p, direction, in, out, false, true);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)hip_stream;
    const int acomp = deriv_direction(direction) ? 1 : p->ncomp;
    if (synth_direction(direction)) {
        const double *a = in;
        if (p->real_h) {
            rc = launch_real_harm(*p, in, p->d_rh, acomp, true, s);
            a = p->d_rh;
        }
        if (!rc) rc = launch_legendre_synth(*p, a, out, deriv_direction(direction), s);
        if (!rc) rc = launch_phase_tail_zero(*p, out, s);
    } else {
        rc = launch_legendre_anal(*p, in, out, anal_mode(direction, p->real_h), s);
        if (!rc && p->real_h) rc = launch_real_harm(*p, out, out, acomp, false, s);
    }
    if (rc) return rc;
    return finish_launch("sht_legendre");
}

int sht_ring_fft(sht_plan *h, int direction, const double *in, double *out, void *hip_stream)
{
    Plan *p = as_plan(h);
    if (!p) { set_error("invalid plan handle"); return SHT_ESTATE; }
    int rc = check_exec_args(p, direction, in, out, true, false);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)hip_stream;
    if (synth_direction(direction)) {
        rc = launch_ring_synth(*p, in, out, weighted_direction(direction), s);
    } else {
        rc = launch_ring_anal(*p, in, out, weighted_direction(direction), s);
        if (!rc) rc = launch_phase_tail_zero(*p, out, s);
    }
    if (rc) return rc;
    return finish_launch("sht_ring_fft");
}

int sht_plan_flops(const sht_plan *h, int direction, double *flops, double *hbm_bytes)
{
    Plan *p = as_plan(const_cast<sht_plan *>(h));
    if (!p) { set_error("invalid plan handle"); return SHT_ESTATE; }
    if (flops) *flops = synth_direction(direction) ? p->flops_synth : p->flops_anal;
    if (hbm_bytes) *hbm_bytes = p->hbm_bytes;
    return SHT_OK;
}

int sht_plan_info(const sht_plan *h, int64_t *n_items, int64_t *workspace_bytes)
{
    Plan *p = as_plan(const_cast<sht_plan *>(h));
    if (!p) { set_error("invalid plan handle"); return SHT_ESTATE; }
    if (n_items) *n_items = p->n_items;
    if (workspace_bytes) *workspace_bytes = p->phase_elems * 16 + (int64_t)p->fft.table_bytes;
    return SHT_OK;
}

}  // extern "C"
