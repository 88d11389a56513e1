// libsht host-only code: error reporting, the handle registry, ring geometries
// (Sect. 2; Gauss-Legendre, HEALPix, ECP and reduced Gauss-Legendre grids of
// Sect. 4.4) and the per-plan tables computed on the CPU (ring-pair slots,
// polar limits of Eqs. 7-8, recursion coefficients and start values of
// Sect. 4.1, work counts).  No HIP: this file also builds with g++ alone.
#include "host.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <unordered_map>
#include <utility>

namespace sht {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    if (g_err[0]) log_msg(1, "error: %s", g_err);
}

int log_level()
{
    static const int level = [] {
        const char *v = getenv("SHT_LOG");
        const int n = v ? atoi(v) : 0;
        return n < 0 ? 0 : (n > 3 ? 3 : n);
    }();
    return level;
}

void log_msg(int level, const char *fmt, ...)
{
    if (level > log_level()) return;
    char line[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(line, sizeof(line), fmt, ap);
    va_end(ap);
    static std::mutex mu;
    std::lock_guard<std::mutex> lk(mu);
    fprintf(stderr, "[sht:%d] %s\n", level, line);
}

// ------------------------------------------------------------------ registry

namespace {
std::mutex g_reg_mu;
std::unordered_map<const void *, std::pair<int, uint64_t>> &registry()
{
    static std::unordered_map<const void *, std::pair<int, uint64_t>> r;
    return r;
}
uint64_t g_serial = 0;
}  // namespace

uint64_t reg_add(const void *obj, int kind)
{
    std::lock_guard<std::mutex> lk(g_reg_mu);
    const uint64_t s = ++g_serial;
    registry()[obj] = {kind, s};
    return s;
}

bool reg_live(const void *obj, int kind, uint64_t *serial)
{
    if (!obj) return false;
    std::lock_guard<std::mutex> lk(g_reg_mu);
    auto it = registry().find(obj);
    if (it == registry().end() || it->second.first != kind) return false;
    if (serial) *serial = it->second.second;
    return true;
}

void reg_remove(const void *obj)
{
    std::lock_guard<std::mutex> lk(g_reg_mu);
    registry().erase(obj);
}

// ------------------------------------------------- allocation bookkeeping

namespace {
thread_local int g_fail_at = 0;   // device allocation that fails (0: none)
thread_local int g_alloc_no = 0;  // device allocations of the current create call
std::atomic<int64_t> g_live_buffers{0}, g_live_bytes{0};
}  // namespace

void fault_arm()
{
    g_alloc_no = 0;
    g_fail_at = 0;
    const char *v = getenv("SHT_FAULT_INJECT");
    if (!v || strncmp(v, "alloc", 5) != 0) return;
    g_fail_at = 1;
    if (v[5] == ':') {
        const int n = atoi(v + 6);
        g_fail_at = n > 0 ? n : 1;
    } else if (v[5] != '\0') {
        g_fail_at = 0;
    }
}

bool fault_should_fail()
{
    ++g_alloc_no;
    return g_fail_at > 0 && g_alloc_no == g_fail_at;
}

void mem_count(int64_t buffers, int64_t bytes)
{
    g_live_buffers += buffers;
    g_live_bytes += bytes;
}

void mem_stats(int64_t *buffers, int64_t *bytes)
{
    if (buffers) *buffers = g_live_buffers.load();
    if (bytes) *bytes = g_live_bytes.load();
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
    auto legendre = [n](long double c, long double &pn, long double &pn1) {
        long double p0 = 1.0L, p1 = c;
        for (int j = 2; j <= n; ++j) {
            long double p2 = ((2.0L * j - 1.0L) * c * p1 - (j - 1.0L) * p0) / j;
            p0 = p1;
            p1 = p2;
        }
        if (n == 1) { p0 = 1.0L; p1 = c; }
        pn = p1;
        pn1 = p0;
    };
    int nh = (n + 1) / 2;
    for (int k = 1; k <= nh; ++k) {
        long double t = pi * (4.0L * k - 1.0L) / (4.0L * n + 2.0L);
        long double dp = 0;
        for (int it = 0; it < 100; ++it) {
            long double c = cosl(t), p1, p0;
            legendre(c, p1, p0);
            dp = n * (c * p1 - p0) / (c * c - 1.0L);
            long double step = p1 / (-sinl(t) * dp);
            t -= step;
            if (fabsl(step) < 1e-18L) {
                c = cosl(t);
                legendre(c, p1, p0);
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

static bool smooth235(int64_t n)
{
    for (int p : {2, 3, 5})
        while (n % p == 0) n /= p;
    return n == 1;
}

// ------------------------------------------------------------ plan tables

// Pair every ring with its mirror at pi - theta (Sect. 4.2 "counterparts on the
// other hemisphere"); unmatched rings form single-ring slots.  Slots are
// ordered from the poles towards the equator (ascending sin theta), so the
// polar-skip boundary of Sect. 3.3 moves monotonically through the tiles.
void build_slots(const Geom &g, std::vector<SlotHost> &slots)
{
    std::vector<int> idx(g.nrings);
    for (int i = 0; i < g.nrings; ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return g.theta[a] < g.theta[b]; });
    const double tol = 8.0 * M_PI * 2.220446049250313e-16;
    slots.clear();
    auto make = [&](int yn, int ys, double t) {
        SlotHost s;
        s.yn = yn;
        s.ys = ys;
        s.cth = cos(t);
        s.sth = sin(t);
        s.chalf = cos(0.5 * t);
        s.shalf = sin(0.5 * t);
        slots.push_back(s);
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
    std::stable_sort(slots.begin(), slots.end(),
                     [](const SlotHost &a, const SlotHost &b) { return a.sth < b.sth; });
}

// Polar optimisation (Sect. 3.3, Eqs. 7-8): the term (m, ring) is skipped when
// sqrt(m^2 + s^2 - 2 m s cos t) - lmax sin t > T.  For a ring pair the more
// conservative of the two hemispheres and of +-s is used (|cos t|).
int slot_mlim(const PlanShape &ps, const SlotHost &s)
{
    if (ps.polar_T < 0) return ps.mmax;
    const double sp = (double)ps.spin;
    for (int m = ps.mmax; m >= 0; --m) {
        double v = sqrt(std::max(0.0, (double)m * m + sp * sp - 2.0 * m * sp * fabs(s.cth))) -
                   (double)ps.lmax * s.sth;
        if (!(v > ps.polar_T)) return m;
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
void build_coef(const PlanShape &ps, std::vector<Coef4> &coef, std::vector<double> &fl,
                std::vector<int64_t> &ofs)
{
    const int s = ps.spin;
    ofs.assign(ps.mmax + 1, 0);
    int64_t total = 0;
    for (int m = 0; m <= ps.mmax; ++m) total += ps.lmax + 1 - std::max(m, s);
    coef.assign((size_t)std::max<int64_t>(total, 1), Coef4{0, 0, 0, 0});
    fl.assign((size_t)std::max<int64_t>(total, 1), 0.0);
    int64_t base = 0;
    for (int m = 0; m <= ps.mmax; ++m) {
        const int l0 = std::max(m, s);
        ofs[m] = base - l0;
        const long double mm = m, ss = s;
        long double f_prev = 1.0L, f_cur = 1.0L;   // f_{l-1}, f_l  (l = l0: f_{l0-1} unused)
        for (int l = l0; l <= ps.lmax; ++l) {
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
            if (l == ps.lmax) alpha = 0.0L;
            const long double beta = alpha * c;
            Coef4 e;
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
        base += ps.lmax + 1 - l0;
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
void build_start(const PlanShape &ps, std::vector<StartCoef> &st)
{
    const int s = ps.spin;
    st.assign((size_t)(ps.mmax + 1) * 2, StartCoef{});
    const long double inv4pi = 1.0L / (4.0L * 3.14159265358979323846264338327950288L);
    for (int m = 0; m <= ps.mmax; ++m) {
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

double count_triples(const PlanShape &ps, const std::vector<SlotHost> &slots, int slots_per_tile)
{
    double triples = 0.0;
    const int ns = (int)slots.size();
    for (int s0 = 0; s0 < ns; s0 += slots_per_tile) {
        const int s1 = std::min(ns, s0 + slots_per_tile);
        for (int sl = s0; sl < s1; ++sl) {
            const int ml = slot_mlim(ps, slots[sl]);
            for (int m = 0; m <= ml; ++m) triples += (double)(ps.lmax + 1 - std::max(m, ps.spin));
        }
    }
    return triples;
}

static bool ranges_overlap(const void *a, size_t na, const void *b, size_t nb)
{
    const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    return a0 < b0 + nb && b0 < a0 + na;
}

int validate_exec(int direction, int spin, bool has_weight, size_t alm_b, size_t map_b, size_t ph_b,
                  const void *in, const void *out, bool stage_fft, bool stage_leg)
{
    if (direction < 0 || direction >= NUM_DIRECTIONS) {
        set_error("unknown direction %d", direction);
        return SHT_EINVAL;
    }
    if (!in || !out) { set_error("in and out must be device pointers"); return SHT_EINVAL; }
    if (weighted_direction(direction) && !has_weight && !stage_leg) {
        set_error("geometry has no ring weights: analysis and its adjoint unavailable");
        return SHT_EINVAL;
    }
    if (deriv_direction(direction) && spin != 1) {
        set_error("first-derivative directions need a plan of spin 1 (plan spin %d)", spin);
        return SHT_EINVAL;
    }
    size_t in_b, out_b;
    if (synth_direction(direction)) {
        in_b = stage_fft ? ph_b : alm_b;
        out_b = stage_leg ? ph_b : map_b;
    } else {
        in_b = stage_leg ? ph_b : map_b;
        out_b = stage_fft ? ph_b : alm_b;
    }
    if (ranges_overlap(in, in_b, out, out_b)) { set_error("input and output buffers overlap"); return SHT_EINVAL; }
    return SHT_OK;
}

}  // namespace sht

using namespace sht;

static Geom *as_geom(const sht_geom *g)
{
    if (!reg_live(g, H_GEOM)) return nullptr;
    return reinterpret_cast<Geom *>(const_cast<sht_geom *>(g));
}

namespace sht {
const Geom *geom_of(const sht_geom *g) { return as_geom(g); }
}  // namespace sht

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

int sht_memory_stats(int64_t *live_buffers, int64_t *live_bytes)
{
    mem_stats(live_buffers, live_bytes);
    return SHT_OK;
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
    const uint64_t serial = reg_add(g, H_GEOM);
    log_msg(1, "geometry %llu created: %d rings, %lld pixels, %s", (unsigned long long)serial, g->nrings,
            (long long)g->npix, g->has_weight ? "ring weights" : "no ring weights");
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
    log_msg(1, "geometry destroyed (%d rings)", G->nrings);
    reg_remove(G);
    delete G;
}

}  // extern "C"
