// Host-code driver for the AddressSanitizer / UndefinedBehaviorSanitizer build:
// exercises the library's host-only code (geometries, handle registry, plan
// tables, argument validation) and the CPU oracle on small cases, including
// invalid and degenerate arguments.  Built and run by
// tests/test_sanitizers_cpu.py with g++/gcc -fsanitize=address,undefined; any
// sanitizer report or failed check ends it with a non-zero status.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../paper_1303_4945_amd/csrc/host.h"

extern "C" {
int oracle_lambda(int lmax, int m, int s, double theta, double *out);
double oracle_wigner_d(int j, int mp, int mm, double beta);
int oracle_synthesis(int nrings, const double *theta, const int64_t *nphi, const double *phi0,
                     const int64_t *ofs, int64_t stride, int lmax, int mmax, int spin, int ntrans,
                     const double *alm, double *map, int nsel, const int *sel, double *F);
int oracle_analysis(int nrings, const double *theta, const int64_t *nphi, const double *phi0,
                    const double *wgt, const int64_t *ofs, int64_t stride, int lmax, int mmax, int spin,
                    int ntrans, const double *map, double *alm, int nsel, const int *msel, double *G);
}

static int failures = 0;
#define CHECK(c)                                                             \
    do {                                                                     \
        if (!(c)) {                                                          \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++failures;                                                      \
        }                                                                    \
    } while (0)

struct Rings {
    std::vector<double> theta, phi0, weight;
    std::vector<int64_t> nphi, ofs;
    int n = 0;
    int64_t npix = 0;
};

static Rings rings_of(sht_geom *g)
{
    Rings r;
    CHECK(sht_geom_info(g, &r.n, &r.npix) == SHT_OK);
    r.theta.resize(r.n);
    r.phi0.resize(r.n);
    r.weight.resize(r.n);
    r.nphi.resize(r.n);
    r.ofs.resize(r.n);
    CHECK(sht_geom_rings(g, r.theta.data(), r.nphi.data(), r.phi0.data(), r.weight.data(), r.ofs.data()) ==
          SHT_OK);
    return r;
}

static void check_tables(const sht::Geom &geom, int lmax, int mmax, int spin, double T)
{
    sht::PlanShape ps;
    ps.lmax = lmax;
    ps.mmax = mmax;
    ps.spin = spin;
    ps.polar_T = T;
    std::vector<sht::SlotHost> slots;
    sht::build_slots(geom, slots);
    int covered = 0;
    for (const auto &s : slots) {
        covered += (s.yn >= 0) + (s.ys >= 0);
        CHECK(s.cth >= 0.0 && s.sth >= 0.0);
        const int ml = sht::slot_mlim(ps, s);
        CHECK(ml >= -1 && ml <= mmax);
    }
    CHECK(covered == geom.nrings);
    std::vector<sht::Coef4> coef;
    std::vector<double> fl;
    std::vector<int64_t> ofs;
    sht::build_coef(ps, coef, fl, ofs);
    for (const auto &c : coef) CHECK(std::isfinite(c.x) && std::isfinite(c.y) && std::isfinite(c.z));
    for (double f : fl) CHECK(std::isfinite(f));
    std::vector<sht::StartCoef> st;
    sht::build_start(ps, st);
    CHECK((int)st.size() == 2 * (mmax + 1));
    for (const auto &s : st) CHECK(s.kmant >= 0.5 && s.kmant < 1.0 && (s.sign == 1 || s.sign == -1));
    const double kept = sht::count_triples(ps, slots, spin ? 32 : 64);
    ps.polar_T = -1.0;
    const double full = sht::count_triples(ps, slots, spin ? 32 : 64);
    CHECK(kept <= full && kept >= 0.0);
}

static void geometries()
{
    sht_geom *g = nullptr;
    for (int n : {1, 2, 3, 7, 64}) {
        CHECK(sht_geom_gauss(n, 2 * n + 1, 0.1, &g) == SHT_OK);
        Rings r = rings_of(g);
        double wsum = 0;
        for (int i = 0; i < r.n; ++i) wsum += r.weight[i] * (double)r.nphi[i];
        CHECK(std::fabs(wsum - 4.0 * M_PI) < 1e-12);
        const sht::Geom *G = reinterpret_cast<const sht::Geom *>(g);
        for (int spin : {0, 1, 2}) {
            const int lmax = std::max(n - 1, spin);
            check_tables(*G, lmax, lmax, spin, 100.0);
            check_tables(*G, lmax, lmax / 2, spin, -1.0);
        }
        sht_geom_destroy(g);
        // the destroyed handle is rejected without being read
        CHECK(sht_geom_info(g, nullptr, nullptr) == SHT_ESTATE);
        sht_geom_destroy(g);
    }
    for (int nside : {1, 2, 4}) {
        CHECK(sht_geom_healpix(nside, &g) == SHT_OK);
        Rings r = rings_of(g);
        CHECK(r.npix == 12 * nside * nside);
        check_tables(*reinterpret_cast<const sht::Geom *>(g), 3 * nside - 1, 3 * nside - 1, 1, 100.0);
        sht_geom_destroy(g);
    }
    for (int kind : {SHT_ECP_FEJER1, SHT_ECP_FEJER2, SHT_ECP_CC})
        for (int n : {2, 3, 8}) {
            CHECK(sht_geom_ecp(n, 2 * n, kind, 0.0, &g) == SHT_OK);
            Rings r = rings_of(g);
            double wsum = 0;
            for (int i = 0; i < r.n; ++i) wsum += r.weight[i] * (double)r.nphi[i];
            CHECK(std::fabs(wsum - 4.0 * M_PI) < 1e-12);
            sht_geom_destroy(g);
        }
    CHECK(sht_geom_reduced_gauss(64, 127, 63, 63, 2, 0.0, &g) == SHT_OK);
    check_tables(*reinterpret_cast<const sht::Geom *>(g), 63, 63, 2, 100.0);
    sht_geom_destroy(g);

    // invalid arguments: status, no object
    const double th[2] = {0.5, 4.0};
    const int64_t np[2] = {4, 4}, np0[2] = {4, 0}, ofs[2] = {0, 10};
    const double p0[2] = {0.0, 0.0};
    CHECK(sht_geom_create(2, th, np, p0, nullptr, nullptr, 1, &g) == SHT_EINVAL && g == nullptr);
    const double th2[2] = {0.5, 1.0};
    CHECK(sht_geom_create(2, th2, np0, p0, nullptr, nullptr, 1, &g) == SHT_EINVAL);
    CHECK(sht_geom_create(2, th2, np, p0, nullptr, nullptr, 0, &g) == SHT_EINVAL);
    CHECK(sht_geom_create(0, th2, np, p0, nullptr, nullptr, 1, &g) == SHT_EINVAL);
    CHECK(sht_geom_create(2, nullptr, np, p0, nullptr, nullptr, 1, &g) == SHT_EINVAL);
    CHECK(sht_geom_create(2, th2, np, p0, nullptr, nullptr, 1, nullptr) == SHT_EINVAL);
    CHECK(sht_geom_gauss(0, 5, 0.0, &g) == SHT_EINVAL);
    CHECK(sht_geom_healpix(0, &g) == SHT_EINVAL);
    CHECK(sht_geom_ecp(1, 4, SHT_ECP_CC, 0.0, &g) == SHT_EINVAL);
    CHECK(sht_geom_ecp(4, 4, 9, 0.0, &g) == SHT_EINVAL);
    CHECK(sht_geom_reduced_gauss(8, 15, 3, 5, 0, 0.0, &g) == SHT_EINVAL);
    CHECK(sht_geom_create(2, th2, np, p0, nullptr, ofs, 2, &g) == SHT_OK);
    Rings r = rings_of(g);
    CHECK(r.npix == 10 + 3 * 2 + 1);
    sht_geom_destroy(g);
    // a pointer that was never a handle
    double junk[8] = {0};
    CHECK(sht_geom_info(reinterpret_cast<sht_geom *>(junk), nullptr, nullptr) == SHT_ESTATE);
    CHECK(sht_geom_info(nullptr, nullptr, nullptr) == SHT_ESTATE);
    CHECK(sht_nalm(3, 5) == 0 && sht_nalm(7, 7) == 36 && sht_alm_index(7, 7, 7) == 35);
}

static void validation()
{
    using sht::validate_exec;
    const size_t alm = 1000, map = 2000, ph = 3000;
    char buf[8192];
    CHECK(validate_exec(-1, 0, true, alm, map, ph, buf, buf + 4000, false, false) == SHT_EINVAL);
    CHECK(validate_exec(8, 0, true, alm, map, ph, buf, buf + 4000, false, false) == SHT_EINVAL);
    CHECK(validate_exec(SHT_ALM2MAP, 0, true, alm, map, ph, nullptr, buf, false, false) == SHT_EINVAL);
    CHECK(validate_exec(SHT_ALM2MAP, 0, true, alm, map, ph, buf, buf + 1000, false, false) == SHT_OK);
    CHECK(validate_exec(SHT_ALM2MAP, 0, true, alm, map, ph, buf, buf + 999, false, false) == SHT_EINVAL);
    CHECK(validate_exec(SHT_MAP2ALM, 0, true, alm, map, ph, buf + 1000, buf, false, false) == SHT_OK);
    CHECK(validate_exec(SHT_MAP2ALM, 0, true, alm, map, ph, buf + 999, buf, false, false) == SHT_EINVAL);
    CHECK(validate_exec(SHT_MAP2ALM, 0, false, alm, map, ph, buf, buf + 4000, false, false) == SHT_EINVAL);
    CHECK(validate_exec(SHT_MAP2ALM, 0, false, alm, map, ph, buf, buf + 4000, false, true) == SHT_OK);
    CHECK(validate_exec(SHT_ALM2MAP_DERIV1, 0, true, alm, map, ph, buf, buf + 4000, false, false) == SHT_EINVAL);
    CHECK(validate_exec(SHT_ALM2MAP_DERIV1, 1, true, alm, map, ph, buf, buf + 4000, false, false) == SHT_OK);
    // staged: the Legendre synthesis writes phases (3000 bytes)
    CHECK(validate_exec(SHT_ALM2MAP, 0, true, alm, map, ph, buf + 2999, buf, false, true) == SHT_EINVAL);
    CHECK(validate_exec(SHT_ALM2MAP, 0, true, alm, map, ph, buf + 3000, buf, false, true) == SHT_OK);
    // staged: the ring synthesis reads phases (3000 bytes) and writes the map
    CHECK(validate_exec(SHT_ALM2MAP, 0, true, alm, map, ph, buf, buf + 2999, true, false) == SHT_EINVAL);
    CHECK(validate_exec(SHT_ALM2MAP, 0, true, alm, map, ph, buf, buf + 3000, true, false) == SHT_OK);
}

static void oracle()
{
    std::vector<double> lam(41);
    for (int s : {0, 2, -2, 3})
        for (int m : {0, 1, 5, 40}) CHECK(oracle_lambda(40, m, s, 0.7, lam.data()) == 0);
    CHECK(std::fabs(oracle_wigner_d(2, 0, 0, 0.3) - 0.5 * (3 * std::cos(0.3) * std::cos(0.3) - 1)) < 1e-15);
    // Gauss-Legendre round trip, spin 0 and spin 2, lmax 6
    sht_geom *g = nullptr;
    const int lmax = 6;
    CHECK(sht_geom_gauss(lmax + 1, 2 * lmax + 1, 0.0, &g) == SHT_OK);
    Rings r = rings_of(g);
    for (int spin : {0, 2}) {
        const int nc = spin ? 2 : 1;
        const int64_t na = sht_nalm(lmax, lmax);
        std::vector<double> a(2 * nc * na), b(2 * nc * na), map(nc * r.npix), F(nc * r.n * (lmax + 1) * 2);
        uint64_t x = 12345;
        for (int c = 0; c < nc; ++c)
            for (int m = 0; m <= lmax; ++m)
                for (int l = m; l <= lmax; ++l) {
                    const int64_t i = (int64_t)c * na + sht_alm_index(lmax, l, m);
                    x = x * 6364136223846793005ull + 1442695040888963407ull;
                    a[2 * i] = (l < spin) ? 0.0 : (double)(x >> 11) / 9007199254740992.0 - 0.5;
                    a[2 * i + 1] = (m == 0 || l < spin) ? 0.0 : (double)(x >> 13 & 0xffff) / 65536.0 - 0.5;
                }
        CHECK(oracle_synthesis(r.n, r.theta.data(), r.nphi.data(), r.phi0.data(), r.ofs.data(), 1, lmax, lmax,
                               spin, 1, a.data(), map.data(), 0, nullptr, F.data()) == 0);
        CHECK(oracle_analysis(r.n, r.theta.data(), r.nphi.data(), r.phi0.data(), r.weight.data(), r.ofs.data(), 1,
                              lmax, lmax, spin, 1, map.data(), b.data(), 0, nullptr, nullptr) == 0);
        double err = 0;
        for (size_t i = 0; i < a.size(); ++i) err = std::max(err, std::fabs(a[i] - b[i]));
        CHECK(err < 1e-13);
        // sampled rings and m
        const int sel[2] = {0, r.n - 1};
        CHECK(oracle_synthesis(r.n, r.theta.data(), r.nphi.data(), r.phi0.data(), r.ofs.data(), 1, lmax, lmax,
                               spin, 1, a.data(), map.data(), 2, sel, nullptr) == 0);
        const int msel[2] = {0, lmax};
        CHECK(oracle_analysis(r.n, r.theta.data(), r.nphi.data(), r.phi0.data(), r.weight.data(), r.ofs.data(), 1,
                              lmax, lmax, spin, 1, map.data(), b.data(), 2, msel, nullptr) == 0);
    }
    sht_geom_destroy(g);
}

int main()
{
    geometries();
    validation();
    oracle();
    if (failures) {
        std::fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    std::printf("sanitize driver: all checks passed\n");
    return 0;
}
