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
#include <mutex>
#include <new>
#include <unordered_map>

#include "sht_internal.h"
#include "trace.h"

namespace sht {

int check_hip(hipError_t e, const char *what)
{
    if (e == hipSuccess) return SHT_OK;
    set_error("%s: %s", what, hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? SHT_ENOMEM : SHT_EDEVICE;
}

// live device buffers and their sizes (for sht_memory_stats)
static std::mutex g_alloc_mu;
static std::unordered_map<void *, size_t> g_allocs;

int dev_alloc(void **ptr, size_t bytes, const char *what)
{
    *ptr = nullptr;
    if (bytes == 0) return SHT_OK;
    if (fault_should_fail()) {
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
    {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        g_allocs[*ptr] = bytes;
    }
    mem_count(1, (int64_t)bytes);
    return SHT_OK;
}

void dev_free(void *ptr)
{
    if (!ptr) return;
    size_t bytes = 0;
    {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        auto it = g_allocs.find(ptr);
        if (it != g_allocs.end()) {
            bytes = it->second;
            g_allocs.erase(it);
        }
    }
    mem_count(-1, -(int64_t)bytes);
    (void)hipFree(ptr);
}

int dev_upload(void *dst, const void *src, size_t bytes, const char *what)
{
    if (bytes == 0) return SHT_OK;
    return check_hip(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice), what);
}

// ------------------------------------------------------------------ plans

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

// Algorithmic work of the Legendre step (see sht.h): per kept (m, slot, l)
// triple the recursion (4 flops for spin 0: two FMAs; 10 for spin s > 0: two
// chains of 5, Sect. 4.1) plus per transform and ring of the slot 4 (spin 0) /
// 16 (spin s > 0) flops of products; HBM: a_lm + 2 x phases + maps.
static void count_work(Plan &p)
{
    const double triples = count_triples(p.shape(), p.slots, p.slots_per_tile);
    const double r = p.spin ? 10.0 : 4.0, c = p.spin ? 16.0 : 4.0;
    p.flops_rec = triples * r;
    p.flops_prod = triples * c * p.ntrans;
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
    const int jpg = p.tune.valu ? valu_jpg(p) : p.tune.synth_ncb * 16 / cpj;
    const int ngroups = (p.ntrans + jpg - 1) / jpg;
    const int MB = p.tune.synth_mblock;
    std::vector<std::vector<WaveItem>> die(NUM_XCD);
    std::vector<double> load(NUM_XCD, 0.0);
    for (int mb = 0; mb <= p.mmax; mb += MB) {
        std::vector<WaveItem> blk;
        double cost = 0.0;
        for (int m = mb; m < std::min(p.mmax + 1, mb + MB); ++m) {
            const double lrange = (double)(p.lmax + 1 - std::max(m, p.spin));
            // one item per active slot tile, or (vector path) per group of K
            // consecutive 64-slot units with an active tile
            const int tstep = p.tune.valu ? valu_k(p, false) * (64 / p.slots_per_tile) : 1;
            for (int t = 0; t < p.ntiles; t += tstep) {
                bool act = false;
                for (int u = t; u < std::min(p.ntiles, t + tstep); ++u) act = act || p.tile_mlim[u] >= m;
                if (!act) continue;
                for (int gI = 0; gI < ngroups; ++gI) {
                    blk.push_back(WaveItem{m, t, gI * jpg, 0});
                    cost += lrange * tstep * p.slots_per_tile;
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
    ++p.generation;
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
    build_slots(p.geom, p.slots);
    p.nslots = (int)p.slots.size();
    p.slots_per_tile = p.spin ? 32 : 64;
    p.ntiles = (p.nslots + p.slots_per_tile - 1) / p.slots_per_tile;
    p.tile_mlim.assign(p.ntiles, -1);
    for (int sl = 0; sl < p.nslots; ++sl) {
        int t = sl / p.slots_per_tile;
        p.tile_mlim[t] = std::max(p.tile_mlim[t], slot_mlim(p.shape(), p.slots[sl]));
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

    std::vector<Coef4> coef;
    std::vector<double> fl;
    std::vector<int64_t> cofs;
    build_coef(p.shape(), coef, fl, cofs);
    static_assert(sizeof(Coef4) == sizeof(double4), "coefficient layout");
    if ((rc = dev_alloc((void **)&p.d_coef, coef.size() * sizeof(double4), "coefficient table"))) return rc;
    if ((rc = dev_upload(p.d_coef, coef.data(), coef.size() * sizeof(double4), "upload"))) return rc;
    if ((rc = dev_alloc((void **)&p.d_fl, fl.size() * sizeof(double), "coefficient table"))) return rc;
    if ((rc = dev_upload(p.d_fl, fl.data(), fl.size() * sizeof(double), "upload"))) return rc;
    if ((rc = dev_alloc((void **)&p.d_coef_ofs, cofs.size() * sizeof(int64_t), "coefficient table"))) return rc;
    if ((rc = dev_upload(p.d_coef_ofs, cofs.data(), cofs.size() * sizeof(int64_t), "upload"))) return rc;

    std::vector<StartCoef> st;
    build_start(p.shape(), st);
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
    p.tune = default_tuning(p);
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

sht_tuning default_tuning(const Plan &p)
{
    sht_tuning t{};
    t.synth_ncb = synth_ncb_default(p.spin, p.ntrans, p.precision);
    t.synth_mblock = 4;
    t.anal_ncb = anal_ncb(p.spin, p.ntrans);
    t.anal_tpw = anal_tpw_built(p.spin, t.anal_ncb);
    // vector units where most matrix-core columns would be empty: one or two
    // spin-0 transforms (2 or 4 of 16 columns), one spin transform (4 of 16)
    t.valu = (p.precision == SHT_FP64 && ((p.spin == 0 && p.ntrans <= 2) || (p.spin > 0 && p.ntrans == 1))) ? 1 : 0;
    return t;
}

int tuning_check(const Plan &p, const sht_tuning &t)
{
    if (t.synth_ncb != 1 && t.synth_ncb != 2) {
        set_error("synth_ncb %d not built (1 or 2)", t.synth_ncb);
        return SHT_EUNSUPPORTED;
    }
    if (t.synth_mblock < 1 || t.synth_mblock > 64) {
        set_error("synth_mblock %d outside [1, 64]", t.synth_mblock);
        return SHT_EUNSUPPORTED;
    }
    if (t.anal_ncb != 1 && t.anal_ncb != 2) {
        set_error("anal_ncb %d not built (1 or 2)", t.anal_ncb);
        return SHT_EUNSUPPORTED;
    }
    if (t.valu != 0 && t.valu != 1) {
        set_error("valu must be 0 or 1");
        return SHT_EUNSUPPORTED;
    }
    if (t.valu && p.precision != SHT_FP64) {
        set_error("the vector-unit kernels are built for SHT_FP64 only");
        return SHT_EUNSUPPORTED;
    }
    if (t.anal_tpw != anal_tpw_built(p.spin, t.anal_ncb)) {
        set_error("anal_tpw %d not built for spin %d and anal_ncb %d", t.anal_tpw, p.spin, t.anal_ncb);
        return SHT_EUNSUPPORTED;
    }
    return SHT_OK;
}

int apply_tuning(Plan &p, const sht_tuning &t)
{
    int rc = tuning_check(p, t);
    if (rc) return rc;
    const sht_tuning old = p.tune;
    p.tune = t;
    if ((rc = build_synth_items(p))) {
        p.tune = old;
        (void)build_synth_items(p);
        return rc;
    }
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

Plan *plan_of(sht_plan *h)
{
    if (!reg_live(h, H_PLAN)) return nullptr;
    return reinterpret_cast<Plan *>(h);
}

static Plan *as_plan(sht_plan *h) { return plan_of(h); }

int check_exec_args(const Plan *p, int direction, const void *in, const void *out, bool stage_fft,
                    bool stage_leg)
{
    const int alm_comp = deriv_direction(direction) ? 1 : p->ncomp;
    const size_t alm_b = (size_t)p->ntrans * alm_comp * p->nalm * 16;
    const size_t map_b = (size_t)p->ntrans * p->ncomp * p->geom.npix * 8;
    const size_t ph_b = (size_t)p->phase_elems * 16;
    int rc = validate_exec(direction, p->spin, p->geom.has_weight, alm_b, map_b, ph_b, in, out, stage_fft,
                           stage_leg);
    if (rc) return rc;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != p->device) {
        (void)hipGetLastError();
        set_error("current device differs from the plan's device %d", p->device);
        return SHT_EDEVICE;
    }
    return SHT_OK;
}

// The launches of a full transform with the given phase and real-harmonics
// workspaces (arguments already checked).
int execute_with(const Plan &pl, int direction, const double *in, double *out, double *phase, double *rh,
                 hipStream_t s)
{
    const Plan *p = &pl;
    int rc;
    const int acomp = deriv_direction(direction) ? 1 : p->ncomp;
    if (synth_direction(direction)) {
        const double *a = in;
        if (p->real_h) {
            if ((rc = launch_real_harm(*p, in, rh, acomp, true, s))) return rc;
            a = rh;
        }
        if ((rc = launch_legendre_synth(*p, a, phase, deriv_direction(direction), s))) return rc;
        if ((rc = launch_ring_synth(*p, phase, out, weighted_direction(direction), s))) return rc;
    } else {
        if ((rc = launch_ring_anal(*p, in, phase, weighted_direction(direction), s))) return rc;
        if ((rc = launch_legendre_anal(*p, phase, out, anal_mode(direction, p->real_h), s))) return rc;
        if (p->real_h && (rc = launch_real_harm(*p, out, out, acomp, false, s))) return rc;
    }
    return finish_launch("sht_execute");
}

int finish_launch(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return check_hip(e, what);
    return SHT_OK;
}

}  // namespace sht

using namespace sht;

extern "C" {

int sht_plan_create(const sht_geom *g, int lmax, int mmax, int spin, int ntrans, int precision,
                    const sht_plan_opts *opts, sht_plan **out)
{
    TraceRange tr("sht_plan_create");
    if (!out) { set_error("out is NULL"); return SHT_EINVAL; }
    *out = nullptr;
    const Geom *G = geom_of(g);
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

    // set-up of the allocation-free entry point on this device (its failure
    // only disables that entry point)
    if (scratch_init(dev) != SHT_OK) set_error("");
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
    fault_arm();
    int rc = plan_build(*p);
    if (rc) {
        plan_free_device(p);
        delete p;
        return rc;
    }
    p->serial = reg_add(p, H_PLAN);
    log_msg(1,
            "plan %llu created on device %d: lmax %d, mmax %d, spin %d, %d transforms, %s, %d slots in %d tiles, "
            "%lld synthesis items; tuning synth_ncb=%d synth_mblock=%d anal_ncb=%d anal_tpw=%d valu=%d",
            (unsigned long long)p->serial, dev, lmax, mmax, spin, ntrans, precision == SHT_FP64 ? "fp64" : "fp32_mfma",
            p->nslots, p->ntiles, (long long)p->n_items, p->tune.synth_ncb, p->tune.synth_mblock, p->tune.anal_ncb,
            p->tune.anal_tpw, p->tune.valu);
    *out = reinterpret_cast<sht_plan *>(p);
    return SHT_OK;
}

void sht_plan_destroy(sht_plan *h)
{
    Plan *p = as_plan(h);
    if (!p) return;
    log_msg(1, "plan %llu destroyed", (unsigned long long)p->serial);
    reg_remove(p);
    (void)hipDeviceSynchronize();
    plan_free_device(p);
    delete p;
}

int sht_execute(sht_plan *h, int direction, const double *in, double *out, void *hip_stream)
{
    TraceRange tr("sht_execute");
    Plan *p = as_plan(h);
    if (!p) { set_error("invalid plan handle"); return SHT_ESTATE; }
    int rc = check_exec_args(p, direction, in, out, false, false);
    if (rc) return rc;
    log_msg(2, "sht_execute plan %llu direction %d stream %p", (unsigned long long)p->serial, direction, hip_stream);
    return execute_with(*p, direction, in, out, p->d_phase, p->d_rh, (hipStream_t)hip_stream);
}

int sht_legendre(sht_plan *h, int direction, const double *in, double *out, void *hip_stream)
{
    TraceRange tr("sht_legendre");
    Plan *p = as_plan(h);
    if (!p) { set_error("invalid plan handle"); return SHT_ESTATE; }
    int rc = check_exec_args(p, direction, in, out, false, true);
    if (rc) return rc;
    log_msg(2, "sht_legendre plan %llu direction %d stream %p", (unsigned long long)p->serial, direction, hip_stream);
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
    TraceRange tr("sht_ring_fft");
    Plan *p = as_plan(h);
    if (!p) { set_error("invalid plan handle"); return SHT_ESTATE; }
    int rc = check_exec_args(p, direction, in, out, true, false);
    if (rc) return rc;
    log_msg(2, "sht_ring_fft plan %llu direction %d stream %p", (unsigned long long)p->serial, direction, hip_stream);
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

int sht_plan_get_tuning(const sht_plan *h, sht_tuning *t)
{
    Plan *p = as_plan(const_cast<sht_plan *>(h));
    if (!p) { set_error("invalid plan handle"); return SHT_ESTATE; }
    if (!t) { set_error("t is NULL"); return SHT_EINVAL; }
    *t = p->tune;
    return SHT_OK;
}

int sht_plan_set_tuning(sht_plan *h, const sht_tuning *t)
{
    Plan *p = as_plan(h);
    if (!p) { set_error("invalid plan handle"); return SHT_ESTATE; }
    if (!t) { set_error("t is NULL"); return SHT_EINVAL; }
    fault_arm();
    const int rc = apply_tuning(*p, *t);
    if (!rc)
        log_msg(1, "plan %llu tuning set: synth_ncb=%d synth_mblock=%d anal_ncb=%d anal_tpw=%d valu=%d",
                (unsigned long long)p->serial, t->synth_ncb, t->synth_mblock, t->anal_ncb, t->anal_tpw, t->valu);
    return rc;
}

int sht_plan_flops(const sht_plan *h, int direction, double *flops_fp64, double *flops_mfma,
                   double *hbm_bytes)
{
    Plan *p = as_plan(const_cast<sht_plan *>(h));
    if (!p) { set_error("invalid plan handle"); return SHT_ESTATE; }
    if (direction < 0 || direction >= NUM_DIRECTIONS) {
        set_error("unknown direction %d", direction);
        return SHT_EINVAL;
    }
    // the same count in both directions: the analysis is the transpose of the
    // synthesis, with the same recursion and products
    const bool f32 = p->precision == SHT_FP32_MFMA;
    if (flops_fp64) *flops_fp64 = f32 ? p->flops_rec : p->flops_rec + p->flops_prod;
    if (flops_mfma) *flops_mfma = f32 ? p->flops_prod : 0.0;
    if (hbm_bytes) *hbm_bytes = p->hbm_bytes;
    return SHT_OK;
}

int sht_plan_info(const sht_plan *h, int64_t *n_items, int64_t *device_bytes)
{
    Plan *p = as_plan(const_cast<sht_plan *>(h));
    if (!p) { set_error("invalid plan handle"); return SHT_ESTATE; }
    if (n_items) *n_items = p->n_items;
    if (device_bytes) {
        const void *bufs[] = {p->d_slot_cos, p->d_slot_sin, p->d_slot_chalf, p->d_slot_shalf, p->d_slot_yn,
                              p->d_slot_ys, p->d_coef, p->d_fl, p->d_coef_ofs, p->d_start, p->d_tile_mlim,
                              p->d_zeros, p->d_dfac, p->d_synth_items, p->d_anal_ms, p->d_phase, p->d_rh,
                              p->fft.d_rows, p->fft.d_tw, p->fft.d_perm, p->fft.d_blue, p->fft.d_mvalid,
                              p->fft.d_phase_rot};
        int64_t total = 0;
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        for (const void *b : bufs) {
            auto it = g_allocs.find(const_cast<void *>(b));
            if (it != g_allocs.end()) total += (int64_t)it->second;
        }
        *device_bytes = total;
    }
    return SHT_OK;
}

}  // extern "C"
