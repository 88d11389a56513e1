// Batches of plans (one persistent Legendre analysis launch over all plans,
// each plan's Legendre synthesis and ring FFTs, optionally replayed from a
// captured HIP graph) and the synthesis tile autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "sht_internal.h"

using namespace sht;

namespace {

void batch_free(Batch *b)
{
    for (int d = 0; d < NUM_DIRECTIONS; ++d)
        if (b->graph[d]) (void)hipGraphExecDestroy(b->graph[d]);
    dev_free(b->d_views);
    dev_free(b->d_ana);
    dev_free(b->d_counter);
}

// Queue of analysis items (m, transform group) of all plans, by cost.
void anal_queue(const Batch &b, std::vector<BatchAnaItem> &q)
{
    const int cpj = b.spin ? 4 : 2;
    const int jpg = b.ana_ncb * 16 / cpj;
    std::vector<std::pair<double, BatchAnaItem>> v;
    for (int pi = 0; pi < (int)b.plans.size(); ++pi) {
        const Plan &p = *b.plans[pi];
        for (int m = 0; m <= p.mmax; ++m) {
            int act = 0;
            for (int t = 0; t < p.ntiles; ++t) act += p.tile_mlim[t] >= m;
            const int nw = ana_nw(b.precision == SHT_FP32_MFMA, b.spin != 0);
            const double cost = (double)(p.lmax + 1 - std::max(m, p.spin)) * (double)((act + nw - 1) / nw + 1);
            for (int t0 = 0; t0 < p.ntrans; t0 += jpg) v.push_back({cost, BatchAnaItem{pi, m, t0, 0}});
        }
    }
    std::stable_sort(v.begin(), v.end(), [](const auto &a, const auto &c) { return a.first > c.first; });
    q.clear();
    for (auto &e : v) q.push_back(e.second);
}

// Everything one execution of the batch puts on the stream.
int batch_enqueue(Batch &b, int direction, const double *const *in, double *const *out, hipStream_t s)
{
    BatchPtrs ptrs;
    std::memset(&ptrs, 0, sizeof(ptrs));
    const int np = (int)b.plans.size();
    int rc;
    if (synth_direction(direction)) {
        // each plan's own die-aware item list (its a_lm rows and phase lines stay
        // in one L2; one cost-ordered queue over all plans measured slower)
        for (int i = 0; i < np; ++i) {
            const double *a = in[i];
            if (b.real_h) {
                if ((rc = launch_real_harm(*b.plans[i], in[i], b.plans[i]->d_rh,
                                           deriv_direction(direction) ? 1 : b.plans[i]->ncomp, true, s)))
                    return rc;
                a = b.plans[i]->d_rh;
            }
            if ((rc = launch_legendre_synth(*b.plans[i], a, b.plans[i]->d_phase, deriv_direction(direction), s)))
                return rc;
        }
        for (int i = 0; i < np; ++i)
            if ((rc = launch_ring_synth(*b.plans[i], b.plans[i]->d_phase, out[i],
                                        weighted_direction(direction), s)))
                return rc;
    } else {
        for (int i = 0; i < np; ++i)
            if ((rc = launch_ring_anal(*b.plans[i], in[i], b.plans[i]->d_phase, weighted_direction(direction),
                                       s)))
                return rc;
        for (int i = 0; i < np; ++i) {
            ptrs.in[i] = b.plans[i]->d_phase;
            ptrs.out[i] = out[i];
        }
        if ((rc = launch_legendre_anal_batch(b, ptrs, anal_mode(direction, b.real_h), s))) return rc;
        if (b.real_h)
            for (int i = 0; i < np; ++i)
                if ((rc = launch_real_harm(*b.plans[i], out[i], out[i],
                                           deriv_direction(direction) ? 1 : b.plans[i]->ncomp, false, s)))
                    return rc;
    }
    return SHT_OK;
}

// Time one Legendre synthesis of the plan (ms per launch) on scratch input.
int time_synth(Plan &p, const double *alm, int reps, double &ms)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        (void)hipGetLastError();
        set_error("event creation failed");
        return SHT_EDEVICE;
    }
    int rc = launch_legendre_synth(p, alm, p.d_phase, false, nullptr);   // warm-up
    if (!rc) rc = check_hip(hipEventRecord(e0, nullptr), "autotune");
    for (int r = 0; r < reps && !rc; ++r) rc = launch_legendre_synth(p, alm, p.d_phase, false, nullptr);
    if (!rc) rc = check_hip(hipEventRecord(e1, nullptr), "autotune");
    if (!rc) rc = check_hip(hipEventSynchronize(e1), "autotune");
    float t = 0.f;
    if (!rc) rc = check_hip(hipEventElapsedTime(&t, e0, e1), "autotune");
    ms = (double)t / (reps > 0 ? reps : 1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

std::string tune_key(const Plan &p)
{
    char buf[256];
    std::snprintf(buf, sizeof buf, "synth_ncb gfx950 lmax=%d mmax=%d spin=%d ntrans=%d nrings=%d prec=%d",
                  p.lmax, p.mmax, p.spin, p.ntrans, p.geom.nrings, p.precision);
    return buf;
}

int tune_cache_lookup(const std::string &key)
{
    const char *path = std::getenv("SHT_TUNE_CACHE");
    if (!path || !*path) return -1;
    FILE *f = std::fopen(path, "r");
    if (!f) return -1;
    char line[512];
    int val = -1;
    while (std::fgets(line, sizeof line, f)) {
        std::string l(line);
        const size_t bar = l.rfind('|');
        if (bar == std::string::npos) continue;
        if (l.substr(0, bar) == key) val = std::atoi(l.c_str() + bar + 1);
    }
    std::fclose(f);
    return val;
}

void tune_cache_store(const std::string &key, int val)
{
    const char *path = std::getenv("SHT_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s|%d\n", key.c_str(), val);
    std::fclose(f);
}

}  // namespace

extern "C" {

int sht_batch_create(int nplans, sht_plan *const *plans, sht_batch **out)
{
    if (!out) { set_error("out is NULL"); return SHT_EINVAL; }
    *out = nullptr;
    if (nplans < 1 || !plans) { set_error("need at least one plan"); return SHT_EINVAL; }
    if (nplans > MAX_BATCH_PLANS) {
        set_error("a batch holds at most %d plans", MAX_BATCH_PLANS);
        return SHT_EINVAL;
    }
    Batch *b = new (std::nothrow) Batch();
    if (!b) { set_error("host allocation failed"); return SHT_ENOMEM; }
    int maxj = 0;
    for (int i = 0; i < nplans; ++i) {
        Plan *p = plan_of(plans[i]);
        if (!p) {
            delete b;
            set_error("plan %d is not a valid plan", i);
            return SHT_ESTATE;
        }
        if (i > 0 && (p->spin != b->spin || p->precision != b->precision || p->device != b->plans[0]->device ||
                      p->real_h != b->real_h)) {
            delete b;
            set_error("all plans of a batch must have the same spin, precision, device and coefficient storage");
            return SHT_EINVAL;
        }
        for (Plan *q : b->plans)
            if (q == p) {
                delete b;
                set_error("plan %d appears twice (plans share no workspace within a batch)", i);
                return SHT_EINVAL;
            }
        b->spin = p->spin;
        b->precision = p->precision;
        b->real_h = p->real_h;
        maxj = std::max(maxj, p->ntrans);
        b->plans.push_back(p);
        b->plan_serial.push_back(p->serial);
    }
    b->device = b->plans[0]->device;
    b->ana_ncb = anal_ncb(b->spin, maxj);
    b->ana_groups = anal_batch_groups(b->spin, b->ana_ncb, b->precision == SHT_FP32_MFMA, b->device);
    fault_arm();
    std::vector<BatchAnaItem> aq;
    anal_queue(*b, aq);
    std::vector<LegView> views;
    for (Plan *p : b->plans) views.push_back(make_leg_view(*p));
    b->nana = (int)aq.size();
    int rc;
    if ((rc = dev_alloc((void **)&b->d_views, views.size() * sizeof(LegView), "batch tables")) ||
        (rc = dev_upload(b->d_views, views.data(), views.size() * sizeof(LegView), "batch tables")) ||
        (rc = dev_alloc((void **)&b->d_ana, std::max<size_t>(1, aq.size()) * sizeof(BatchAnaItem), "batch tables")) ||
        (rc = dev_alloc((void **)&b->d_counter, 64, "batch counter"))) {
        batch_free(b);
        delete b;
        return rc;
    }
    if (!aq.empty() && (rc = dev_upload(b->d_ana, aq.data(), aq.size() * sizeof(BatchAnaItem), "batch tables"))) {
        batch_free(b);
        delete b;
        return rc;
    }
    reg_add(b, H_BATCH);
    *out = reinterpret_cast<sht_batch *>(b);
    return SHT_OK;
}

int sht_batch_execute(sht_batch *h, int direction, const double *const *in, double *const *out,
                      void *hip_stream)
{
    if (!reg_live(h, H_BATCH)) { set_error("invalid batch handle"); return SHT_ESTATE; }
    Batch *b = reinterpret_cast<Batch *>(h);
    if (!in || !out) { set_error("in and out arrays are required"); return SHT_EINVAL; }
    if (direction < 0 || direction >= NUM_DIRECTIONS) { set_error("unknown direction %d", direction); return SHT_EINVAL; }
    const int np = (int)b->plans.size();
    for (int i = 0; i < np; ++i) {
        uint64_t serial = 0;
        if (!reg_live(b->plans[i], H_PLAN, &serial) || serial != b->plan_serial[i]) {
            set_error("plan %d of the batch was destroyed", i);
            return SHT_ESTATE;
        }
        int rc = check_exec_args(b->plans[i], direction, in[i], out[i], false, false);
        if (rc) return rc;
    }
    hipStream_t s = (hipStream_t)hip_stream;
    if (!s) {   // the null stream cannot be captured: plain launches
        int rc = batch_enqueue(*b, direction, in, out, s);
        if (rc) return rc;
        return finish_launch("sht_batch_execute");
    }
    std::vector<uintptr_t> key;
    for (int i = 0; i < np; ++i) {
        key.push_back((uintptr_t)in[i]);
        key.push_back((uintptr_t)out[i]);
        key.push_back((uintptr_t)b->plans[i]->generation);
    }
    if (!b->graph[direction] || b->graph_key[direction] != key || b->graph_stream[direction] != s) {
        if (b->graph[direction]) {
            (void)hipGraphExecDestroy(b->graph[direction]);
            b->graph[direction] = nullptr;
        }
        int rc = check_hip(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "graph capture");
        if (rc) return rc;
        rc = batch_enqueue(*b, direction, in, out, s);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(s, &g);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if ((rc = check_hip(e, "graph capture"))) return rc;
        hipGraphExec_t ex = nullptr;
        rc = check_hip(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0), "graph instantiation");
        (void)hipGraphDestroy(g);
        if (rc) return rc;
        b->graph[direction] = ex;
        b->graph_key[direction] = key;
        b->graph_stream[direction] = s;
    }
    return check_hip(hipGraphLaunch(b->graph[direction], s), "graph launch");
}

void sht_batch_destroy(sht_batch *h)
{
    if (!reg_live(h, H_BATCH)) return;
    Batch *b = reinterpret_cast<Batch *>(h);
    reg_remove(b);
    (void)hipDeviceSynchronize();
    batch_free(b);
    delete b;
}

int sht_autotune(sht_plan *h, double budget_seconds)
{
    Plan *p = plan_of(h);
    if (!p) { set_error("invalid plan handle"); return SHT_ESTATE; }
    if (!(budget_seconds >= 0.0)) { set_error("budget must be >= 0"); return SHT_EINVAL; }
    const std::string key = tune_key(*p);
    std::vector<int> cand = {1};
    if (p->ntrans * (p->spin ? 4 : 2) > 16) cand.push_back(2);
    const int cached = tune_cache_lookup(key);
    if (cached > 0 && std::find(cand.begin(), cand.end(), cached) != cand.end()) {
        if (cached != p->synth_ncb) {
            p->synth_ncb = cached;
            return build_synth_items(*p);
        }
        return SHT_OK;
    }
    if (cand.size() < 2 || budget_seconds == 0.0) return SHT_OK;
    // scratch input: zero coefficients (the kernels' time does not depend on the values)
    double *alm = nullptr;
    const size_t bytes = (size_t)p->ntrans * p->ncomp * p->nalm * 16;
    int rc = dev_alloc((void **)&alm, bytes, "autotune scratch");
    if (rc) return rc;
    if ((rc = check_hip(hipMemset(alm, 0, bytes), "autotune scratch"))) {
        dev_free(alm);
        return rc;
    }
    const int orig = p->synth_ncb;
    int best = orig;
    double best_ms = 1e300;
    const auto t_start = std::chrono::steady_clock::now();
    for (int c : cand) {
        p->synth_ncb = c;
        if ((rc = build_synth_items(*p))) break;
        double ms = 0.0;
        if ((rc = time_synth(*p, alm, 2, ms))) break;
        if (ms < best_ms) {
            best_ms = ms;
            best = c;
        }
        const double spent = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
        if (spent > budget_seconds) break;
    }
    dev_free(alm);
    p->synth_ncb = rc ? orig : best;
    const int rc2 = build_synth_items(*p);
    if (rc) return rc;
    if (rc2) return rc2;
    tune_cache_store(key, best);
    return SHT_OK;
}

}  // extern "C"
