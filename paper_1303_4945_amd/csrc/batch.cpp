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
#include "trace.h"

using namespace sht;

namespace {

void batch_free(Batch *b)
{
    for (int d = 0; d < NUM_DIRECTIONS; ++d)
        if (b->graph[d]) (void)hipGraphExecDestroy(b->graph[d]);
    for (hipStream_t s : b->aux) (void)hipStreamDestroy(s);
    for (hipEvent_t e : b->join) (void)hipEventDestroy(e);
    b->aux.clear();
    b->join.clear();
    dev_free(b->d_views);
    dev_free(b->d_ana);
    dev_free(b->d_syn);
    dev_free(b->d_counter);
}

// Queue of analysis items of all plans.  SHT_QUEUE_COST: items (plan, m,
// transform group) by decreasing cost (degree range x passes over the active
// slot tiles); SHT_QUEUE_MPAIRS: items (plan, m and mmax - m, group), whose
// degree ranges add up to about lmax + 2, by decreasing pair cost.
void anal_queue(const Batch &b, std::vector<BatchAnaItem> &q)
{
    const int cpj = b.spin ? 4 : 2;
    const int jpg = b.ana_ncb * 16 / cpj;
    const int nw = ana_nw(b.precision == SHT_FP32_MFMA, b.spin != 0);
    std::vector<std::pair<double, BatchAnaItem>> v;
    for (int pi = 0; pi < (int)b.plans.size(); ++pi) {
        const Plan &p = *b.plans[pi];
        auto cost = [&](int m) {
            int act = 0;
            for (int t = 0; t < p.ntiles; ++t) act += p.tile_mlim[t] >= m;
            return (double)(p.lmax + 1 - std::max(m, p.spin)) * (double)((act + nw - 1) / nw + 1);
        };
        if (b.queue_order == SHT_QUEUE_MPAIRS) {
            for (int m = 0; m <= p.mmax - m; ++m) {
                const int m2 = p.mmax - m;
                const double c = cost(m) + (m2 != m ? cost(m2) : 0.0);
                for (int t0 = 0; t0 < p.ntrans; t0 += jpg)
                    v.push_back({c, BatchAnaItem{pi, m, t0, m2 != m ? m2 : -1}});
            }
        } else {
            for (int m = 0; m <= p.mmax; ++m) {
                const double c = cost(m);
                for (int t0 = 0; t0 < p.ntrans; t0 += jpg) v.push_back({c, BatchAnaItem{pi, m, t0, -1}});
            }
        }
    }
    std::stable_sort(v.begin(), v.end(), [](const auto &a, const auto &c) { return a.first > c.first; });
    q.clear();
    for (auto &e : v) q.push_back(e.second);
}

// Queue of synthesis items of all plans (persistent synthesis): one item per
// (plan, m, slot tile active at m, transform group of the plan's column
// blocks); SHT_QUEUE_MPAIRS: the same tile and group at m and mmax - m in one
// item.  Items come in blocks of the plan's synth_mblock consecutive m (of the
// first m of a pair), and every block goes to one die's segment (the least
// loaded, blocks by decreasing cost), so that the lines of F that a block
// writes stay in one die's L2; within a segment, items by decreasing cost.
void synth_queue(Batch &b, std::vector<BatchSynItem> &q)
{
    const int cpj = b.spin ? 4 : 2;
    using Item = std::pair<double, BatchSynItem>;
    struct Block {
        double cost = 0.0;
        std::vector<Item> items;
    };
    std::vector<Block> blocks;
    for (int pi = 0; pi < (int)b.plans.size(); ++pi) {
        const Plan &p = *b.plans[pi];
        const int jpg = p.tune.synth_ncb * 16 / cpj;
        const int MB = std::max(1, p.tune.synth_mblock);
        auto lrange = [&](int m) { return (double)(p.lmax + 1 - std::max(m, p.spin)); };
        const bool pairs = b.queue_order == SHT_QUEUE_MPAIRS;
        const int mend = pairs ? p.mmax / 2 : p.mmax;   // last first-m of an item
        for (int m0 = 0; m0 <= mend; m0 += MB) {
            Block blk;
            for (int m = m0; m <= std::min(mend, m0 + MB - 1); ++m) {
                const int m2 = pairs ? p.mmax - m : -1;
                for (int t = 0; t < p.ntiles; ++t) {
                    const bool a1 = p.tile_mlim[t] >= m, a2 = pairs && m2 != m && p.tile_mlim[t] >= m2;
                    if (!a1 && !a2) continue;
                    const double c = (a1 ? lrange(m) : 0.0) + (a2 ? lrange(m2) : 0.0);
                    for (int t0 = 0; t0 < p.ntrans; t0 += jpg) {
                        blk.items.push_back({c, BatchSynItem{pi, a1 ? m : m2, (a1 && a2) ? m2 : -1, t, t0, {0, 0, 0}}});
                        blk.cost += c;
                    }
                }
            }
            if (!blk.items.empty()) blocks.push_back(std::move(blk));
        }
    }
    std::stable_sort(blocks.begin(), blocks.end(), [](const Block &a, const Block &c) { return a.cost > c.cost; });
    std::vector<std::vector<Item>> die(NUM_XCD);
    std::vector<double> load(NUM_XCD, 0.0);
    for (Block &blk : blocks) {
        const int d = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[d] += blk.cost;
        die[d].insert(die[d].end(), blk.items.begin(), blk.items.end());
    }
    q.clear();
    for (int d = 0; d < NUM_XCD; ++d) {
        std::stable_sort(die[d].begin(), die[d].end(), [](const Item &a, const Item &c) { return a.first > c.first; });
        b.syn_ofs[d] = (int)q.size();
        for (auto &e : die[d]) q.push_back(e.second);
    }
    b.syn_ofs[NUM_XCD] = (int)q.size();
}

// (Re)builds the synthesis queue when the plans' work lists changed since it
// was built, or when forced (new queue order).  Host work, a device
// synchronization (the old queue may still be read) and an upload: refused
// while the stream s is being captured.
int refresh_synth_queue(Batch &b, hipStream_t s, bool force)
{
    if (b.concurrent != 2) {   // only schedule 2 uses the queue: built when it is chosen
        if (b.d_syn) (void)hipDeviceSynchronize();
        dev_free(b.d_syn);
        b.d_syn = nullptr;
        b.nsyn = 0;
        for (int &o : b.syn_ofs) o = 0;
        b.syn_ok = false;
        b.syn_gen.clear();
        return SHT_OK;
    }
    std::vector<uint64_t> gen;
    for (const Plan *p : b.plans) gen.push_back(p->generation);
    if (!force && gen == b.syn_gen) return SHT_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (s && hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) {
        set_error("a plan of the batch was retuned: run the batch once outside stream capture first");
        return SHT_ESTATE;
    }
    if (b.d_syn) (void)hipDeviceSynchronize();
    const Plan &p0 = *b.plans[0];
    b.syn_ok = true;
    for (const Plan *p : b.plans)
        if (p->tune.valu || p->tune.synth_ncb != p0.tune.synth_ncb || p->flush_chunks != p0.flush_chunks)
            b.syn_ok = false;
    dev_free(b.d_syn);
    b.d_syn = nullptr;
    b.nsyn = 0;
    for (int &o : b.syn_ofs) o = 0;
    b.syn_gen.clear();
    if (!b.syn_ok) {
        b.syn_gen = gen;
        return SHT_OK;
    }
    b.syn_ncb = p0.tune.synth_ncb;
    b.syn_flush = p0.flush_chunks;
    b.syn_groups = synth_batch_groups(b.spin, b.syn_ncb, b.precision == SHT_FP32_MFMA, b.device);
    std::vector<BatchSynItem> q;
    synth_queue(b, q);
    int rc = dev_alloc((void **)&b.d_syn, std::max<size_t>(1, q.size()) * sizeof(BatchSynItem), "batch tables");
    if (!rc && !q.empty()) rc = dev_upload(b.d_syn, q.data(), q.size() * sizeof(BatchSynItem), "batch tables");
    if (rc) {   // no queue: the plans' own launches run until a later call builds it
        dev_free(b.d_syn);
        b.d_syn = nullptr;
        for (int &o : b.syn_ofs) o = 0;
        b.syn_ok = false;
        return rc;
    }
    b.nsyn = (int)q.size();
    b.syn_gen = gen;
    return SHT_OK;
}

bool persistent_synth(const Batch &b) { return b.concurrent == 2 && b.syn_ok; }

int upload_queue(Batch &b)
{
    std::vector<BatchAnaItem> aq;
    anal_queue(b, aq);
    b.nana = (int)aq.size();
    dev_free(b.d_ana);
    b.d_ana = nullptr;
    int rc;
    if ((rc = dev_alloc((void **)&b.d_ana, std::max<size_t>(1, aq.size()) * sizeof(BatchAnaItem), "batch tables")))
        return rc;
    if (!aq.empty()) return dev_upload(b.d_ana, aq.data(), aq.size() * sizeof(BatchAnaItem), "batch tables");
    return SHT_OK;
}

// Stream of plan i's launch chain: its own stream when the batch runs plans
// concurrently (forked from and joined into the caller's stream), else the
// caller's stream.
hipStream_t chain_stream(const Batch &b, int i, hipStream_t s) { return b.concurrent ? b.aux[i] : s; }

int fork_chains(Batch &b, hipStream_t s)
{
    if (!b.concurrent) return SHT_OK;
    hipEvent_t fork = b.join.back();
    int rc = check_hip(hipEventRecord(fork, s), "batch fork");
    for (size_t i = 0; i < b.plans.size() && !rc; ++i)
        rc = check_hip(hipStreamWaitEvent(b.aux[i], fork, 0), "batch fork");
    return rc;
}

int join_chains(Batch &b, hipStream_t s)
{
    if (!b.concurrent) return SHT_OK;
    int rc = SHT_OK;
    for (size_t i = 0; i < b.plans.size() && !rc; ++i) {
        rc = check_hip(hipEventRecord(b.join[i], b.aux[i]), "batch join");
        if (!rc) rc = check_hip(hipStreamWaitEvent(s, b.join[i], 0), "batch join");
    }
    return rc;
}

// Legendre synthesis of plan i into phase (with the real-harmonics conversion first).
int plan_legendre_synth(Batch &b, int i, int direction, const double *in, double *phase, hipStream_t s)
{
    Plan &p = *b.plans[i];
    const double *a = in;
    int rc;
    if (b.real_h) {
        if ((rc = launch_real_harm(p, in, p.d_rh, deriv_direction(direction) ? 1 : p.ncomp, true, s))) return rc;
        a = p.d_rh;
    }
    return launch_legendre_synth(p, a, phase, deriv_direction(direction), s);
}

// Persistent Legendre analysis over all plans, then the real-harmonics conversion.
int batch_legendre_anal(Batch &b, int direction, const double *const *phase, double *const *out, hipStream_t s)
{
    BatchPtrs ptrs;
    std::memset(&ptrs, 0, sizeof(ptrs));
    const int np = (int)b.plans.size();
    for (int i = 0; i < np; ++i) {
        ptrs.in[i] = phase[i];
        ptrs.out[i] = out[i];
    }
    int rc;
    bool valu = false;
    for (const Plan *p : b.plans) valu = valu || p->tune.valu;
    if (valu) {
        // plans on the vector-unit path: each plan's own analysis launch (the
        // persistent queue runs the matrix-core kernels), same results as the plans
        for (int i = 0; i < np; ++i)
            if ((rc = launch_legendre_anal(*b.plans[i], phase[i], out[i], anal_mode(direction, b.real_h), s))) return rc;
    } else if ((rc = launch_legendre_anal_batch(b, ptrs, anal_mode(direction, b.real_h), s))) {
        return rc;
    }
    if (b.real_h)
        for (int i = 0; i < np; ++i)
            if ((rc = launch_real_harm(*b.plans[i], out[i], out[i], deriv_direction(direction) ? 1 : b.plans[i]->ncomp,
                                       false, s)))
                return rc;
    return SHT_OK;
}

// Persistent Legendre synthesis of all plans on s into phase[i] (with the
// real-harmonics conversions first).
int batch_legendre_synth(Batch &b, int direction, const double *const *in, double *const *phase, hipStream_t s)
{
    BatchPtrs ptrs;
    std::memset(&ptrs, 0, sizeof(ptrs));
    int rc;
    for (int i = 0; i < (int)b.plans.size(); ++i) {
        Plan &p = *b.plans[i];
        ptrs.in[i] = in[i];
        ptrs.out[i] = phase[i];
        if (b.real_h) {
            if ((rc = launch_real_harm(p, in[i], p.d_rh, deriv_direction(direction) ? 1 : p.ncomp, true, s))) return rc;
            ptrs.in[i] = p.d_rh;
        }
    }
    return launch_legendre_synth_batch(b, ptrs, deriv_direction(direction), s);
}

// Everything one execution of the batch puts on the stream.
int batch_enqueue(Batch &b, int direction, const double *const *in, double *const *out, hipStream_t s)
{
    const int np = (int)b.plans.size();
    int rc;
    if (synth_direction(direction) && persistent_synth(b)) {
        // one persistent Legendre launch over all plans, then every plan's ring
        // FFTs on its own stream
        std::vector<double *> ph(np);
        for (int i = 0; i < np; ++i) ph[i] = b.plans[i]->d_phase;
        if ((rc = batch_legendre_synth(b, direction, in, ph.data(), s))) return rc;
        if ((rc = fork_chains(b, s))) return rc;
        for (int i = 0; i < np; ++i)
            if ((rc = launch_ring_synth(*b.plans[i], b.plans[i]->d_phase, out[i], weighted_direction(direction),
                                        chain_stream(b, i, s))))
                return rc;
        return join_chains(b, s);
    }
    if ((rc = fork_chains(b, s))) return rc;
    if (synth_direction(direction)) {
        // per plan: its die-aware Legendre item list, then its ring FFTs
        for (int i = 0; i < np; ++i) {
            const hipStream_t cs = chain_stream(b, i, s);
            if ((rc = plan_legendre_synth(b, i, direction, in[i], b.plans[i]->d_phase, cs))) return rc;
            if ((rc = launch_ring_synth(*b.plans[i], b.plans[i]->d_phase, out[i], weighted_direction(direction), cs)))
                return rc;
        }
        return join_chains(b, s);
    }
    for (int i = 0; i < np; ++i)
        if ((rc = launch_ring_anal(*b.plans[i], in[i], b.plans[i]->d_phase, weighted_direction(direction),
                                   chain_stream(b, i, s))))
            return rc;
    if ((rc = join_chains(b, s))) return rc;
    std::vector<const double *> ph(np);
    for (int i = 0; i < np; ++i) ph[i] = b.plans[i]->d_phase;
    return batch_legendre_anal(b, direction, ph.data(), out, s);
}

int check_batch_args(Batch *b, int direction, const double *const *in, double *const *out, bool leg_only)
{
    if (!in || !out) { set_error("in and out arrays are required"); return SHT_EINVAL; }
    if (direction < 0 || direction >= NUM_DIRECTIONS) { set_error("unknown direction %d", direction); return SHT_EINVAL; }
    for (size_t i = 0; i < b->plans.size(); ++i) {
        uint64_t serial = 0;
        if (!reg_live(b->plans[i], H_PLAN, &serial) || serial != b->plan_serial[i]) {
            set_error("plan %zu of the batch was destroyed", i);
            return SHT_ESTATE;
        }
        int rc = check_exec_args(b->plans[i], direction, in[i], out[i], false, leg_only);
        if (rc) return rc;
    }
    return SHT_OK;
}

// Mean time (ms) of `reps` launches of fn after one warm-up launch.
template <typename F>
int time_launches(F fn, int reps, double &ms)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        (void)hipGetLastError();
        set_error("event creation failed");
        return SHT_EDEVICE;
    }
    int rc = fn();   // warm-up
    if (!rc) rc = check_hip(hipEventRecord(e0, nullptr), "autotune");
    for (int r = 0; r < reps && !rc; ++r) rc = fn();
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
    std::snprintf(buf, sizeof buf, "sht-tuning gfx950 lmax=%d mmax=%d spin=%d ntrans=%d nrings=%d prec=%d",
                  p.lmax, p.mmax, p.spin, p.ntrans, p.geom.nrings, p.precision);
    return buf;
}

std::string tune_text(const sht_tuning &t)
{
    char buf[160];
    std::snprintf(buf, sizeof buf, "synth_ncb=%d,synth_mblock=%d,anal_ncb=%d,anal_tpw=%d,valu=%d", t.synth_ncb,
                  t.synth_mblock, t.anal_ncb, t.anal_tpw, t.valu);
    return buf;
}

bool tune_parse(const char *s, sht_tuning &t)
{
    sht_tuning r{};
    if (std::sscanf(s, "synth_ncb=%d,synth_mblock=%d,anal_ncb=%d,anal_tpw=%d,valu=%d", &r.synth_ncb,
                    &r.synth_mblock, &r.anal_ncb, &r.anal_tpw, &r.valu) != 5)
        return false;
    t = r;
    return true;
}

// the last line of the cache file with this key (false: none)
bool tune_cache_lookup(const std::string &key, sht_tuning &t)
{
    const char *path = std::getenv("SHT_TUNE_CACHE");
    if (!path || !*path) return false;
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        std::string l(line);
        const size_t bar = l.rfind('|');
        if (bar == std::string::npos) continue;
        sht_tuning c{};
        if (l.substr(0, bar) == key && tune_parse(l.c_str() + bar + 1, c)) {
            t = c;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

void tune_cache_store(const std::string &key, const sht_tuning &t)
{
    const char *path = std::getenv("SHT_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s|%s\n", key.c_str(), tune_text(t).c_str());
    std::fclose(f);
}

}  // namespace

extern "C" {

int sht_batch_create(int nplans, sht_plan *const *plans, sht_batch **out)
{
    TraceRange tr("sht_batch_create");
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
    std::vector<LegView> views;
    for (Plan *p : b->plans) views.push_back(make_leg_view(*p));
    int rc;
    if ((rc = dev_alloc((void **)&b->d_views, views.size() * sizeof(LegView), "batch tables")) ||
        (rc = dev_upload(b->d_views, views.data(), views.size() * sizeof(LegView), "batch tables")) ||
        (rc = upload_queue(*b)) || (rc = refresh_synth_queue(*b, nullptr, true)) ||
        (rc = dev_alloc((void **)&b->d_counter, 64 * (NUM_XCD + 2), "batch counters"))) {
        batch_free(b);
        delete b;
        return rc;
    }
    for (int i = 0; i <= nplans && !rc; ++i) {
        hipEvent_t e = nullptr;
        rc = check_hip(hipEventCreateWithFlags(&e, hipEventDisableTiming), "batch events");
        if (!rc) b->join.push_back(e);
        if (i < nplans && !rc) {
            hipStream_t st = nullptr;
            rc = check_hip(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "batch streams");
            if (!rc) b->aux.push_back(st);
        }
    }
    if (rc) {
        batch_free(b);
        delete b;
        return rc;
    }
    const uint64_t serial = reg_add(b, H_BATCH);
    log_msg(1, "batch %llu created: %d plans, spin %d, %s, %d analysis queue items, %d persistent work groups",
            (unsigned long long)serial, nplans, b->spin, b->precision == SHT_FP64 ? "fp64" : "fp32_mfma", b->nana,
            b->ana_groups);
    *out = reinterpret_cast<sht_batch *>(b);
    return SHT_OK;
}

int sht_batch_configure(sht_batch *h, int queue_order, int concurrent)
{
    if (!reg_live(h, H_BATCH)) { set_error("invalid batch handle"); return SHT_ESTATE; }
    Batch *b = reinterpret_cast<Batch *>(h);
    if (queue_order != SHT_QUEUE_COST && queue_order != SHT_QUEUE_MPAIRS) {
        set_error("unknown queue order %d", queue_order);
        return SHT_EINVAL;
    }
    if (concurrent < 0 || concurrent > 2) { set_error("concurrent must be 0, 1 or 2"); return SHT_EINVAL; }
    (void)hipDeviceSynchronize();
    fault_arm();
    const int old_order = b->queue_order, old_conc = b->concurrent;
    b->queue_order = queue_order;
    b->concurrent = concurrent;
    int rc = upload_queue(*b);
    if (!rc) rc = refresh_synth_queue(*b, nullptr, true);
    if (rc) {   // the previous schedule stays
        b->queue_order = old_order;
        b->concurrent = old_conc;
        (void)upload_queue(*b);
        (void)refresh_synth_queue(*b, nullptr, true);
        return rc;
    }
    if (concurrent == 2 && !b->syn_ok)
        log_msg(1, "batch: persistent synthesis needs every plan on the matrix-core path with one shape; "
                   "per-plan synthesis launches instead");
    for (int d = 0; d < NUM_DIRECTIONS; ++d)
        if (b->graph[d]) {
            (void)hipGraphExecDestroy(b->graph[d]);
            b->graph[d] = nullptr;
        }
    return SHT_OK;
}

int sht_batch_legendre(sht_batch *h, int direction, const double *const *in, double *const *out,
                       void *hip_stream)
{
    TraceRange tr("sht_batch_legendre");
    if (!reg_live(h, H_BATCH)) { set_error("invalid batch handle"); return SHT_ESTATE; }
    Batch *b = reinterpret_cast<Batch *>(h);
    int rc = check_batch_args(b, direction, in, out, true);
    if (rc) return rc;
    log_msg(2, "sht_batch_legendre direction %d, %d plans, stream %p", direction, (int)b->plans.size(), hip_stream);
    hipStream_t s = (hipStream_t)hip_stream;
    const int np = (int)b->plans.size();
    if ((rc = refresh_synth_queue(*b, s, false))) return rc;
    if (synth_direction(direction) && persistent_synth(*b)) {
        if ((rc = batch_legendre_synth(*b, direction, in, out, s))) return rc;
        for (int i = 0; i < np; ++i)
            if ((rc = launch_phase_tail_zero(*b->plans[i], out[i], s))) return rc;
    } else if (synth_direction(direction)) {
        if ((rc = fork_chains(*b, s))) return rc;
        for (int i = 0; i < np; ++i) {
            const hipStream_t cs = chain_stream(*b, i, s);
            if ((rc = plan_legendre_synth(*b, i, direction, in[i], out[i], cs))) return rc;
            if ((rc = launch_phase_tail_zero(*b->plans[i], out[i], cs))) return rc;
        }
        if ((rc = join_chains(*b, s))) return rc;
    } else {
        if ((rc = batch_legendre_anal(*b, direction, in, out, s))) return rc;
    }
    return finish_launch("sht_batch_legendre");
}

int sht_batch_execute(sht_batch *h, int direction, const double *const *in, double *const *out,
                      void *hip_stream)
{
    TraceRange tr("sht_batch_execute");
    if (!reg_live(h, H_BATCH)) { set_error("invalid batch handle"); return SHT_ESTATE; }
    Batch *b = reinterpret_cast<Batch *>(h);
    int rc0 = check_batch_args(b, direction, in, out, false);
    if (rc0) return rc0;
    if ((rc0 = refresh_synth_queue(*b, (hipStream_t)hip_stream, false))) return rc0;
    log_msg(2, "sht_batch_execute direction %d, %d plans, stream %p", direction, (int)b->plans.size(), hip_stream);
    const int np = (int)b->plans.size();
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
        log_msg(2, "batch: capturing direction %d into a graph", direction);
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
    log_msg(1, "batch destroyed (%d plans)", (int)b->plans.size());
    reg_remove(b);
    (void)hipDeviceSynchronize();
    batch_free(b);
    delete b;
}

int sht_autotune(sht_plan *h, double budget_seconds)
{
    TraceRange tr("sht_autotune");
    Plan *p = plan_of(h);
    if (!p) { set_error("invalid plan handle"); return SHT_ESTATE; }
    if (!(budget_seconds >= 0.0)) { set_error("budget must be >= 0"); return SHT_EINVAL; }
    fault_arm();
    const std::string key = tune_key(*p);
    sht_tuning cached{};
    if (tune_cache_lookup(key, cached) && tuning_check(*p, cached) == SHT_OK) {
        log_msg(1, "plan %llu: cached tuning %s", (unsigned long long)p->serial, tune_text(cached).c_str());
        return apply_tuning(*p, cached);
    }
    if (budget_seconds == 0.0) return SHT_OK;

    // candidates of each knob; the synthesis and the analysis knobs are
    // independent of each other and are timed on their own kernels
    const int cols = p->ntrans * (p->spin ? 4 : 2);
    std::vector<int> s_ncb = {1}, a_ncb = {1};
    if (cols > 16) {
        s_ncb.push_back(2);
        a_ncb.push_back(2);
    }
    const std::vector<int> s_mb = {2, 4, 8};
    // scratch operands: zero coefficients and phases (the kernels' time does
    // not depend on the values)
    double *alm = nullptr;
    const size_t abytes = (size_t)p->ntrans * p->ncomp * p->nalm * 16;
    int rc = dev_alloc((void **)&alm, abytes, "autotune scratch");
    if (rc) return rc;
    rc = check_hip(hipMemset(alm, 0, abytes), "autotune scratch");
    if (!rc) rc = check_hip(hipMemset(p->d_phase, 0, (size_t)p->phase_elems * 16), "autotune scratch");
    const sht_tuning orig = p->tune;
    sht_tuning best = orig;
    best.valu = 0;   // the matrix-core knobs first, then the vector path against them
    const auto t_start = std::chrono::steady_clock::now();
    auto spent = [&] {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    };
    double best_ms = 1e300;
    for (size_t i = 0; i < s_ncb.size() && !rc; ++i)
        for (size_t j = 0; j < s_mb.size() && !rc; ++j) {
            sht_tuning c = best;
            c.synth_ncb = s_ncb[i];
            c.synth_mblock = s_mb[j];
            if (tuning_check(*p, c) != SHT_OK) continue;
            if ((rc = apply_tuning(*p, c))) break;
            double ms = 0.0;
            rc = time_launches([&] { return launch_legendre_synth(*p, alm, p->d_phase, false, nullptr); }, 2, ms);
            if (!rc && ms < best_ms) {
                best_ms = ms;
                best = c;
            }
            if (spent() > budget_seconds) break;
        }
    best_ms = 1e300;
    const sht_tuning after_synth = best;
    for (size_t i = 0; i < a_ncb.size() && !rc; ++i) {
        sht_tuning c = after_synth;
        c.anal_ncb = a_ncb[i];
        c.anal_tpw = anal_tpw_built(p->spin, c.anal_ncb);
        if (tuning_check(*p, c) != SHT_OK) continue;
        if ((rc = apply_tuning(*p, c))) break;
        double ms = 0.0;
        rc = time_launches([&] { return launch_legendre_anal(*p, p->d_phase, alm, 0, nullptr); }, 2, ms);
        if (!rc && ms < best_ms) {
            best_ms = ms;
            best = c;
        }
        if (spent() > budget_seconds) break;
    }
    // vector-unit kernels (FP64) against the best matrix-core shape, on the
    // time of one synthesis plus one analysis
    if (!rc && p->precision == SHT_FP64) {
        double pair_ms[2] = {1e300, 1e300};
        for (int vv = 0; vv < 2 && !rc; ++vv) {
            sht_tuning c = best;
            c.valu = vv;
            if ((rc = apply_tuning(*p, c))) break;
            double ms1 = 0.0, ms2 = 0.0;
            rc = time_launches([&] { return launch_legendre_synth(*p, alm, p->d_phase, false, nullptr); }, 2, ms1);
            if (!rc) rc = time_launches([&] { return launch_legendre_anal(*p, p->d_phase, alm, 0, nullptr); }, 2, ms2);
            pair_ms[vv] = ms1 + ms2;
        }
        if (!rc) best.valu = pair_ms[1] < pair_ms[0] ? 1 : 0;
    }
    dev_free(alm);
    const int rc2 = apply_tuning(*p, rc ? orig : best);
    if (rc) return rc;
    if (rc2) return rc2;
    tune_cache_store(key, best);
    log_msg(1, "plan %llu: autotuned %s", (unsigned long long)p->serial, tune_text(best).c_str());
    return SHT_OK;
}

}  // extern "C"
