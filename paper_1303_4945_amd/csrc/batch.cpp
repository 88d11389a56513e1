// Batches of plans and the tile autotuner.
#include <hip/hip_runtime.h>

#include <new>

#include "sht_internal.h"

using namespace sht;

extern "C" {

int sht_batch_create(int nplans, sht_plan *const *plans, sht_batch **out)
{
    if (!out) { set_error("out is NULL"); return SHT_EINVAL; }
    *out = nullptr;
    if (nplans < 1 || !plans) { set_error("need at least one plan"); return SHT_EINVAL; }
    Batch *b = new (std::nothrow) Batch();
    if (!b) { set_error("host allocation failed"); return SHT_ENOMEM; }
    int spin = -1;
    for (int i = 0; i < nplans; ++i) {
        Plan *p = reinterpret_cast<Plan *>(plans[i]);
        if (!p || p->magic != kPlanMagic) {
            delete b;
            set_error("plan %d is not a valid plan", i);
            return SHT_ESTATE;
        }
        if (spin >= 0 && p->spin != spin) {
            delete b;
            set_error("all plans of a batch must have the same spin");
            return SHT_EINVAL;
        }
        spin = p->spin;
        b->plans.push_back(p);
    }
    *out = reinterpret_cast<sht_batch *>(b);
    return SHT_OK;
}

int sht_batch_execute(sht_batch *h, int direction, const double *const *in, double *const *out,
                      void *hip_stream)
{
    Batch *b = reinterpret_cast<Batch *>(h);
    if (!b || b->magic != kBatchMagic) { set_error("invalid batch handle"); return SHT_ESTATE; }
    if (!in || !out) { set_error("in and out arrays are required"); return SHT_EINVAL; }
    for (size_t i = 0; i < b->plans.size(); ++i) {
        int rc = sht_execute(reinterpret_cast<sht_plan *>(b->plans[i]), direction, in[i], out[i],
                             hip_stream);
        if (rc) return rc;
    }
    return SHT_OK;
}

void sht_batch_destroy(sht_batch *h)
{
    Batch *b = reinterpret_cast<Batch *>(h);
    if (!b || b->magic != kBatchMagic) return;
    b->magic = kDeadMagic;
    delete b;
}

int sht_autotune(sht_plan *h, double budget_seconds)
{
    Plan *p = reinterpret_cast<Plan *>(h);
    if (!p || p->magic != kPlanMagic) { set_error("invalid plan handle"); return SHT_ESTATE; }
    if (!(budget_seconds >= 0.0)) { set_error("budget must be >= 0"); return SHT_EINVAL; }
    return SHT_OK;
}

}  // extern "C"
