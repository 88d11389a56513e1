// The allocation-free transform entry point: the phase (and real-harmonics)
// workspace of a full transform lives in a statically sized device array of
// the library instead of the plan's allocation.  For callers that cannot
// allocate device memory while they run (work captured into a graph, tight
// serving loops, harnesses that forbid allocation).
//
// The array is a file-scope device variable: each device that loads the
// library holds its own copy until the process ends.  Its address is resolved
// with hipGetSymbolAddress once per device, at plan creation (the array's name
// in host code is only a stand-in for the symbol, never a device address).
// Every call on one device shares that device's copy; calls that overlap on one
// device (different streams without ordering) race on it.  Nothing in it must
// start at zero: each transform writes every workspace entry it reads.
#include <hip/hip_runtime.h>

#include <mutex>
#include <unordered_map>

#include "sht_internal.h"
#include "trace.h"

namespace sht {

constexpr size_t SCRATCH_BYTES = size_t(64) << 20;   // 64 MiB per device

static __device__ __align__(256) double2 scratch[SCRATCH_BYTES / sizeof(double2)];

static std::mutex g_scratch_mu;
static std::unordered_map<int, void *> g_scratch_ptr;   // device -> address of its copy

int scratch_init(int device)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr.count(device)) return SHT_OK;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != device) {
        (void)hipGetLastError();
        set_error("scratch set-up: device %d is not current", device);
        return SHT_EDEVICE;
    }
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();
        set_error("hipGetSymbolAddress of the static scratch failed: %s", hipGetErrorString(e));
        return SHT_EDEVICE;
    }
    g_scratch_ptr[device] = ptr;
    return SHT_OK;
}

static void *scratch_of(int device)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    return it == g_scratch_ptr.end() ? nullptr : it->second;
}

size_t exec_workspace_bytes(const Plan &p, size_t *rh_offset)
{
    const size_t ph = ((size_t)p.phase_elems * 16 + 255) / 256 * 256;
    const size_t rh = p.real_h ? (size_t)p.ntrans * p.ncomp * p.nalm * 16 : 0;
    if (rh_offset) *rh_offset = ph;
    return ph + rh;
}

}  // namespace sht

using namespace sht;

extern "C" {

int sht_execute_noalloc(sht_plan *h, int direction, const double *in, double *out, void *hip_stream)
{
    TraceRange tr("sht_execute_noalloc");
    Plan *p = plan_of(h);
    if (!p) { set_error("invalid plan handle"); return SHT_ESTATE; }
    int rc = check_exec_args(p, direction, in, out, false, false);
    if (rc) return rc;
    log_msg(2, "sht_execute_noalloc plan %llu direction %d stream %p", (unsigned long long)p->serial, direction,
            hip_stream);
    size_t rh_ofs = 0;
    const size_t need = exec_workspace_bytes(*p, &rh_ofs);
    if (need > SCRATCH_BYTES) {
        set_error("the plan needs %zu bytes of workspace; the static scratch holds %zu (use sht_execute)", need,
                  SCRATCH_BYTES);
        return SHT_EINVAL;
    }
    char *base = static_cast<char *>(scratch_of(p->device));
    if (!base) {   // set-up failed at plan creation: one more try (device is current)
        if ((rc = scratch_init(p->device))) return rc;
        base = static_cast<char *>(scratch_of(p->device));
    }
    double *phase = reinterpret_cast<double *>(base);
    double *rh = p->real_h ? reinterpret_cast<double *>(base + rh_ofs) : nullptr;
    return execute_with(*p, direction, in, out, phase, rh, (hipStream_t)hip_stream);
}

int sht_noalloc_capacity(int64_t *bytes)
{
    if (!bytes) { set_error("bytes is NULL"); return SHT_EINVAL; }
    *bytes = (int64_t)SCRATCH_BYTES;
    return SHT_OK;
}

}  // extern "C"
