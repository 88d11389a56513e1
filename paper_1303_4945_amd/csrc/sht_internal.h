// Internal declarations of libsht (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/sht.h"
#include "host.h"

namespace sht {

const Geom *geom_of(const sht_geom *g);   // registered geometry or nullptr

// wavefronts per analysis work group: eight for spin > 0 in FP64 (half the
// passes over a_lm of four; the LDS then holds one work group per CU), four
// for spin 0 (measured faster) and in the FP32 form (whose separate partial-sum
// buffers would not fit eight)
constexpr int ana_nw(bool f32, bool spin) { return (f32 || !spin) ? 4 : 8; }
constexpr int NUM_XCD = 8;      // accelerator dies of the MI355X (work groups go round robin)

// Synthesis work item of one wavefront: one m, one slot tile, one group of
// transforms starting at t0 (m < 0: padding, no work).
struct WaveItem {
    int m;
    int tile;
    int t0;
    int pad;
};

// Items of the persistent batch analysis kernel (plan index into the batch's
// tables): one m, or (queue of m pairs) m and m2 = mmax - m one after the other.
struct BatchAnaItem {
    int plan;
    int m;
    int t0;
    int m2;   // second m of the item (-1: none)
};

// Items of the persistent batch synthesis kernel: one wavefront's (m, slot
// tile, transform group) of one plan, or (queue of m pairs) the same tile and
// group at m and then at m2 = mmax - m (-1: none).
struct BatchSynItem {
    int plan;
    int m;
    int m2;
    int tile;
    int t0;
    int pad[3];
};
// Segment offsets of the synthesis queue, one segment per accelerator die.
struct SynQueues {
    int ofs[NUM_XCD + 1];
};

// Device-side view of one plan for the Legendre kernels.
struct LegView {
    int lmax, mmax, spin, ntrans, nrings, nslots, ntiles;
    int rescale_bits;       // S
    int thresh_bits;        // T_r: rescale when |mu| >= 2^T_r
    double polar_T;         // Eq. 8 (<0: no polar skip)
    const double *slot_cos, *slot_sin, *slot_chalf, *slot_shalf;
    const int *slot_yn, *slot_ys;
    const double4 *coef;        // (alpha, beta, delta+, delta-) per (m, l)
    const double *fl;           // f_l per (m, l): lambda = f mu
    const int64_t *coef_ofs;    // coef + coef_ofs[m] + l  for l >= l0(m) (same for fl)
    const StartCoef *start;     // [m][chain] chain 0: +s (or 0), chain 1: -s
    const int *tile_mlim;       // per tile: largest m with an active slot (-1: none)
    const double *zeros;        // 2 (lmax + 1) zeros: operand source of unused columns
    const double *dfac;         // sqrt(l (l + 1)), l = 0 .. lmax + 1 (derivative synthesis)
    int64_t nalm;
};

struct FftRing;  // per-ring FFT descriptor (ringfft.hip)

struct FftPlan {
    // device tables
    void *d_rows = nullptr;      // FftRow[]: one entry per FFT work item
    int nrows = 0;
    double2 *d_tw = nullptr;     // twiddle tables, all lengths
    int *d_perm = nullptr;       // digit-reversal permutations
    double2 *d_blue = nullptr;   // Bluestein chirps and kernel spectra
    int *d_mvalid = nullptr;     // per ring: largest m whose F/G entry is meaningful
    double2 *d_phase_rot = nullptr;  // per ring: e^{i m phi0} tables (coarse/fine)
    size_t table_bytes = 0;
};

struct Plan {
    uint64_t serial = 0;             // registry serial of this plan
    uint64_t generation = 0;         // bumped whenever its work lists change (autotuner)
    int device = 0;
    int lmax = 0, mmax = 0, spin = 0, ntrans = 0, precision = 0, ncomp = 1;
    Geom geom;
    sht_plan_opts opts{};
    double polar_T = 100.0;
    int rescale_bits = 256;
    int flush_chunks = 4;
    bool real_h = false;             // real spherical harmonics storage
    double *d_rh = nullptr;          // its conversion workspace (coefficients)
    int64_t nalm = 0;
    // slots
    std::vector<SlotHost> slots;
    int nslots = 0, ntiles = 0, slots_per_tile = 32;
    std::vector<int> tile_mlim;
    // host-side work lists
    std::vector<WaveItem> synth_items;
    sht_tuning tune{};               // launch shapes (synthesis column blocks, m blocks, ...)
    std::vector<int> anal_ms;
    // device memory
    double *d_slot_cos = nullptr, *d_slot_sin = nullptr, *d_slot_chalf = nullptr,
           *d_slot_shalf = nullptr;
    int *d_slot_yn = nullptr, *d_slot_ys = nullptr;
    double4 *d_coef = nullptr;
    double *d_fl = nullptr;
    int64_t *d_coef_ofs = nullptr;
    StartCoef *d_start = nullptr;
    int *d_tile_mlim = nullptr;
    double *d_zeros = nullptr;
    double *d_dfac = nullptr;
    WaveItem *d_synth_items = nullptr;
    int *d_anal_ms = nullptr;
    double *d_phase = nullptr;       // F / G workspace
    int64_t phase_elems = 0;         // complex elements
    FftPlan fft;
    double flops_rec = 0, flops_prod = 0, hbm_bytes = 0;   // recursion, products (one direction)
    int64_t n_items = 0;
    PlanShape shape() const
    {
        PlanShape ps;
        ps.lmax = lmax; ps.mmax = mmax; ps.spin = spin; ps.ntrans = ntrans; ps.polar_T = polar_T;
        return ps;
    }
};

constexpr int MAX_BATCH_PLANS = 64;

// analysis kernel mode bits
constexpr int ANA_MODE_GRAD = 1;    // real-field gradient factor fac_m
constexpr int ANA_MODE_DERIV = 2;   // adjoint of the derivative synthesis
// (real spherical harmonics: no fac_m, the gradient is the plain transpose)
inline int anal_mode(int d, bool real_h)
{
    return ((!real_h && (d == SHT_ALM2MAP_GRAD || d == SHT_ALM2MAP_DERIV1_GRAD)) ? ANA_MODE_GRAD : 0) |
           (deriv_direction(d) ? ANA_MODE_DERIV : 0);
}

// Legendre-step operands of the plans of a batch, passed by value to the
// persistent kernels (so that a captured graph holds them as parameters).
struct BatchPtrs {
    const double *in[MAX_BATCH_PLANS];
    double *out[MAX_BATCH_PLANS];
};

struct Batch {
    std::vector<Plan *> plans;
    int queue_order = SHT_QUEUE_COST;    // analysis queue: by cost, or (m, mmax - m) pairs
    int concurrent = 1;                  // per-plan launch chains on concurrent streams
    std::vector<hipStream_t> aux;        // one stream per plan (default priority)
    std::vector<hipEvent_t> join;        // one event per plan, plus the fork event last
    std::vector<uint64_t> plan_serial;   // registry serials of the borrowed plans
    int device = 0;
    int ana_groups = 1;                  // work groups of the persistent analysis launch
    int spin = 0, precision = 0, ana_ncb = 1;
    bool real_h = false;
    int nana = 0;
    LegView *d_views = nullptr;
    BatchAnaItem *d_ana = nullptr;
    unsigned *d_counter = nullptr;       // [0]: analysis queue, [16 (1 + d)]: synthesis queue of die d
    // persistent synthesis (concurrent == 2): one queue over all plans, built
    // for the plans' tunings at the generations in syn_gen; syn_ok: every plan
    // on the matrix-core path with the same column blocks and carry interval
    bool syn_ok = false;
    int nsyn = 0, syn_groups = 1, syn_ncb = 1, syn_flush = 4;
    int syn_ofs[NUM_XCD + 1] = {};       // items of die d: d_syn[syn_ofs[d] .. syn_ofs[d + 1])
    BatchSynItem *d_syn = nullptr;
    std::vector<uint64_t> syn_gen;
    // captured graphs, one per direction, keyed by the user pointers and the
    // plans' generations (a retuned plan has new item lists and launch shapes)
    hipGraphExec_t graph[NUM_DIRECTIONS] = {};
    std::vector<uintptr_t> graph_key[NUM_DIRECTIONS];
    hipStream_t graph_stream[NUM_DIRECTIONS] = {};
};

LegView make_leg_view(const Plan &p);

// Legendre step launchers (legendre.hip)
int launch_legendre_synth(const Plan &p, const double *alm, double *phase, bool deriv, hipStream_t s);
int synth_ncb_default(int spin, int ntrans, int precision);
int build_synth_items(Plan &p);
// tuning: defaults for a plan, validity (SHT_OK or SHT_EUNSUPPORTED with a
// message), and applying one (rebuilds the work lists, bumps the generation)
sht_tuning default_tuning(const Plan &p);
int tuning_check(const Plan &p, const sht_tuning &t);
int apply_tuning(Plan &p, const sht_tuning &t);
int anal_tpw_built(int spin, int ncb);   // tiles per wavefront of the built analysis kernels
int valu_jpg(const Plan &p);             // transforms per work item of the vector-unit kernels
int valu_k(const Plan &p, bool anal);    // slot tiles per lane group of the vector-unit kernels
int launch_legendre_anal(const Plan &p, const double *phase, double *alm, int mode, hipStream_t s);

// persistent batch launchers (legendre.hip); pointer tables already staged in b.d_ptr
int launch_legendre_anal_batch(const Batch &b, const BatchPtrs &ptrs, int mode, hipStream_t s);
int launch_legendre_synth_batch(const Batch &b, const BatchPtrs &ptrs, bool deriv, hipStream_t s);
// work groups (one wavefront each) of the persistent synthesis launch on the given device
int synth_batch_groups(int spin, int ncb, bool f32, int device);
// work groups of the persistent analysis launch on the given device
int anal_batch_groups(int spin, int ncb, bool f32, int device);
int anal_ncb(int spin, int ntrans);

// ring FFT (ringfft.hip)
int fft_plan_build(Plan &p);
void fft_plan_free(FftPlan &f);
int launch_ring_synth(const Plan &p, const double *phase, double *map, bool use_weights, hipStream_t s);
int launch_ring_anal(const Plan &p, const double *map, double *phase, bool use_weights,
                     hipStream_t s);
int launch_phase_tail_zero(const Plan &p, double *phase, hipStream_t s);

// real spherical harmonics storage <-> complex a_lm (realharm.hip)
int launch_real_harm(const Plan &p, const double *in, double *out, int ncomp, bool to_complex, hipStream_t s);

// device memory helpers
int dev_alloc(void **ptr, size_t bytes, const char *what);
void dev_free(void *ptr);
int dev_upload(void *dst, const void *src, size_t bytes, const char *what);
int check_hip(hipError_t e, const char *what);
int check_exec_args(const Plan *p, int direction, const void *in, const void *out, bool fft_only,
                    bool leg_only);
Plan *plan_of(sht_plan *h);   // registered plan or nullptr
int finish_launch(const char *what);
int execute_with(const Plan &p, int direction, const double *in, double *out, double *phase, double *rh,
                 hipStream_t s);
// bytes of the workspaces of one full transform (phases, real-harmonics coefficients)
size_t exec_workspace_bytes(const Plan &p, size_t *rh_offset);
// static device scratch of the allocation-free entry point (noalloc.hip):
// resolves its address on the device (once per device)
int scratch_init(int device);

}  // namespace sht
