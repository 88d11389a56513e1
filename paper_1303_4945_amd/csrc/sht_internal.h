// Internal declarations of libsht (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/sht.h"

namespace sht {

constexpr uint32_t kGeomMagic = 0x53474d31u;   // live geometry
constexpr uint32_t kPlanMagic = 0x53504c31u;   // live plan
constexpr uint32_t kBatchMagic = 0x53424331u;  // live batch
constexpr uint32_t kDeadMagic = 0xdeadbeefu;

void set_error(const char *fmt, ...);

struct Geom {
    uint32_t magic = kGeomMagic;
    int nrings = 0;
    std::vector<double> theta, phi0, weight;
    std::vector<int64_t> nphi, ofs;
    int64_t stride = 1;
    bool has_weight = false;
    int64_t npix = 0;
};

// One recurrence chain slot: a ring and (optionally) its mirror ring.
// The recursion runs at the representative colatitude t <= pi/2 of the slot;
// the ring at pi - t (if any) follows from the parity relation.
struct SlotHost {
    int yn = -1, ys = -1;       // ring at t and ring at pi - t (-1: none)
    double cth = 0, sth = 0;    // cos t >= 0, sin t
    double chalf = 0, shalf = 0;  // cos t/2, sin t/2
};

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

// Items of the persistent batch analysis kernel (plan index into the batch's tables).
struct BatchAnaItem {
    int plan;
    int m;
    int t0;
    int pad;
};

// Per-(m, chain) start value: lambda_{l0} = sign * K * cos(t/2)^p * sin(t/2)^q.
struct StartCoef {
    double kmant;   // mantissa of K in [0.5, 1)
    int kexp;       // binary exponent of K
    int p, q;       // powers of cos(theta/2), sin(theta/2)
    int sign;       // +1 / -1
    int pad;
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
    uint32_t magic = kPlanMagic;
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
    int synth_ncb = 1;               // column blocks (16 columns) per synthesis item
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
    double flops_synth = 0, flops_anal = 0, hbm_bytes = 0;
    int64_t n_items = 0;
    // tuning
    int synth_waves = 1;
};

constexpr int MAX_BATCH_PLANS = 64;

// Legendre-step operands of the plans of a batch, passed by value to the
// persistent kernels (so that a captured graph holds them as parameters).
// directions of sht_execute (SHT_ALM2MAP .. SHT_ALM2MAP_DERIV1_GRAD); the
// ones that go from a_lm to maps run the synthesis kernels
constexpr int NUM_DIRECTIONS = 8;
inline bool synth_direction(int d)
{
    return d == SHT_ALM2MAP || d == SHT_MAP2ALM_ADJOINT || d == SHT_ALM2MAP_DERIV1;
}
// first-derivative synthesis and its adjoints: spin-1 plans, one a_lm component
inline bool deriv_direction(int d)
{
    return d == SHT_ALM2MAP_DERIV1 || d == SHT_ALM2MAP_DERIV1_ADJOINT || d == SHT_ALM2MAP_DERIV1_GRAD;
}
// ring weights in the FFT step: analysis and the adjoint of analysis
inline bool weighted_direction(int d) { return d == SHT_MAP2ALM || d == SHT_MAP2ALM_ADJOINT; }
// analysis kernel mode bits
constexpr int ANA_MODE_GRAD = 1;    // real-field gradient factor fac_m
constexpr int ANA_MODE_DERIV = 2;   // adjoint of the derivative synthesis
// (real spherical harmonics: no fac_m, the gradient is the plain transpose)
inline int anal_mode(int d, bool real_h)
{
    return ((!real_h && (d == SHT_ALM2MAP_GRAD || d == SHT_ALM2MAP_DERIV1_GRAD)) ? ANA_MODE_GRAD : 0) |
           (deriv_direction(d) ? ANA_MODE_DERIV : 0);
}

struct BatchPtrs {
    const double *in[MAX_BATCH_PLANS];
    double *out[MAX_BATCH_PLANS];
};

struct Batch {
    uint32_t magic = kBatchMagic;
    std::vector<Plan *> plans;
    int spin = 0, precision = 0, ana_ncb = 1;
    bool real_h = false;
    int nana = 0;
    LegView *d_views = nullptr;
    BatchAnaItem *d_ana = nullptr;
    unsigned *d_counter = nullptr;
    // captured graphs, one per direction, keyed by the user pointers
    hipGraphExec_t graph[NUM_DIRECTIONS] = {};
    std::vector<const void *> graph_key[NUM_DIRECTIONS];
    hipStream_t graph_stream[NUM_DIRECTIONS] = {};
};

LegView make_leg_view(const Plan &p);

// Legendre step launchers (legendre.hip)
int launch_legendre_synth(const Plan &p, const double *alm, double *phase, bool deriv, hipStream_t s);
int synth_ncb_default(int spin, int ntrans, int precision);
int build_synth_items(Plan &p);
int launch_legendre_anal(const Plan &p, const double *phase, double *alm, int mode, hipStream_t s);

// persistent batch launchers (legendre.hip); pointer tables already staged in b.d_ptr
int launch_legendre_anal_batch(const Batch &b, const BatchPtrs &ptrs, int mode, hipStream_t s);
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
int finish_launch(const char *what);

}  // namespace sht
