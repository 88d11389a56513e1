// Host-only part of libsht (no HIP types): error reporting, the registry of
// live handles, ring geometries and the per-plan tables that are computed on
// the CPU (ring-pair slots, polar limits of Eqs. 7-8, recursion coefficients
// and start values of Sect. 4.1, work counts).  Compiled into the library and,
// on its own, into the sanitizer test driver.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/sht.h"

namespace sht {

void set_error(const char *fmt, ...);

// Diagnostics on stderr, one line each, by the level in $SHT_LOG (read once):
// 0 off (default), 1 handles created and destroyed, tuning choices and errors,
// 2 also every entry-point call, 3 also every kernel launch with its grid.
int log_level();
void log_msg(int level, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

// ---- registry of live handles --------------------------------------------
// A handle is valid while it is registered; it is looked up before anything
// is read through it, so a destroyed (or never created) handle is rejected
// without touching freed memory.  Every registration gets a new serial, so a
// new object that reuses a freed address is told apart from the old one.
enum HandleKind { H_GEOM = 1, H_PLAN = 2, H_BATCH = 3 };
uint64_t reg_add(const void *obj, int kind);
bool reg_live(const void *obj, int kind, uint64_t *serial = nullptr);
void reg_remove(const void *obj);

// ---- device allocation bookkeeping (diagnostics and fault injection) ------
// SHT_FAULT_INJECT=alloc makes the first device allocation of a create call
// fail, alloc:N the N-th one; fault_arm() is called at the start of every
// call that allocates.
void fault_arm();
bool fault_should_fail();
void mem_count(int64_t buffers, int64_t bytes);
void mem_stats(int64_t *buffers, int64_t *bytes);

// ---- geometry --------------------------------------------------------------
struct Geom {
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
    int yn = -1, ys = -1;         // ring at t and ring at pi - t (-1: none)
    double cth = 0, sth = 0;      // cos t >= 0, sin t
    double chalf = 0, shalf = 0;  // cos t/2, sin t/2
};

// Per-(m, chain) start value: lambda_{l0} = sign * K * cos(t/2)^p * sin(t/2)^q.
struct StartCoef {
    double kmant;   // mantissa of K in [0.5, 1)
    int kexp;       // binary exponent of K
    int p, q;       // powers of cos(theta/2), sin(theta/2)
    int sign;       // +1 / -1
    int pad;
};

// Step coefficients of one degree (alpha, beta, alpha + beta - 2, alpha - beta - 2);
// the same 32-byte layout as the device's double4.
struct alignas(32) Coef4 {
    double x, y, z, w;
};

// Band limits and options that the table builders need.
struct PlanShape {
    int lmax = 0, mmax = 0, spin = 0, ntrans = 1;
    double polar_T = 100.0;   // < 0: no polar skipping
};

void build_slots(const Geom &g, std::vector<SlotHost> &slots);
// largest m whose terms the polar criterion keeps at this slot (-1: none)
int slot_mlim(const PlanShape &ps, const SlotHost &s);
void build_coef(const PlanShape &ps, std::vector<Coef4> &coef, std::vector<double> &fl,
                std::vector<int64_t> &ofs);
void build_start(const PlanShape &ps, std::vector<StartCoef> &st);
// (m, slot, l) triples left after polar skipping, slots grouped into tiles
// whose polar limit is the largest of their slots
double count_triples(const PlanShape &ps, const std::vector<SlotHost> &slots, int slots_per_tile);

// Validation of a transform call shared by every entry point: direction,
// pointers, weights, spin of the derivative directions and non-overlap of
// the byte ranges of input and output.
int validate_exec(int direction, int spin, bool has_weight, size_t alm_bytes, size_t map_bytes,
                  size_t phase_bytes, const void *in, const void *out, bool stage_fft, bool stage_leg);

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

}  // namespace sht
