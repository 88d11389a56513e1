/*
 * sht.h -- C ABI of libsht, spherical harmonic transforms on AMD MI355X (gfx950).
 *
 * The operations follow Sect. 2 of Reinecke & Seljebotn (2013), "Libsharp --
 * spherical harmonic transforms revisited":
 *
 *   synthesis (alm2map, Eq. 1):  p_xy = sum_m sum_l a_lm lambda_lm(theta_y)
 *                                       exp(i m phi0_y + 2 pi i m x / Nphi_y)
 *   analysis  (map2alm, Eq. 2):  a_lm = sum_y sum_x p_xy w_y lambda_lm(theta_y)
 *                                       exp(-i m phi0_y - 2 pi i m x / Nphi_y)
 *   adjoint synthesis (Sect. 4.5, Eq. 16 with W = 1): the analysis sums with
 *                                 every weight equal to one (Y^T);
 *   adjoint analysis (Sect. 4.5):  W Y, the synthesis with every ring times w_y;
 *   first-derivative maps (Sect. 4.3): df/dtheta and df/(sin theta dphi) of a
 *                                 spin-0 field, as a spin-1 synthesis.
 *
 * Both are split into a Legendre step (Eqs. 4, 5: the phases F_{m,y}, G_{m,y})
 * and per-ring real FFTs (Eqs. 3, 6).  Every spin 0 <= s <= lmax is supported
 * (Sect. 4.1); several transforms of identical type run together (Sect. 3.2).
 *
 * Conventions
 *   - real fields: only m >= 0 is stored, a_{l,-m} = (-1)^m conj(a_lm);
 *     Im(a_l0) is ignored on input and returned as 0; coefficients with
 *     l < |spin| are ignored on input and returned as 0;
 *   - spin s > 0 takes E/B coefficients and Q/U maps with
 *     +-s a_lm = -(E_lm +- i B_lm), Q + iU = sum_lm s a_lm s Y_lm and
 *     Q - iU = (-1)^s sum_lm -s a_lm -s Y_lm (what real Q, U imply, since
 *     -s Y_lm = (-1)^(s+m) conj(s Y_l,-m)); for s = 2 the HEALPix convention;
 *   - the ring weights w_y of Eq. 2 include the 2 pi / Nphi_y factor
 *     (Gauss-Legendre: w_GL * 2 pi / Nphi; HEALPix: 4 pi / Npix).
 *
 * Layouts (double precision; complex numbers as interleaved (re, im) pairs,
 * never C99 complex, see Sect. 3.1):
 *   a_lm   double[ntrans][ncomp][nalm][2], index(l, m) = m(2 lmax + 1 - m)/2 + l
 *   maps   double[ntrans][ncomp][npix], pixel x of ring y at ofs[y] + x*stride
 *   phases double[ntrans][ncomp][nrings][mmax + 1][2]  (F for synthesis, G for
 *          analysis; ring index = the geometry's ring order)
 *   ncomp is 1 for spin 0 and 2 for spin s > 0 (E,B resp. Q,U).
 *
 * Memory and ownership
 *   - every data pointer passed to sht_execute / sht_legendre / sht_ring_fft
 *     is DEVICE memory owned by the caller; it is only borrowed for the
 *     stream-ordered work and must stay valid until that work completes;
 *   - geometry, plan and batch objects are owned by the library and freed by
 *     their destroy functions; a plan owns its device tables and its phase
 *     workspace (ntrans * ncomp * nrings * (mmax+1) * 16 bytes);
 *   - a plan (or batch) must not be executed on two streams at once.
 *
 * Errors
 *   Every function returns an sht_status (0 = SHT_OK) and never aborts or
 *   exits.  Arguments are validated on the host before any GPU work is
 *   queued.  The message of the last failure on the calling thread is
 *   available from sht_last_error().  Asynchronous device failures are
 *   reported as SHT_EDEVICE by a later call.
 */
#ifndef SHT_H
#define SHT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SHT_OK = 0,
    SHT_EINVAL = 1,        /* invalid argument */
    SHT_ENOMEM = 2,        /* host or device allocation failed */
    SHT_EDEVICE = 3,       /* no usable gfx950 device, or a HIP call failed */
    SHT_EUNSUPPORTED = 4,  /* valid request that this library does not implement */
    SHT_ESTATE = 5         /* object destroyed, corrupted, or in use */
} sht_status;

enum { SHT_FP64 = 0, SHT_FP32_MFMA = 1 };
enum { SHT_ALM2MAP = 0, SHT_MAP2ALM = 1, SHT_ALM2MAP_ADJOINT = 2, SHT_ALM2MAP_GRAD = 3,
       SHT_MAP2ALM_ADJOINT = 4, SHT_ALM2MAP_DERIV1 = 5, SHT_ALM2MAP_DERIV1_ADJOINT = 6,
       SHT_ALM2MAP_DERIV1_GRAD = 7 };

typedef struct sht_geom sht_geom;
typedef struct sht_plan sht_plan;
typedef struct sht_batch sht_batch;

/* Plan options; zero-initialise and set what is needed (NULL = defaults). */
typedef struct sht_plan_opts {
    int no_polar_skip;     /* 1: evaluate every (m, ring) term (Sect. 3.3 off) */
    double polar_T;        /* >0: override T of Eq. 8 (default max(100, 0.01 lmax)) */
    int rescale_bits;      /* >0: exponent step S of the extended-range recursion
                              (default 256; valid 64..700) */
    int flush_chunks;      /* FP32_MFMA: FP32 partial sums are carried into FP64
                              after this many 16-degree chunks (default 4) */
    int real_harmonics;    /* 1: coefficients in real spherical harmonics storage
                              (Sect. 4.5): r_lm in the slot of Re a_lm and r_l,-m
                              in the slot of Im a_lm (m > 0), with R_l0 = Y_l0,
                              R_lm = sqrt(2) Re Y_lm, R_l,-m = sqrt(2) Im Y_lm, i.e.
                              a_lm = (r_lm - i r_l,-m) / sqrt(2).  The transform is
                              then a plain real-linear map: SHT_ALM2MAP_ADJOINT and
                              SHT_ALM2MAP_GRAD both return its transpose (no fac_m),
                              and the same holds for the DERIV1 directions.  Costs
                              a workspace of the size of the coefficients. */
    int reserved[7];
} sht_plan_opts;

/* ---- geometry (Sect. 2, Sect. 4.4) ---- */

/* Arbitrary iso-latitude grid.  theta in [0, pi]; nphi >= 1; phi0: azimuth of
   the first pixel of each ring; weight: w_y of Eq. 2 (may be NULL: analysis
   is then unavailable, adjoint synthesis still works); ofs: first pixel index
   of each ring (NULL: rings stored back to back in the given order);
   stride: distance between neighbouring pixels of a ring (>= 1).
   All arrays are host memory of length nrings and are copied. */
int sht_geom_create(int nrings, const double *theta, const int64_t *nphi,
                    const double *phi0, const double *weight, const int64_t *ofs,
                    int64_t stride, sht_geom **out);
/* Gauss-Legendre grid: nrings rings at the roots of P_nrings(cos theta),
   north to south, nphi pixels each, weights w_GL * 2 pi / nphi. */
int sht_geom_gauss(int nrings, int64_t nphi, double phi0, sht_geom **out);
/* HEALPix ring-scheme grid (4 nside - 1 rings, 12 nside^2 pixels), uniform
   weights 4 pi / Npix. */
int sht_geom_healpix(int nside, sht_geom **out);

/* Equidistant-cylindrical (ECP) grids (Sect. 4.4, "Extended support for ECP
   grids"), nphi pixels per ring, north to south:
     SHT_ECP_FEJER1: nrings rings at (n + 1/2) pi / nrings, n = 0 .. nrings-1;
     SHT_ECP_FEJER2: nrings rings at n pi / (nrings + 1), n = 1 .. nrings;
     SHT_ECP_CC:     nrings >= 2 rings at n pi / (nrings - 1), n = 0 .. nrings-1
                     (both poles included).
   Weights: Fejer's first and second rules and the Clenshaw-Curtis rule for
   the integral over x = cos theta (exact for polynomials in x of degree
   nrings - 1), each times 2 pi / nphi. */
enum { SHT_ECP_FEJER1 = 0, SHT_ECP_FEJER2 = 1, SHT_ECP_CC = 2 };
int sht_geom_ecp(int nrings, int64_t nphi, int kind, double phi0, sht_geom **out);

/* Reduced Gauss-Legendre grid (Sect. 4.4, "Reduced Gauss-Legendre grid"): the
   rings of sht_geom_gauss(nrings, ...), ring y with 2 m_y + 1 pixels rounded up
   to the next integer whose prime factors are 2, 3 and 5 (at most nphi_max),
   where m_y <= mmax is the largest m whose terms the polar criterion of
   Eqs. 7-8 keeps at that ring for lmax and spin (threshold T = max(100,
   lmax / 100), |cos theta| for both spin signs).  Weights w_GL * 2 pi / nphi_y.
   Not exact for analysis, but accurate to the criterion's precision. */
int sht_geom_reduced_gauss(int nrings, int64_t nphi_max, int lmax, int mmax, int spin, double phi0,
                           sht_geom **out);
/* Number of rings and of map pixels (max pixel index + 1). */
int sht_geom_info(const sht_geom *g, int *nrings, int64_t *npix);
/* Copy the ring tables out (any pointer may be NULL). */
int sht_geom_rings(const sht_geom *g, double *theta, int64_t *nphi, double *phi0,
                   double *weight, int64_t *ofs);
void sht_geom_destroy(sht_geom *g);

/* ---- a_lm indexing (m-major triangle, Sect. 2) ---- */
int64_t sht_alm_index(int lmax, int l, int m);   /* m(2 lmax + 1 - m)/2 + l */
int64_t sht_nalm(int lmax, int mmax);            /* number of stored a_lm */

/* ---- plans ---- */

/* A plan binds a geometry (copied), band limits lmax >= mmax >= 0, a spin
   0 <= spin <= lmax, the number of simultaneous transforms ntrans >= 1 (Sect. 3.2)
   and the arithmetic of the Legendre step (SHT_FP64, or SHT_FP32_MFMA: FP64
   recursion, FP32 matrix-core products with FP64 carry).  Uses the current
   HIP device. */
int sht_plan_create(const sht_geom *g, int lmax, int mmax, int spin, int ntrans,
                    int precision, const sht_plan_opts *opts, sht_plan **out);
void sht_plan_destroy(sht_plan *p);

/* Full transform, stream-ordered on hip_stream (a hipStream_t; NULL = null stream).
   SHT_ALM2MAP: in = a_lm, out = maps.  SHT_MAP2ALM: in = maps, out = a_lm
   (needs weights).  SHT_ALM2MAP_ADJOINT: in = maps, out = Y^T maps.
   SHT_ALM2MAP_GRAD: in = dL/dmap of a real loss L, out = dL/dRe a + i dL/dIm a for
   the stored coefficients (m >= 0), i.e. fac_m Y^T g with fac_0 = 1 and
   fac_m = 2 for m > 0, because a_{l,-m} = (-1)^m conj(a_lm) enters the map too;
   entries the synthesis ignores (Im a_l0, l < |spin|) get gradient 0.
   SHT_MAP2ALM_ADJOINT (Sect. 4.5, the adjoint of analysis Y^T W): in = a_lm,
   out = W Y a, the synthesis with every ring multiplied by its weight w_y
   (needs weights).  For real maps x the pair satisfies
   <x, W Y a> = sum over l, m >= 0 of fac_m Re(a_lm conj((Y^T W x)_lm)).
   SHT_ALM2MAP_DERIV1 (Sect. 4.3, maps of first derivatives; needs a plan of
   spin 1): in = spin-0 a_lm of a real field f, laid out [ntrans][1][nalm][2];
   out = maps [ntrans][2][npix] holding df/dtheta and df/(sin theta dphi).
   Computed as the spin-1 synthesis of E_lm = sqrt(l (l + 1)) a_lm, B_lm = 0.
   SHT_ALM2MAP_DERIV1_ADJOINT: in = maps [ntrans][2][npix], out = its adjoint
   [ntrans][1][nalm][2], sqrt(l (l + 1)) times the E part of the spin-1 Y^T;
   SHT_ALM2MAP_DERIV1_GRAD: the same times fac_m (the gradient of a real loss).
   in and out must not overlap. */
int sht_execute(sht_plan *p, int direction, const double *in, double *out,
                void *hip_stream);

/* Allocation-free form of sht_execute, for callers that cannot allocate device
   memory while they run: work captured into a HIP graph, tight serving loops,
   harnesses that forbid allocation.  Same arguments, directions and results
   (bit for bit) as sht_execute; the plan's phase workspace (and, with
   real_harmonics, its coefficient workspace) is replaced by a static device
   array of the library of 64 MiB per device (sht_noalloc_capacity), which each
   device holds from the first plan creation on it until the process ends.
   The call allocates nothing.  SHT_EINVAL when the plan needs more workspace
   than that (ntrans * ncomp * nrings * (mmax + 1) * 16 bytes of phases, plus
   ntrans * ncomp * nalm * 16 with real_harmonics).  Every call on one device
   shares that device's array: calls that overlap in time on one device (on
   streams not ordered with each other) race and give undefined results. */
int sht_execute_noalloc(sht_plan *p, int direction, const double *in, double *out,
                        void *hip_stream);
/* Bytes of the static workspace of sht_execute_noalloc. */
int sht_noalloc_capacity(int64_t *bytes);

/* Legendre step only (Eqs. 4, 5).  SHT_ALM2MAP (and SHT_MAP2ALM_ADJOINT, the
   same Legendre step): in = a_lm, out = F phases; SHT_ALM2MAP_DERIV1: in =
   spin-0 a_lm, out = F phases of the derivative maps.
   SHT_MAP2ALM / SHT_ALM2MAP_ADJOINT / SHT_ALM2MAP_GRAD: in = G phases, out = a_lm
   (GRAD also applies fac_m); the DERIV1 adjoints: out = one component.
   Phase entries of (m, ring) terms that the polar criterion (Eqs. 7-8) drops
   are returned as zero, here and from sht_ring_fft. */
int sht_legendre(sht_plan *p, int direction, const double *in, double *out,
                 void *hip_stream);

/* Ring FFT step only (Eqs. 3, 6).  SHT_ALM2MAP: in = F phases, out = maps.
   SHT_MAP2ALM_ADJOINT: in = F phases, out = maps times the ring weights w_y;
   SHT_MAP2ALM: in = maps, out = G phases with weights w_y;
   SHT_ALM2MAP_ADJOINT and SHT_ALM2MAP_GRAD: the same with all weights one;
   the DERIV1 directions as ALM2MAP (synthesis) and ALM2MAP_ADJOINT (others). */
int sht_ring_fft(sht_plan *p, int direction, const double *in, double *out,
                 void *hip_stream);

/* Algorithmic work of one Legendre step in the given direction after polar
   skipping (the same in both directions, the analysis being the transpose of
   the synthesis).  With K the kept (m, ring slot, degree) triples (Sect. 3.3),
   J = ntrans, and per triple r = 4 (spin 0) or 10 (spin s > 0: two chains,
   Sect. 4.1) flops of recursion and c = 4 or 16 flops of products per
   transform:
     flops_fp64  = K r + K J c for SHT_FP64 (recursion on the vector units,
                   products on FP64 matrix cores), K r for SHT_FP32_MFMA;
     flops_mfma  = K J c for SHT_FP32_MFMA (FP32 matrix-core products), 0 for
                   SHT_FP64;
     hbm_bytes   = the minimal HBM traffic of a whole transform: a_lm and maps
                   once, the phases written and read once.
   Any output pointer may be NULL.  SHT_EINVAL for an unknown direction. */
int sht_plan_flops(const sht_plan *p, int direction, double *flops_fp64, double *flops_mfma,
                   double *hbm_bytes);

/* Size report of a plan: n_legendre_items = wavefront work items of its
   Legendre synthesis launch (including the padding items of the die-aware
   order), device_bytes = all device memory the plan owns (tables, work lists,
   phase workspace, FFT tables).  Either pointer may be NULL. */
int sht_plan_info(const sht_plan *p, int64_t *n_legendre_items, int64_t *device_bytes);

/* Device buffers currently allocated by the library in this process, and
   their total size (diagnostics: a failed create call must leave both where
   they were).  Either pointer may be NULL. */
int sht_memory_stats(int64_t *live_buffers, int64_t *live_bytes);

/* ---- batches of plans (mixed band limits and grids) ---- */

/* A batch runs several plans (same spin, precision and coefficient storage;
   one direction per call) as one stream-ordered unit (Sect. 3.2's simultaneous
   transforms, with mixed band limits and grids): the Legendre analyses of
   every plan are merged into one persistent launch over a queue of items
   popped by an atomic counter (plans tuned to the vector path run their own
   analysis launches instead); the Legendre syntheses (each plan's die-aware
   item list) and the ring FFTs run per plan, on concurrent streams; on a
   non-null stream the whole sequence is captured once into a HIP graph and
   replayed (captured again when the buffers, the stream or the tuning of a
   plan change).  The plans are borrowed and must outlive the batch; results
   equal the plans' own bit for bit. */
int sht_batch_create(int nplans, sht_plan *const *plans, sht_batch **out);
int sht_batch_execute(sht_batch *b, int direction, const double *const *in,
                      double *const *out, void *hip_stream);
void sht_batch_destroy(sht_batch *b);

/* Legendre step only of every plan of the batch (as sht_legendre per plan):
   in/out hold one phase buffer and one coefficient buffer per plan.  Plain
   launches on hip_stream (no graph); the analysis directions run the batch's
   persistent launch. */
int sht_batch_legendre(sht_batch *b, int direction, const double *const *in,
                       double *const *out, void *hip_stream);

/* Scheduling of a batch:
   queue_order  SHT_QUEUE_COST: analysis items (plan, m, transform group)
                ordered by decreasing cost (degree range x active slot tiles);
                SHT_QUEUE_MPAIRS: items are pairs (m, mmax - m) of one plan,
                whose cost is nearly the same for every pair (Sect. 4.2's
                load balance), ordered by decreasing pair cost;
   concurrent   1: every plan's launch chain (synthesis: Legendre step then
                ring FFTs; analysis: ring FFTs) runs on a stream of its own
                between a fork and a join on the caller's stream, so that small
                plans fill the gaps of large ones; 0: one stream; 2: as 1 for
                the ring FFTs, while the Legendre syntheses of all plans run as
                one persistent launch over one queue of (plan, m, slot tile,
                transform group) items in the queue order (needs every plan on
                the matrix-core kernels with the same synthesis column blocks
                and carry interval, else the plans' own launches run).
   Defaults: SHT_QUEUE_COST, concurrent 1.  Results do not depend on either.
   SHT_EINVAL for other values. */
enum { SHT_QUEUE_COST = 0, SHT_QUEUE_MPAIRS = 1 };
int sht_batch_configure(sht_batch *b, int queue_order, int concurrent);

/* Launch-shape parameters of a plan's Legendre kernels (Sect. 3.2: block sizes
   are machine dependent and picked by measurement).  The matrix-core shapes
   give the same results bit for bit; the vector path adds the same terms in
   another order (results equal to rounding, about 1e-15 relative). */
typedef struct sht_tuning {
    int synth_ncb;      /* synthesis: 16-column blocks per wavefront (1 or 2) */
    int synth_mblock;   /* synthesis: consecutive m values dealt to one
                           accelerator die (1 .. 64) */
    int anal_ncb;       /* analysis: 16-column blocks per work group (1 or 2) */
    int anal_tpw;       /* analysis: slot tiles per wavefront and pass (1 or 2) */
    int valu;           /* 1: products on the vector units instead of the matrix
                           cores (SHT_FP64 only; the default where most
                           matrix-core columns would be empty: spin 0 with one
                           or two transforms, spin > 0 with one) */
    int reserved[11];
} sht_tuning;

/* Current tuning of a plan. */
int sht_plan_get_tuning(const sht_plan *p, sht_tuning *t);
/* Set a tuning (SHT_EUNSUPPORTED for a combination that is not built for the
   plan's spin and precision; the plan keeps its previous tuning then).  Not
   while work of the plan is in flight. */
int sht_plan_set_tuning(sht_plan *p, const sht_tuning *t);

/* Pick the tuning of a plan by timing the candidate combinations on scratch
   data (one Legendre synthesis and analysis each) for about budget_seconds;
   results are cached in the text file named by $SHT_TUNE_CACHE (if set), one
   line per plan shape, so that a later plan of the same shape takes the cached
   choice without timing (budget 0: only the cache is consulted).  Batches that
   hold the plan capture their launches again at their next execution. */
int sht_autotune(sht_plan *p, double budget_seconds);

/* Message of the calling thread's last failed call ("" if none).
   Diagnostics: the environment variable SHT_LOG (read once per process) writes
   one line per event to stderr -- 1: handles created and destroyed, tunings and
   recorded errors; 2: also every call of sht_execute, sht_legendre,
   sht_ring_fft and the batch entry points; 3: also every kernel launch.  Every
   entry point that does work opens a roctx range named after itself, which ROCm
   tracers (rocprofv3 --marker-trace) record beside the kernels. */
const char *sht_last_error(void);
const char *sht_strerror(int status);

#ifdef __cplusplus
}
#endif
#endif /* SHT_H */
