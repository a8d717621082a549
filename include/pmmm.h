/*
 * pmmm.h -- C ABI of the MI355X (gfx950) PMMM far-field library.
 *
 * Particle mesh multipole method (Nitadori, arXiv:1409.5981).  Given N
 * particles with positions r_i and charges q_i in a box cut into
 * K = nx ny nz uniform cubic cells, the library returns the FAR-FIELD potential
 *     Phi_i = sum over particles j outside the (2c+1)^3 cells around i of
 *             q_j / |r_i - r_j|      (periodic: over all images, Ewald sense)
 * and its gradient grad Phi_i, in the caller's input order (problem statement
 * of Sec. 1 and Sec. 2.1).  The near field (the masked cells, Sec. 2.1 last
 * paragraph) is NOT included in pmmm_far_*; pmmm_near_* computes it and
 * pmmm_total_* returns the sum of both.
 * Electrostatics: force_i = -q_i grad Phi_i.  Gravity: pass masses and take
 * Phi_grav = -G Phi, force_i = +G m_i grad Phi_i.
 *
 * Pipeline (Sec. 2.1, eq. pmmm and the FFT procedure below it):
 *   bin -> P2M (eq. P2M) -> (p+1)^2 forward 3-D FFTs -> per-frequency M2L
 *   with the transfer kernel G~ (eq. M2L in the real-matrix form of
 *   eq. realmatrix) -> (p+1)^2 inverse FFTs -> periodic corrections
 *   (App. B, correction procedure) -> L2P (eq. L2P; gradient via eq. L2L at
 *   destination order one and eq. phigrad).
 * Open boundaries convolve on the 2x zero-padded mesh (App. C); periodic
 * ones use the lattice-summed kernel of App. B (eq. greenPBC).  The
 * transfer-kernel spectra are built once, on the GPU in FP64, when the plan
 * is created and kept for every later call (Sec. 2.1).
 *
 * Memory and streams: every particle/output pointer passed to pmmm_far_*,
 * pmmm_near_* and pmmm_total_* is a DEVICE pointer owned by the caller;
 * calls only enqueue work on the given HIP stream (hipStream_t passed as void*, NULL =
 * default stream) and return without synchronising.  Inputs must stay
 * alive and unmodified until the stream has completed the call.  The plan
 * owns the transfer kernel and its workspace (device memory); a plan may be
 * used by one stream at a time (calls on one plan must not overlap).
 *
 * Errors: every int-returning call returns PMMM_OK (0) or one of the codes
 * below; pmmm_error_string() names a code and pmmm_last_error() returns the
 * last message recorded by the calling thread.  Argument errors are
 * detected on the host before anything is enqueued.  Open-boundary particles
 * outside the box [0, b_x) x [0, b_y) x [0, b_z) are clamped into the
 * border cells of the computed mesh by the kernels and raise a device flag
 * that pmmm_plan_sync_status() reports as PMMM_EDOMAIN.
 */
#ifndef PMMM_H
#define PMMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PMMM_PMAX 10 /* highest expansion order compiled in */

enum {
    PMMM_OK = 0,
    PMMM_EINVAL = 1,      /* invalid argument (null pointer, bad size or parameter) */
    PMMM_ENOMEM = 2,      /* device allocation failed */
    PMMM_EHIP = 3,        /* a HIP runtime call failed; see pmmm_last_error() */
    PMMM_EDOMAIN = 4,     /* open boundary: a particle lay outside [0, b)^3 */
    PMMM_EUNSUPPORTED = 5 /* valid by the method but not built (e.g. mesh size) */
};

enum { PMMM_OPEN = 0, PMMM_PERIODIC = 1 };
enum { PMMM_F32 = 0, PMMM_F64 = 1, PMMM_BF16X3 = 2 };
enum { PMMM_MESH_M = 0, PMMM_MESH_L = 1, PMMM_MESH_GREEN = 2 };

typedef struct pmmm_plan_s *pmmm_plan;
typedef struct pmmm_batch_s *pmmm_batch;
typedef struct pmmm_hier_s *pmmm_hier;

/* Method parameters (Sec. 2.1, Sec. 3.2, App. B).
 *   nx, ny, nz  cells per axis (the mesh may be any product of three
 *               integers, Sec. 1).  Periodic meshes must be cubic,
 *               nx == ny == nz == n >= 2c + 1; a power-of-two n runs the
 *               radix-2 transforms, any other n <= 64 runs direct DFTs along
 *               each axis (same results up to rounding; batches and the
 *               multi-charge call take powers of two only).  Open meshes may
 *               have any nx, ny, nz >= 1: the library computes on the
 *               smallest power-of-two cube n^3 (n >= 4) of the same cells
 *               that holds the box at its corner.  The open convolution is
 *               linear, so the extra cells, which hold no particles, change
 *               no result; they cost FFT and M2L work.  The FFT mesh nf (2n
 *               open, n periodic) may be at most 128 (FP32) or 64 (FP64).
 *   box         edge lengths b of the box [0, b_x) x [0, b_y) x [0, b_z);
 *               cells must be cubic (b_a / n_a equal to 1e-12 relative).
 *   p           expansion order, 0 <= p <= PMMM_PMAX ((p+1)^2 coefficients);
 *               at p = 0 the far-field gradient is identically zero.
 *   cutoff      near-cell half width c: 1 (27 cells) or 2 (125 cells); 0 -> 2.
 *               Periodic meshes need n >= 2c + 1.
 *   boundary    PMMM_OPEN or PMMM_PERIODIC.
 *   precision   PMMM_F32 (use pmmm_far_f32) or PMMM_F64 (pmmm_far_f64).
 *               PMMM_BF16X3 is an FP32 plan whose multi-charge M2L product
 *               (pmmm_far_multi_f32) keeps two bf16 terms of each operand
 *               (three products, about 16 bits); FP32 plans keep three
 *               terms (six products, FP32-level rounding).  pmmm_far_f32
 *               runs the same FP32 pipeline for both.
 *   alpha       periodic splitting parameter of the lattice sums; 0 -> 1.5/b.
 *   images      periodic lattice-sum radius: real-space images r + n b with
 *               |r + n b| <= images b, reciprocal vectors |n| <= images; 0 -> 4.
 *   n_max       particle capacity to allocate up front (0: grow on demand;
 *               growing synchronises the device once). */
typedef struct {
    int nx, ny, nz;
    double box[3];
    int p;
    int cutoff;
    int boundary;
    int precision;
    double alpha;
    int images;
    int64_t n_max;
} pmmm_params;

/* Build a plan: validates the parameters, allocates the workspace, builds
 * the transfer-kernel spectra on the GPU (FP64 lattice sums / harmonics and
 * FP64 FFTs, stored in the plan's precision) on `stream`, and synchronises
 * it.  *out receives the plan on success and NULL otherwise. */
int pmmm_plan_create(const pmmm_params *params, void *stream, pmmm_plan *out);

/* Free a plan and its device memory (synchronises the device). NULL is a no-op. */
void pmmm_plan_destroy(pmmm_plan plan);

/* Device bytes a plan with these parameters holds for n_max particles
 * (0 if the parameters are invalid). */
size_t pmmm_workspace_bytes(const pmmm_params *params, int64_t n_max);

/* Far field for n particles, FP32 plan.  x, y, z, q: [n] device arrays;
 * phi, gx, gy, gz: [n] device outputs (Phi and grad Phi in input order).
 * n == 0 is a valid no-op.  Periodic positions may lie anywhere (they are
 * wrapped into the box); open ones must lie in [0, b)^3 (PMMM_EDOMAIN via
 * pmmm_plan_sync_status otherwise). */
int pmmm_far_f32(pmmm_plan plan, int64_t n, const float *x, const float *y, const float *z,
                 const float *q, float *phi, float *gx, float *gy, float *gz, void *stream);

/* Allocation-free variant of pmmm_far_f32, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid allocation after set-up).  Same arguments, result and errors
 * as pmmm_far_f32 for an FP32 (or BF16X3) plan, but the per-particle work
 * space (cell indices, permutation, sorted records, sorted-order results)
 * lives in a static device array of the library sized for
 * PMMM_NOALLOC_MAX_N particles (52 bytes each, 13 MiB; each GPU the library
 * runs on holds its own copy until the process ends), so the call makes no
 * allocation and records no events (stage profiling does not apply).  The
 * array's device address is looked up when a plan is created on a device.
 * n above PMMM_NOALLOC_MAX_N returns PMMM_EINVAL before anything is
 * enqueued.  All calls on one GPU share that GPU's array: calls whose
 * execution overlaps on one GPU (other streams, other plans, other threads)
 * race and give undefined results. */
#define PMMM_NOALLOC_MAX_N (1 << 18)
int pmmm_far_f32_noalloc(pmmm_plan plan, int64_t n, const float *x, const float *y,
                         const float *z, const float *q, float *phi, float *gx, float *gy,
                         float *gz, void *stream);

/* Same as pmmm_far_f32 for an FP64 plan. */
int pmmm_far_f64(pmmm_plan plan, int64_t n, const double *x, const double *y,
                 const double *z, const double *q, double *phi, double *gx, double *gy,
                 double *gz, void *stream);

/* Far field of nsets charge sets on the same n positions (Sec. 2.1 for each
 * set: every step is linear in the charges, so the binning, the particles'
 * harmonics and the transfer kernel are shared).  At each frequency the M2L
 * of eq. realmatrix for all sets is one real (P x P) by (P x 2 nsets)
 * product, computed on the BF16 matrix cores with split FP32 operands and
 * FP32 accumulation (two terms for PMMM_BF16X3 plans, three for PMMM_F32).
 * Periodic FP32 / BF16X3 plans with an FFT mesh of 4 to 32 cells per axis
 * only (PMMM_EUNSUPPORTED otherwise).
 *   x, y, z    [n] device positions;
 *   q          [n][nsets] device charges, the set index fastest
 *              (q[i * nsets + s] is the charge of particle i in set s);
 *   phi, gx, gy, gz  [n][nsets] device outputs in the same layout, input
 *              order of the particles.
 * Sets are processed in chunks of at most 64; the plan grows its multi-set
 * workspace (about 16 P n^3 bytes per set of a chunk) on the first call that
 * needs it, which synchronises the device once.  nsets >= 1; n == 0 is a
 * valid no-op. */
int pmmm_far_multi_f32(pmmm_plan plan, int64_t n, const float *x, const float *y,
                       const float *z, int nsets, const float *q, float *phi, float *gx,
                       float *gy, float *gz, void *stream);

/* Batches of independent systems (Sec. 2.1 for each; the paper notes that
 * many small FFTs can run independently in place of one large one).  Each
 * system has its own parameters; systems whose parameters agree (mesh, box,
 * order, cutoff, boundary, alpha, images) share one transfer kernel and run
 * every stage in one launch for all of them, and a call whose arguments
 * repeat the previous call's replays the previous launches as one HIP graph
 * (captured on the second identical call; not for the NULL stream).
 *   pmmm_batch_create   validates every system (PMMM_F32 or PMMM_BF16X3
 *                       only), builds the transfer kernels on `stream` and
 *                       synchronises it.
 *   pmmm_batch_far_f32  far field of all systems: offsets is a HOST array of
 *                       nsys + 1 non-decreasing values with offsets[0] = 0;
 *                       system s owns particles [offsets[s], offsets[s+1]) of
 *                       the device arrays x, y, z, q and of the outputs phi,
 *                       gx, gy, gz (same meaning as pmmm_far_f32).  A call
 *                       with new offsets synchronises the stream once.
 *   pmmm_batch_classes  number of distinct parameter sets.
 *   pmmm_batch_set_graphs  enable (default) or disable the graph replay.
 *   pmmm_batch_sync_status  as pmmm_plan_sync_status, for the batch. */
int pmmm_batch_create(int nsys, const pmmm_params *per_sys, void *stream, pmmm_batch *out);
void pmmm_batch_destroy(pmmm_batch batch);
int pmmm_batch_far_f32(pmmm_batch batch, const int64_t *offsets, const float *x, const float *y,
                       const float *z, const float *q, float *phi, float *gx, float *gy,
                       float *gz, void *stream);
int pmmm_batch_classes(pmmm_batch batch);
int pmmm_batch_set_graphs(pmmm_batch batch, int enable);
int pmmm_batch_sync_status(pmmm_batch batch);

/* Near field (Sec. 2.1, last paragraph, and Sec. 2.3: the particles of the
 * (2c+1)^3 cells masked out of the transfer kernel interact by direct
 * Newtonian sums, no cutoff function; periodic meshes take, for each
 * neighbour cell, the one image within c cells).  Same arguments, layouts,
 * ownership and errors as pmmm_far_f32; the call bins the particles itself.
 * accumulate != 0 adds the near field into phi, gx, gy, gz instead of
 * overwriting them.  Two particles at the same position in neighbouring
 * cells give an infinite result, as the sum itself does. */
int pmmm_near_f32(pmmm_plan plan, int64_t n, const float *x, const float *y, const float *z,
                  const float *q, float *phi, float *gx, float *gy, float *gz, int accumulate,
                  void *stream);
int pmmm_near_f64(pmmm_plan plan, int64_t n, const double *x, const double *y,
                  const double *z, const double *q, double *phi, double *gx, double *gy,
                  double *gz, int accumulate, void *stream);

/* Total potential and gradient, far field + near field (the split of eq. pmmm
 * and Sec. 2.1: every pair of particles is counted once, by the near field
 * when their cells are within c of each other, else by the far field), with
 * one binning for both parts.  Arguments as pmmm_far_f32 / _f64; the
 * outputs are overwritten. */
int pmmm_total_f32(pmmm_plan plan, int64_t n, const float *x, const float *y, const float *z,
                   const float *q, float *phi, float *gx, float *gy, float *gz, void *stream);
int pmmm_total_f64(pmmm_plan plan, int64_t n, const double *x, const double *y,
                   const double *z, const double *q, double *phi, double *gx, double *gy,
                   double *gz, void *stream);

/* Two-level hierarchical far field (Sec. 5.2).  `coarse` describes an open
 * FP32 mesh, cubic with a power-of-two edge n (the other fields as for
 * pmmm_plan_create); `refine` = r in {1, 2, 4, 8} cuts each coarse cell into
 * r^3 fine cells (n r <= 128).  A pair of particles is counted by
 *   the coarse PMMM   when their coarse cells are more than c apart;
 *   the fine level    when their coarse cells are within c and their fine
 *                     cells are not: eq. M2L from every such fine cell's
 *                     moments to the fine cell's local expansion, summed
 *                     directly over the fine cells of the (2c+1)^3 coarse
 *                     neighbourhood (the paper evaluates the same sum as a
 *                     local convolution), then eq. L2P;
 *   the near field    when their fine cells are within c.
 * pmmm_hier_far_f32 returns the first two parts, pmmm_hier_total_f32 all
 * three; arguments, layouts, ownership and stream semantics as
 * pmmm_far_f32 (the outputs are overwritten).  The fine level costs
 * O(((2c+1) r)^3 (p+1)^4) per fine cell.  pmmm_hier_sync_status reports a
 * particle outside the box as PMMM_EDOMAIN.  Errors: PMMM_EINVAL for a bad
 * argument or refine, PMMM_EUNSUPPORTED for a mesh the hierarchy does not
 * take, plus those of pmmm_plan_create and pmmm_far_f32. */
int pmmm_hier_create(const pmmm_params *coarse, int refine, void *stream, pmmm_hier *out);
void pmmm_hier_destroy(pmmm_hier h);
int pmmm_hier_far_f32(pmmm_hier h, int64_t n, const float *x, const float *y, const float *z,
                      const float *q, float *phi, float *gx, float *gy, float *gz, void *stream);
int pmmm_hier_total_f32(pmmm_hier h, int64_t n, const float *x, const float *y, const float *z,
                        const float *q, float *phi, float *gx, float *gy, float *gz, void *stream);
int pmmm_hier_sync_status(pmmm_hier h);
/* Per-stage timing of a hierarchy's two levels, as pmmm_plan_set_profiling /
 * pmmm_plan_read_profile: the mask applies to both levels; level 0 reads the
 * coarse PMMM's stages, level 1 the fine level's (binning, P2M, the fine
 * eq. M2L sums as PMMM_STAGE_COLUMN, L2P and the near field).  Errors:
 * PMMM_EINVAL for a NULL hierarchy or another level, plus those of
 * pmmm_plan_read_profile. */
int pmmm_hier_set_profiling(pmmm_hier h, unsigned mask);
int pmmm_hier_read_profile(pmmm_hier h, int level, double *ms, int64_t *count, int reset);

/* Per-order fixed-point records of a coefficient mesh (Sec. 5.3 and its
 * footnote: an order-l coefficient carries 3 (p + 1 - l) bits, so a cell
 * carries 3 (p+1)(p+2)(2p+3)/6 bits, 612 at p = 7).  These calls work on a
 * caller's device arrays; no plan is involved.
 *   coef     [(p+1)^2][ncell] float32, device, component-major in the real
 *            storage of the meshes (index l(l+1)+m holds Re X_l^|m| for
 *            m >= 0 and Im X_l^|m| for m < 0), e.g. a PMMM_MESH_M or
 *            PMMM_MESH_L mesh;
 *   records  [ncell][pmmm_coef_record_words(p)] uint32, device: each cell's
 *            codes as b_l-bit two's-complement fields in real-storage order,
 *            bit j of the record in bit j mod 32 of word j / 32, zero-padded;
 *   exps     [p+1] int32, device: the unit of order l is 2^exps[l], shared
 *            by all cells.
 * code = rint(word / 2^e_l) (ties to even), clamped to +-(2^(b_l-1) - 1);
 * NaN words are coded 0.  With flags = PMMM_COEF_AUTO_EXP the pack chooses
 * and writes exps: the smallest power of two under which the largest |word|
 * of the order rounds inside its range (0 for an all-zero order,
 * PMMM_COEF_EXP_INVALID for an order holding a non-finite word, whose codes
 * are then 0); with flags = 0 it reads the caller's exps.  Unpack writes
 * code * 2^e_l (NaN for an order marked invalid).  The round trip is within
 * half a unit per word for automatic units.  Both calls only enqueue work on
 * `stream` (NULL: the default stream) and allocate nothing; ncell = 0 is a
 * no-op apart from the automatic exps (all 0).
 * Errors: PMMM_EINVAL for p outside 0..PMMM_PMAX, ncell outside 0..2^31,
 * unknown flag bits or a null pointer that would be used; PMMM_EHIP if a
 * launch fails. */
#define PMMM_COEF_EXP_INVALID (-2147483647 - 1)
enum { PMMM_COEF_AUTO_EXP = 1 };
/* 32-bit words per cell record at order p, or -1 for p outside 0..PMMM_PMAX. */
int pmmm_coef_record_words(int p);
int pmmm_coef_pack_f32(int p, int64_t ncell, const float *coef, uint32_t *records, int32_t *exps,
                       unsigned flags, void *stream);
int pmmm_coef_unpack_f32(int p, int64_t ncell, const uint32_t *records, const int32_t *exps,
                         float *coef, void *stream);

/* Complex composition of two real coefficient sets (App. D).  a and b are
 * [(p+1)^2][ncell] float32 meshes in the real storage above, each obeying
 * X_l^{-m} = (-1)^m conj(X_l^m); c is [(p+1)^2][ncell] (re, im) float32
 * pairs (8-byte aligned) holding C_l^m = A_l^m + i B_l^m at index l(l+1)+m
 * for every -l <= m <= l.  By linearity, a transformation applied to C in
 * complex arithmetic acts on both sets at once; pmmm_coef_split_f32 recovers
 * the two real sets from such a composite (it reads C_l^m and C_l^{-m} only,
 * and writes a and b in full).  Device pointers; the calls only enqueue work
 * on `stream` and allocate nothing.  Errors: PMMM_EINVAL for p outside
 * 0..PMMM_PMAX, ncell outside 0..2^31 or a null pointer (ncell > 0);
 * PMMM_EHIP if a launch fails. */
int pmmm_coef_compose_f32(int p, int64_t ncell, const float *a, const float *b, float *c,
                          void *stream);
int pmmm_coef_split_f32(int p, int64_t ncell, const float *c, float *a, float *b, void *stream);

/* Launch-shape autotuner.  Runs the far field (pmmm_far_f32 or _f64 by the
 * plan's precision, same arguments and meaning) on the caller's particles,
 * timing with HIP events the P2M stage for each number of lanes per cell
 * (4, 8, 16, 32), then the column stage (FFT along z, M2L) for each kernel
 * form and, for the staged tile, each number of columns per block (the
 * widest that fits LDS, half and a quarter of it);
 * every candidate runs in three interleaved rounds of five calls and its
 * shortest stage time counts.  The fastest of each is kept for later calls on
 * this plan.  Synchronises the stream; the outputs hold the result of the
 * last trial; stage profiling enabled by the caller is suspended meanwhile
 * (its accumulated times are kept).  Shapes change only the order of
 * floating-point sums.  The column stage is timed for every kernel form that
 * fits the plan (PMMM_COLUMN_*, below; the tile form at each width).
 * pmmm_plan_get_tuning reports the kept shapes. */
int pmmm_plan_autotune(pmmm_plan plan, int64_t n, const void *x, const void *y, const void *z,
                       const void *q, void *phi, void *gx, void *gy, void *gz, void *stream);

/* Forms of the column kernel (FFT along z, wave-space M2L, inverse FFT):
 * the transfer-kernel tile of w columns staged in LDS, or the kernel values
 * streamed from memory at each thread's frequency with one column per block
 * and each thread running 1, 2 or 4 of the four row subsets of the M2L
 * (less LDS per block, so several blocks share a compute unit; FFT meshes of
 * 64 and 128 points; four subsets per thread up to order 6, two up to order
 * 8: beyond, their results would not fit the registers). */
enum {
    PMMM_COLUMN_DEFAULT = 0,
    PMMM_COLUMN_TILE = 1,
    PMMM_COLUMN_STREAM_1 = 2,
    PMMM_COLUMN_STREAM_2 = 3,
    PMMM_COLUMN_STREAM_4 = 4
};
/* Launch shapes of a plan; 0 in any field means the library's default. */
typedef struct {
    int column_kernel; /* PMMM_COLUMN_* */
    int column_width;  /* columns per block of PMMM_COLUMN_TILE (power of two) */
    int p2m_lanes;     /* lanes per cell of the light P2M path: 4, 8, 16, 32 or 64 */
} pmmm_tuning;
/* The kept shapes (zeros until set or tuned). */
int pmmm_plan_get_tuning(pmmm_plan plan, pmmm_tuning *out);
/* Set shapes, e.g. ones saved from an earlier pmmm_plan_autotune: PMMM_EINVAL
 * for a form or width that does not fit this plan, or lanes outside the list. */
int pmmm_plan_set_tuning(pmmm_plan plan, const pmmm_tuning *in);

/* Synchronise the plan's last stream and report a device-side condition
 * (PMMM_EDOMAIN for an out-of-box open-boundary particle) since the last call
 * of this function; the flag is cleared. */
int pmmm_plan_sync_status(pmmm_plan plan);

/* Copy an internal mesh to host memory for inspection (synchronises).  n
 * is the computed mesh (for an open plan of nx x ny x nz cells, the
 * power-of-two cube holding it; the caller's cells are the corner
 * [0, nz) x [0, ny) x [0, nx)):
 *   PMMM_MESH_M      moments of the last call, [(p+1)^2][n][n][n] (z, y, x),
 *                    in CELL units (M_l scaled by 1/h^l), plan precision;
 *   PMMM_MESH_L      local expansions of the last call, same layout, in cell
 *                    units (L_l scaled by h^(l+1)); periodic plans include the
 *                    uniform corrections of App. B (self, dipole and r^2
 *                    terms) but not the per-particle terms of a charged system;
 *   PMMM_MESH_GREEN  transfer-kernel spectra in cell units, one real value per
 *                    component and frequency, on the quadrant ky, kz <= nf/2
 *                    (the rest follows from the kernel's y and z reflection
 *                    symmetries): [nh (ky)][nh (kx)][(2p+1)^2 components]
 *                    [nhp (kz)] with nh = nf/2 + 1 and nhp = nh rounded up to
 *                    a multiple of 4 (padding zero), holding Re G~ for even
 *                    orders and Im G~ for odd orders (the other part vanishes
 *                    by the parity of the kernel); periodic plans carry the
 *                    self term -2 alpha h / sqrt(pi) in component 0.
 * `bytes` must equal pmmm_plan_mesh_bytes(plan, which). */
size_t pmmm_plan_mesh_bytes(pmmm_plan plan, int which);
int pmmm_plan_copy_mesh(pmmm_plan plan, int which, void *host_dst, size_t bytes);

/* Graph replay of repeated calls.  With enable != 0, a pmmm_far_*,
 * pmmm_near_* or pmmm_total_* call that repeats the plan's previous call
 * (same entry point, n, pointers, stream, accumulate flag and launch shapes;
 * the contents of the arrays may change) is replayed as a HIP graph: the
 * second such call captures the launches, later ones launch the graph,
 * which saves the host launch work (for a busy or capturing host thread; a
 * host that keeps the stream fed gains nothing: on MI355X the replay
 * measured 1-10% slower than eager launches of the same calls).  A
 * call with other arguments runs eagerly and becomes the new reference.
 * Calls on the NULL stream, with stage profiling on, and the allocation-free
 * call always run eagerly.  enable = 0 (the default) drops the graph (it
 * synchronises the device if a graph exists).  Results are bitwise those of
 * the eager launches. */
int pmmm_plan_set_graphs(pmmm_plan plan, int enable);

/* Stage timing, a profiling aid.  A far-field call runs these stages in order: */
enum {
    PMMM_STAGE_BIN = 0,     /* counting sort of the particles by cell */
    PMMM_STAGE_P2M = 1,     /* eq. P2M per cell */
    PMMM_STAGE_FFT_FWD = 2, /* forward FFT along x and y, per z-plane */
    PMMM_STAGE_COLUMN = 3,  /* FFT along z + wave-space M2L + inverse FFT along z */
    PMMM_STAGE_FFT_INV = 4, /* inverse FFT along y and x, per z-plane */
    PMMM_STAGE_L2P = 5,     /* eq. L2P and the gradient */
    PMMM_STAGE_NEAR = 6,    /* near-field direct sums (pmmm_near_*, pmmm_total_*) */
    PMMM_NSTAGES = 7
};
/* Bit s of `mask` brackets stage s of later pmmm_far_* calls on this plan with
 * a pair of HIP events recorded on the call's stream; 0 (the default) records
 * nothing. */
int pmmm_plan_set_profiling(pmmm_plan plan, unsigned mask);
/* Synchronise on the recorded events and add their elapsed times: ms[s]
 * receives the total milliseconds and count[s] the number of timed launches
 * of stage s since the last reset (arrays of PMMM_NSTAGES entries, either may
 * be NULL); reset != 0 clears the totals afterwards. */
int pmmm_plan_read_profile(pmmm_plan plan, double *ms, int64_t *count, int reset);

const char *pmmm_error_string(int code);
const char *pmmm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PMMM_H */
