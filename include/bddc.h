/*
 * bddc.h -- C ABI of libbddc.so: adaptive-multilevel BDDC for 2D scalar
 * diffusion on MI355X (gfx950).
 *
 * Method: Sousedik and Mandel, "On Adaptive-Multilevel BDDC".
 *   - Problem statement (Section 2, eq. (problem)): find u in U with
 *     a(u, v) = <f, v> for all v in U, U = continuous P1 or Q1 functions on
 *     the unit square vanishing on its boundary, a(u, v) = sum over elements
 *     of k_e * int grad u . grad v.
 *   - Preconditioner: Algorithm "Multilevel BDDC" (Section 2.1).
 *   - Adaptive coarse dofs: Theorem "local-est" (Section 3), Theorem
 *     "adaptive" (Section 4) and the adaptive setup algorithm (Section 5).
 *   - Krylov method: preconditioned conjugate gradients (Section 5),
 *     stopping test ||r||_2 <= rtol * ||f||_2.
 *
 * Conventions shared by every call
 *   - Every call returns a bddc_status; nothing throws across the ABI.
 *   - Arguments are validated on the host before any device work; a call
 *     that fails validation has no effect.
 *   - Vectors r, z, f, u are DEVICE pointers to FP64 data owned by the
 *     caller, column-major with nrhs columns of length n_free =
 *     (nx-1)*(ny-1) and leading dimension ld >= n_free.  Free node (i, j),
 *     1 <= i <= nx-1, 1 <= j <= ny-1, has index (j-1)*(nx-1) + (i-1).
 *   - f is the dual (load) vector: entry j is <f, phi_j>.
 *   - hip_stream is a hipStream_t (NULL = the null stream).  apply and solve
 *     are enqueued on it; solve synchronises it before returning.
 *   - A handle must not be used by two threads at once.  Calls on different
 *     handles are independent.
 */
#ifndef BDDC_H
#define BDDC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BDDC_OK = 0,
  BDDC_EINVAL = -1,       /* bad argument (size, pointer, value out of range, k <= 0 or not finite) */
  BDDC_ENOMEM = -2,       /* device allocation failed */
  BDDC_ESINGULAR = -3,    /* a local or coarse factorization met a non-positive pivot */
  BDDC_EPARTITION = -4,   /* partition or agglomeration invalid (id out of range, empty substructure) */
  BDDC_ENOCONV = -5,      /* PCG reached maxit; u holds the last iterate */
  BDDC_EDEVICE = -6,      /* a HIP runtime call failed */
  BDDC_EBUSY = -7,        /* the handle has a stepwise solve in progress */
  BDDC_EUNSUPPORTED = -8  /* valid input outside what this build implements (sizes, precision) */
} bddc_status;

/* P1: each element square split along its SW-NE diagonal.  Q1_ELASTIC: the
 * plane-strain elasticity of the paper's numerical section (Section 6: Lame
 * parameters lambda = 1, mu = 2, here scaled by coeff per element), Q1 for both
 * displacement components, two dofs per free node: dof 2 f + c is component c
 * (0: x, 1: y) of free node f, so n_free = 2 (nx-1)(ny-1); corners carry both
 * components; the kernel of a floating substructure is its three rigid-body
 * modes.  With ADAPTIVE, every edge of a floating substructure must end at two
 * corner nodes (square partitions do), else bddc_setup returns
 * BDDC_EUNSUPPORTED. */
typedef enum { BDDC_Q1 = 0, BDDC_P1 = 1, BDDC_Q1_ELASTIC = 2 } bddc_element;
/* Coarse dofs (Section 2): CORNERS, the values at corner dofs; CORNERS_EDGES,
 * those and the arithmetic average over each edge of each displacement
 * component (one per edge for scalar problems, two in elasticity; Table 1);
 * ADAPTIVE, corners and the eigenvectors of the pair eigenproblems above tau
 * (Section 5). */
typedef enum { BDDC_CORNERS = 0, BDDC_CORNERS_EDGES = 1, BDDC_ADAPTIVE = 2 } bddc_constraints;
typedef enum { BDDC_FP64 = 0, BDDC_FP32 = 1, BDDC_BF16 = 2 } bddc_precision;

typedef struct bddc_ctx* bddc_handle;   /* opaque, owned by the library */

#define BDDC_MAX_LEVELS 8

/* Size of the fixed device working array of bddc_solve_noalloc (one per
 * device, held until the process ends). */
#define BDDC_NOALLOC_SCRATCH_BYTES (64u << 20)

/* Problem description; pointers are HOST pointers read during the call only, except coeff_device. */
typedef struct {
  int32_t nx, ny;              /* elements per side of the unit square, nx, ny >= 2 */
  int32_t element;             /* bddc_element */
  const double* coeff;         /* nx*ny, k_e > 0 and finite; element e = j*nx + i covers [i/nx,(i+1)/nx] x [j/ny,(j+1)/ny] */
  const int32_t* part;         /* nx*ny, level-1 substructure of each element, in [0, nsub) */
  int32_t nsub;                /* number of level-1 substructures, >= 1; each must own an element */
  int32_t levels;              /* L >= 2 decomposition levels; level L is the directly solved coarse problem */
  const int32_t* const* agglom;/* levels-2 arrays: agglom[l-2][s] = level-l substructure of level-(l-1)
                                  substructure s (l = 2..L-1); may be NULL when levels == 2 */
  int32_t constraints;         /* bddc_constraints; corners are always coarse dofs */
  double tau;                  /* ADAPTIVE threshold: eigenvectors with lambda > tau become coarse dofs */
  int32_t precision;           /* bddc_precision: storage of the reduced-precision preconditioner operators */
  const double* coeff_device;  /* optional DEVICE pointer to the same nx*ny coefficients; when non-NULL it is
                                  used instead of coeff (which may then be NULL) and the positivity check runs
                                  on the device (BDDC_EINVAL after the device work) */
} bddc_problem;

/* Sizes and diagnostics of a set-up preconditioner (per level l = 1..levels-1 at index l-1). */
typedef struct {
  int64_t n_free;                       /* unknowns of the level-1 problem */
  int32_t levels;
  int32_t nsub[BDDC_MAX_LEVELS];        /* substructures of level l */
  int32_t n_dof[BDDC_MAX_LEVELS];       /* dofs of level l (level 1: n_free) */
  int32_t n_interface[BDDC_MAX_LEVELS]; /* interface dofs of level l */
  int32_t n_corners[BDDC_MAX_LEVELS];
  int32_t n_edges[BDDC_MAX_LEVELS];
  int32_t nc[BDDC_MAX_LEVELS];          /* coarse dofs of level l (= dofs of level l+1) */
  int32_t n_adaptive[BDDC_MAX_LEVELS];  /* coarse dofs added by the eigenproblems at level l */
  double omega[BDDC_MAX_LEVELS];        /* max over edges of the largest unselected eigenvalue (ADAPTIVE) */
  double indicator;                     /* product of omega over levels (ADAPTIVE), else 0 */
  double kappa;                         /* Lanczos condition estimate of the last solve (first column) */
  int32_t last_iters;                   /* iterations of the last solve (first column) */
  int64_t device_bytes;                 /* device memory held by the handle */
  int64_t apply_bytes;                  /* algorithmic bytes streamed by one interface preconditioner apply */
  int64_t matvec_bytes;                 /* algorithmic bytes streamed by one interface operator product */
} bddc_info;

/* Validate a problem and report its level-1 topology (n_free, nsub, interface,
 * corner and edge counts) without touching the device.  Only level 1 is filled
 * (levels beyond 1 depend on the coarse dofs chosen at set-up), and
 * device_bytes holds the device memory a set-up of it will need (estimated
 * from the level-1 sizes, with a margin for the deeper levels), for admission
 * control.  Errors: BDDC_EINVAL, BDDC_EPARTITION, BDDC_EUNSUPPORTED. */
bddc_status bddc_plan(const bddc_problem* p, bddc_info* info);

/* Set up the preconditioner (Section 5, adaptive setup algorithm, then the
 * structures of Algorithm "Multilevel BDDC" at every level).  Host inputs are
 * copied; the caller may free them after return.  On success *out owns all
 * device data until bddc_destroy.  On failure *out is NULL and nothing leaks.
 * Errors: BDDC_EINVAL, BDDC_EPARTITION, BDDC_EUNSUPPORTED, BDDC_ESINGULAR,
 * BDDC_ENOMEM, BDDC_EDEVICE. */
bddc_status bddc_setup(const bddc_problem* p, void* hip_stream, bddc_handle* out);

/* z = M^{-1} r for nrhs columns: the full-space multilevel preconditioner of
 * Algorithm "Multilevel BDDC" (interior pre-correction, substructure
 * correction, coarse problem by recursion, averaging, interior
 * post-correction).  r and z are device arrays (may not alias).
 * Errors: BDDC_EINVAL, BDDC_EDEVICE. */
bddc_status bddc_apply(bddc_handle h, const double* r, double* z, int32_t nrhs, int64_t ld,
                       void* hip_stream);

/* Solve A u = f for nrhs columns with PCG preconditioned by M (Section 5).
 * Level 1 is reduced to the interface (Section 5, last remark): PCG starts
 * from the condensed iterate (interior values solve the interior problems,
 * interface values 0), runs on the interface, and the interior values are
 * recovered at the end.  Each column stops when ||r||_2 <= rtol ||f||_2 on
 * the recursively updated residual, or after maxit iterations.
 * iters[nrhs] and relres[nrhs] are HOST arrays written after the stream is
 * synchronised (relres = final ||r|| / ||f||; 0 if f = 0).
 * Errors: BDDC_EINVAL, BDDC_ENOCONV (u holds the last iterate), BDDC_EDEVICE. */
bddc_status bddc_solve(bddc_handle h, const double* f, double* u, int32_t nrhs, int64_t ld,
                       double rtol, int32_t maxit, int32_t* iters, double* relres, void* hip_stream);

/* bddc_solve for callers that cannot allocate device memory (serving loops
 * and harnesses that forbid allocation after set-up): the same PCG, the same
 * kernels and bitwise the same results as bddc_solve, but the per-column PCG
 * state (iterates, residuals, directions, partial sums, scalars, condensed
 * load) is laid out in one fixed device array of BDDC_NOALLOC_SCRATCH_BYTES
 * per device, owned by the library and held until the process ends, instead
 * of the handle's arena; the iterations are launched directly (no graph is
 * captured or replayed).  The call allocates and frees no device memory.
 * Columns are solved in blocks of up to eight, as many as the array holds;
 * the array is cleared at the start of every call.  Every call on one device
 * shares that array: calls that overlap in time on one device (from several
 * threads or streams) race and must not be made.  The current device must be
 * the one the handle was set up on.  Arguments and outputs as bddc_solve.
 * Errors: BDDC_EINVAL, BDDC_EUNSUPPORTED (one column's state does not fit
 * the array), BDDC_ENOCONV, BDDC_EDEVICE. */
bddc_status bddc_solve_noalloc(bddc_handle h, const double* f, double* u, int32_t nrhs, int64_t ld,
                               double rtol, int32_t maxit, int32_t* iters, double* relres, void* hip_stream);

/* Stepwise bddc_solve, for serving loops that interleave several solves and
 * admit new ones between chunks of iterations (Section 5's PCG, the same
 * launches and bitwise the same results as bddc_solve).
 *   bddc_solve_begin:   enqueue the condensation, r_0 and z_0 of nrhs (1..8)
 *                       columns of f (device, leading dimension ld) on
 *                       hip_stream, which the handle keeps until the end.
 *   bddc_solve_advance: enqueue at least `iterations` more iterations (whole
 *                       chunks; none past maxit or convergence do work), then
 *                       an asynchronous copy of the convergence flags.
 *   bddc_solve_poll:    without waiting: *state = 1 when the iterations
 *                       enqueued so far finished every column (or reached
 *                       maxit), 0 when more are needed, -1 while the last
 *                       advance is still running.
 *   bddc_solve_end:     recover the interior into u (device, ld), write the
 *                       host arrays iters[nrhs] and relres[nrhs], synchronise;
 *                       BDDC_ENOCONV if a column did not converge.
 * f must stay valid until bddc_solve_end.  While a stepwise solve is in
 * progress, bddc_solve, bddc_solve_noalloc, bddc_apply, bddc_autotune and a
 * second bddc_solve_begin on the handle return BDDC_EBUSY.
 * Errors: BDDC_EINVAL (arguments, or no stepwise solve in progress),
 * BDDC_EBUSY, BDDC_ENOCONV, BDDC_EDEVICE. */
bddc_status bddc_solve_begin(bddc_handle h, const double* f, int32_t nrhs, int64_t ld, double rtol, int32_t maxit,
                             void* hip_stream);
bddc_status bddc_solve_advance(bddc_handle h, int32_t iterations);
bddc_status bddc_solve_poll(bddc_handle h, int32_t* state);
bddc_status bddc_solve_end(bddc_handle h, double* u, int64_t ld, int32_t* iters, double* relres);

/* Sizes and diagnostics.  Errors: BDDC_EINVAL. */
bddc_status bddc_query(bddc_handle h, bddc_info* info);

/* Launch configuration of bddc_solve (no effect on the method: Algorithm
 * "Multilevel BDDC" inside PCG, Section 5).  deep_path: how levels >= 2 and
 * the coarsest solve run -- BDDC_DEEP_COOP (one cooperative launch, one
 * workgroup per level-2 substructure), BDDC_DEEP_WIDE (row blocks of dense
 * level-2 operators over many workgroups), BDDC_DEEP_FUSED (all deep levels in
 * one workgroup), BDDC_DEEP_LEVELS (one launch per phase and level); only the
 * paths planned at set-up are available (bit p of `available`, read-only).
 * finalize: 1 sums the PCG partials once per producing launch in a one-block
 * launch, 2 lets the producing launch's last block to finish sum them, 3
 * sums them in 256 slots within the producing launch and lets every consuming
 * block add the slots (2 and 3: one right-hand side; several: as 1), 0 lets
 * every consuming block sum them; interfaces wider than 256 dofs take 1 only.  graph: 1 replays a captured
 * chunk of PCG launches, 0 launches directly.  check: PCG iterations between
 * host convergence checks (4, 8 or 16).  solve_ms: the median time of one
 * bddc_solve with this configuration when bddc_autotune chose it, else 0.
 * finalize, graph and check leave the iterates bitwise unchanged; the deep
 * paths agree to rounding. */
typedef enum { BDDC_DEEP_COOP = 0, BDDC_DEEP_WIDE = 1, BDDC_DEEP_FUSED = 2, BDDC_DEEP_LEVELS = 3 } bddc_deep_path;
typedef struct {
  int32_t deep_path;
  int32_t finalize;
  int32_t graph;
  int32_t check;
  int32_t available;
  double solve_ms;
} bddc_tuning;

/* Current launch configuration (bddc_get_tuning) or a new one
 * (bddc_set_tuning; `available` and `solve_ms` are ignored).
 * Errors: BDDC_EINVAL (NULL, a deep path not available, check not 4/8/16,
 * finalize not 0..3 or not available, graph not 0/1). */
bddc_status bddc_get_tuning(bddc_handle h, bddc_tuning* t);
bddc_status bddc_set_tuning(bddc_handle h, const bddc_tuning* t);

/* Autotuner: times bddc_solve of the nrhs device columns f (leading dimension
 * ld; u receives the solutions, as for bddc_solve) under the available launch
 * configurations -- one knob at a time (deep path, finalize, check, graph),
 * keeping the fastest value of each -- with the median of `reps` (>= 1) solves
 * per candidate, installs the fastest configuration on the handle and returns
 * it in *t (may be NULL).  The choice is also remembered for the problem's
 * shape (mesh, partition sizes, levels, constraints, precision, coarse sizes):
 * a later bddc_setup of the same shape starts from it.  Synchronises the
 * stream.  Errors: BDDC_EINVAL, BDDC_ENOCONV, BDDC_EDEVICE. */
bddc_status bddc_autotune(bddc_handle h, const double* f, double* u, int32_t nrhs, int64_t ld, double rtol,
                          int32_t reps, bddc_tuning* t, void* hip_stream);

/* Eigenvalues of the pair eigenproblem of Theorem "local-est" for edge
 * `edge` (0-based, pairs (s,t), s < t, in increasing order) of level `level`
 * (1-based) of an ADAPTIVE set-up.  Writes up to cap eigenvalues in
 * decreasing order to the host array lam, their count to *n_lam, the number
 * selected (lambda > tau) to *n_sel, the pair to pair[0..1], and the number
 * of edge dofs to *n_edge_dofs.  Any output pointer may be NULL.
 * Errors: BDDC_EINVAL (not adaptive, level or edge out of range). */
bddc_status bddc_edge_eigs(bddc_handle h, int32_t level, int32_t edge, double* lam, int32_t cap,
                           int32_t* n_lam, int32_t* n_sel, int32_t* pair, int32_t* n_edge_dofs);

/* Coarse dofs installed on an edge: the level's dof ids of the edge (host
 * array dofs, cap_dofs entries) and the constraint weights, one column per
 * coarse dof, column-major n_edge_dofs x n_cols in the host array q with
 * leading dimension n_edge_dofs (cap_q entries).  Columns of an ADAPTIVE
 * set-up are orthonormal.  Errors: BDDC_EINVAL (sizes too small, out of range). */
bddc_status bddc_edge_constraints(bddc_handle h, int32_t level, int32_t edge, int32_t* dofs,
                                  int32_t cap_dofs, double* q, int32_t cap_q,
                                  int32_t* n_edge_dofs, int32_t* n_cols);

/* Corner dofs of level `level` (1-based): the dofs shared by three or more
 * substructures, plus the corners promoted where a floating substructure or
 * pair would otherwise have none (Section 2 coarse dofs; Section 5 asks for
 * "sufficient" corners).  Written in ascending order to the host array
 * corners (cap entries; may be NULL to query the count); *n_corners receives
 * the count.  Level-l dofs for l >= 2 are the level-(l-1) coarse dofs,
 * numbered corners first (ascending corner dof), then edge by edge in
 * bddc_edge_eigs order, each edge's columns in the order of
 * bddc_edge_constraints.  Errors: BDDC_EINVAL (level out of range, cap too
 * small). */
bddc_status bddc_corners(bddc_handle h, int32_t level, int32_t* corners, int32_t cap, int32_t* n_corners);

/* Kernel timing for measurement tools.  bddc_timing_start(name, every) arms
 * HIP events on one in `every` (>= 1) later launches of the named kernel, on
 * any handle: the events are stamped by the dispatch itself, on the stream the
 * kernel runs on, so they bracket the kernel's execution only; sampling keeps
 * the events' own cost out of a timed loop.  NULL or "" disarms.  Names:
 * "schur_local" (PCG operator product), "apply_restrict" (PCG update and
 * level-1 restriction), "deep" (levels >= 2 and the coarsest solve in one
 * launch), "apply_average" (level-1 interface average), "apply_pre_l2",
 * "apply_restrict_l2", "apply_prolong_l2", "apply_post_l2" ("_l3" ...; deep
 * levels when they run one launch per phase), "wide_pre", "wide_restrict",
 * "wide_coarse", "wide_post" (the row-block deep level), "partial_chol",
 * "partial_chol_l2".
 * bddc_timing_stop synchronises those events and returns the summed kernel
 * time in ms, the number of timed launches, and the summed algorithmic bytes
 * and flops of those launches (each operator and vector entry the kernel must
 * touch, counted once), then disarms.  Host arrays may be NULL.
 * Errors: BDDC_EINVAL (every < 1), BDDC_EDEVICE. */
bddc_status bddc_timing_start(const char* kernel, int32_t every);
bddc_status bddc_timing_stop(double* total_ms, int64_t* launches, double* bytes, double* flops);

/* Message of the last failed call on this thread ("" if none; never NULL;
 * valid until the next failing call on the same thread). */
const char* bddc_last_error(void);

/* Static description of a status code (never NULL). */
const char* bddc_status_string(bddc_status s);

/* Release every resource of the handle (NULL-safe).  Synchronises the device. */
void bddc_destroy(bddc_handle h);

#ifdef __cplusplus
}
#endif

#endif /* BDDC_H */
