/*
 * mm.h -- C ABI of the MI355X coupled Maxwell-LLG time stepper.
 *
 * Method: Yao, Jambunathan, Zeng & Nonaka, "A Massively Parallel Time-Domain
 * Coupled Electrodynamics-Micromagnetics Solver": the second-order coupled
 * scheme of Sec. 3.2.2 on the Yee grid of Sec. 3.1 -- per step an H-M
 * half step (Step 1), the E update (Step 2), and a second H-M half step
 * (Step 3).
 *
 * Conventions (all entry points):
 *   - SI units throughout.
 *   - A "cell map" is a host array of nx*ny*nz doubles, x fastest
 *     (element (i,j,k) at i + nx*(j + ny*k)).
 *   - Field arrays use their staggered extents, x fastest.  Per axis a the
 *     node count is n_a+1 on a PEC axis and n_a on a periodic axis:
 *       Ex: nx   x NY x NZ      Hx: NX x ny x nz
 *       Ey: NX x ny   x NZ      Hy: nx x NY x nz
 *       Ez: NX x NY x nz        Hz: nx x ny x NZ     (NX = x node count, ...)
 *     M on the faces of family f (normal to axis f) has H_f's extent; all
 *     three components are stored per face (Sec. 3.1).
 *   - Every entry point returns an mm_status; 0 is success.  Argument errors
 *     are returned immediately.  Conditions found on the device (a sub-step
 *     that hit max_iter, a non-finite residual) are recorded in a sticky
 *     word and returned by the next synchronising call (mm_sync, mm_probe,
 *     mm_get_field, mm_stats); the time stepping itself continues.
 *   - A context is not thread-safe.  Separate contexts are independent.
 *   - All device work of a context is enqueued on the stream given in
 *     mm_options (NULL = the null stream).
 */
#ifndef MM_H
#define MM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MM_OK = 0,
  MM_EINVAL = -1,      /* bad argument: shape, dt above the CFL limit, Ms < 0, tol <= 0 ... */
  MM_ENOMEM = -2,      /* device or host allocation failed */
  MM_EDEVICE = -3,     /* a HIP call failed */
  MM_ENOCONV = -4,     /* some H-M sub-step stopped at max_iter without reaching tol */
  MM_ENONFINITE = -5,  /* a sub-step residual was NaN or infinite */
  MM_ESTATE = -6       /* call not allowed in the context's current state */
} mm_status;

typedef enum { MM_BC_PEC = 0, MM_BC_PERIODIC = 1 } mm_bc;         /* Sec. 3.2.3 */
typedef enum { MM_FP64 = 0, MM_FP32 = 1 } mm_precision;

/* Uniform Cartesian mesh (Sec. 3.1). */
typedef struct {
  int32_t nx, ny, nz;     /* cells per axis, each >= 1 */
  int32_t bc[3];          /* mm_bc per axis */
  double dx, dy, dz;      /* cell sizes (m) */
} mm_grid;

/* Material properties at cell centres (Sec. 3.1): host cell maps, copied by
 * mm_init.  NULL selects the default in brackets.
 *   eps_r  relative permittivity [1]          sigma  conductivity, S/m [0]
 *   mu_r   relative permeability [1]          Ms     saturation magnetisation, A/m [0]
 *   alpha  Gilbert damping [0]                gamma  gyromagnetic ratio, rad/(s T) [-1.759e11]
 *   m0_dir 3 consecutive cell maps (x, y, z components) giving the direction
 *          of the initial magnetisation; M0 = Ms * m0_dir at cell centres
 *          [+z].  Faces take the mean of their two cells, renormalised to the
 *          face Ms (Sec. 3.1).
 * Edges take the mean of their 4 cells for eps and sigma; faces the mean of
 * their 2 cells for Ms and mu (a PEC wall face uses its single cell); alpha
 * and gamma on a face average the face's magnetic cells only.  A face is
 * magnetic when its Ms is > 0 (Sec. 2, eq:Faraday2 / eq:Faraday3). */
typedef struct {
  const double *eps_r, *sigma, *mu_r, *Ms, *alpha, *gamma;
  const double *m0_dir;
} mm_materials;

/* Uniform static bias H0 (A/m); it enters H_eff only (Sec. 2). */
typedef struct { double H0[3]; } mm_bias;

/* Soft current source J_src (Sec. 3.2, Step 2): J = profile * g(t) with
 * g(t) = exp(-(t-t0)^2 / (2 Tp^2)) * cos(2 pi f0 t)  (pulse of Sec. 5.2.1),
 * evaluated at t^{n+1/2}.  `profile` is a host array on component `comp`'s
 * edge extent (A/m^2); entries on PEC walls are ignored. */
typedef struct {
  int32_t comp;           /* 0: Jx, 1: Jy, 2: Jz */
  const double *profile;
  double f0, Tp, t0;
} mm_source;

/* Hard source (Sec. 3.2: a hard source is imposed on its field right after
 * that field's update).  After every update of component `field` (0-2: Ex,
 * Ey, Ez after Step 2, value at t^{n+1}; 3-5: Hx, Hy, Hz after the Faraday
 * half step of Step 1, at t^{n+1/2}, and of Step 3, at t^{n+1}, before the
 * H-M iteration reads it), the entries inside the bounding box of the
 * nonzero interior entries of `profile` are set to profile * g(t), g the
 * pulse of mm_source.  `profile` is a host array on the component's
 * staggered extent (V/m or A/m); entries pinned by a PEC wall (tangential E,
 * normal H) stay zero; zeros inside the box are held at zero. */
typedef struct {
  int32_t field;
  const double *profile;
  double f0, Tp, t0;
} mm_hard_source;

/* Surface current on a PEC wall (Sec. 5.2.1: the excitation is the surface
 * current density J_s on the wall, imposed through the jump of tangential H
 * there).  J_s (A/m) runs along `comp` on the wall normal to `axis` at its
 * low (side 0) or high (side 1) end.  The boundary condition n x H = J_s,
 * n the unit normal into the domain, gives the tangential H = J_s x n; it is
 * held, as a hard source, on the tangential-H faces half a cell inside the
 * wall (the nearest H samples on the Yee grid).  `profile`: host array on
 * component `comp`'s edge extent; only its entries on the wall plane are
 * read. */
typedef struct {
  int32_t axis, side, comp;
  const double *profile;
  double f0, Tp, t0;
} mm_surface_current;

#define MM_MAX_HARD 8

/* Open boundary (Sec. 3.2.3): a split-field perfectly matched layer.
 * cells[2a], cells[2a+1]: thickness in cells of the layer at the low / high
 * end of axis a (a PEC axis; 0: none; the wall behind it stays PEC).  Each
 * E and H component is split into the parts driven by the two terms of its
 * curl; in the layer each part takes the macroscopic update and is damped
 * by exp(-kappa dt/2) (E) or exp(-kappa dt/4) (each H half step) before and
 * after it, kappa = kappa_max (depth / thickness)^order along the part's
 * axis, kappa_max = -(order + 1) c ln(R0) / (2 thickness).  kappa is a rate
 * shared by E and H, so the layer is matched in any non-conducting,
 * non-magnetic material.  Magnetic faces inside a layer and the adjoint
 * with a layer are not supported (MM_EINVAL). */
typedef struct {
  int32_t cells[6];
  double R0;              /* 0 < R0 < 1 */
  double order;           /* >= 1 */
} mm_pml;

/* Options.  dev_alloc/dev_free, when both are set, supply all device memory
 * of the context (e.g. a caching allocator); otherwise hipMalloc/hipFree. */
typedef struct {
  int32_t prec;           /* mm_precision.  MM_FP32: E, H and the cell maps are stored
                             and updated in FP32; M, the LLG solve, the residual and
                             the probe accumulators stay FP64 */
  double tol;             /* sub-step stopping tolerance on max |dM|/Ms (Sec. 3.2.2), > 0 */
  int32_t max_iter;       /* iteration cap per sub-step, >= 1 */
  int32_t fixed_iter;     /* > 0: exactly this many iterations per sub-step (no test) */
  void *hip_stream;       /* hipStream_t or NULL */
  void *(*dev_alloc)(size_t bytes, void *ctx);
  void (*dev_free)(void *ptr, void *ctx);
  void *alloc_ctx;
  int32_t scheme;         /* 0 or 2: the second-order iterative H-M sub-step
                             (Sec. 3.2.2); 1: the first-order scheme of Sec. 3.2.1
                             (one explicit Landau-Lifshitz step of M per half step,
                             then eq:H_update; tol, max_iter and fixed_iter unused) */
  const mm_pml *pml;      /* NULL: no open boundary */
  int32_t fused;          /* H-M sub-step form: 0 automatic (fused for at least 2^18
                             evolving magnetic faces), 1 fused whenever allowed, -1
                             never.  Fused: iterations 1-3 of a sub-step in one
                             launch, pipelined along z with the iterates on chip
                             (same results, bit for bit); allowed with the
                             second-order scheme, no open boundary, no hard H
                             source or surface current, under 2^24 magnetic faces */
} mm_options;

typedef struct mm_ctx mm_ctx;

/* Create a context: validates the arguments (dt must not exceed the vacuum
 * CFL limit 1/(c sqrt(1/dx^2+1/dy^2+1/dz^2))), copies every host input,
 * builds the magnetic-face list and the edge/face material data, zeroes E
 * and H and sets M to its initial value.  Host inputs may be freed on
 * return.  src may be NULL.  Returns MM_EINVAL (with *out = NULL) on a bad
 * argument. */
mm_status mm_init(mm_ctx **out, const mm_grid *g, double dt, const mm_materials *mat,
                  const mm_bias *bias, const mm_source *src, const mm_options *opt);

/* Advance n >= 0 full time steps (Step 1, Step 2, Step 3 of Sec. 3.2.2,
 * then probe sampling at level n+1).  Asynchronous on the context's stream. */
mm_status mm_step(mm_ctx *c, int64_t n);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): mm_step
 * without any allocation.  The sub-step control (final-count words, the
 * completion barrier, the residual partials) lives in a fixed 4 MiB device
 * array that the library holds on each device until the process ends,
 * instead of in the context; the results are those of mm_step, bit for
 * bit.  Everything else the steps write must already exist: the iteration
 * log and the probe series storage are made (and grown) by mm_step, so a
 * caller runs mm_step first for a step count at least as large.  Errors,
 * before any work is enqueued: MM_ESTATE when probes were added after the
 * last mm_step or adjoint checkpoints are enabled; MM_EINVAL when the steps
 * would run past that storage or the control needs more than 4 MiB
 * (2 x (max_iter + 2) x blocks x 8 bytes plus 256; max_iter 100 fits);
 * MM_EDEVICE when the array's address could not be resolved at mm_init.
 * Every call on one device shares that device's array: calls that overlap
 * in time on one device (other streams, other threads) race and must not
 * be issued.  Asynchronous on the context's stream, as mm_step. */
mm_status mm_step_noalloc(mm_ctx *c, int64_t n);

/* Probes.  kind 0: sample field `field` (see below) at staggered index
 * (i,j,k) after every step.  kind 1: Poynting flux through the node plane
 * x = i, P = dy dz sum_{j,k} [Ey Hz - Ez Hy] with Hz, Hy averaged from the
 * two cells beside the plane; i must be an interior node.  Field ids:
 * 0-2 Ex,Ey,Ez; 3-5 Hx,Hy,Hz; 6+3f+c component c of M on the faces of
 * family f; 15-17 normal B on x/y/z faces (mu0 (H + M_n) on magnetic faces,
 * mu H elsewhere, Sec. 2).  Must be added before the first step. */
typedef struct {
  int32_t kind, field, i, j, k;
} mm_probe_desc;

mm_status mm_add_probe(mm_ctx *c, const mm_probe_desc *d, int32_t *id);

/* Add a hard source (see mm_hard_source).  Before the first step only
 * (MM_ESTATE after).  MM_EINVAL: field outside 0-5, a null profile, no
 * nonzero interior entry, an H source whose box holds an evolving magnetic
 * face, a box reaching into an open-boundary layer (an index whose position
 * along a layer axis, the node or the cell centre, lies inside the layer),
 * more than MM_MAX_HARD sources (surface currents included), or the adjoint
 * enabled (it does not cover hard sources).  An H source moves the tiles its
 * box touches out of the fused Faraday pass. */
mm_status mm_add_hard_source(mm_ctx *c, const mm_hard_source *s);

/* Add a surface current (see mm_surface_current); conditions as for
 * mm_add_hard_source, plus MM_EINVAL for a periodic `axis`, comp == axis or
 * side outside {0, 1}. */
mm_status mm_add_surface_current(mm_ctx *c, const mm_surface_current *s);

/* Copy up to `cap` recorded values of probe `id` (one FP64 per step, oldest
 * first) to host `out` (may be NULL to query); *n_written gets the number
 * of recorded steps.  *sum (may be NULL) gets sum_n dt * value_n, the
 * time-integrated value accumulated on the device in FP64 in step order.
 * Synchronises the stream. */
mm_status mm_probe(mm_ctx *c, int32_t id, double *out, size_t cap, size_t *n_written,
                   double *sum);

/* Copy field `field` (ids as for probes, 0-17) to the host array `dst` of
 * doubles on its staggered extent (converted from FP32 in FP32 mode).
 * Synchronises the stream. */
mm_status mm_get_field(mm_ctx *c, int32_t field, double *dst);

/* Overwrite E or H component `field` (0-5) from the host array `src` of
 * doubles on its staggered extent; tangential E and normal H on PEC walls
 * are forced to zero.  Allowed at any step boundary. */
mm_status mm_set_field(mm_ctx *c, int32_t field, const double *src);

/* Device-side access to E or H component `field` (0-5), in the storage
 * precision (8-byte doubles, or 4-byte floats in MM_FP32; mm_info out[6]):
 * `dst` / `src` is device memory on the context's device holding the
 * component's staggered extent densely, x fastest (the host layout of
 * mm_get_field).  Both are enqueued on the context's stream and return
 * without waiting; the caller orders its own use of the buffer against that
 * stream.  mm_set_field_device forces tangential E and normal H on PEC walls
 * to zero, as mm_set_field does; allowed at any step boundary. */
mm_status mm_get_field_device(mm_ctx *c, int32_t field, void *dst);
mm_status mm_set_field_device(mm_ctx *c, int32_t field, const void *src);

/* Iteration counts of the sub-steps done so far (two per step, in order)
 * into `iters` (up to cap; may be NULL); *n gets the total count.
 * Synchronises the stream and returns the sticky device condition. */
mm_status mm_stats(mm_ctx *c, int32_t *iters, size_t cap, size_t *n);

/* Wait for the stream; returns the sticky device condition (MM_OK,
 * MM_ENOCONV or MM_ENONFINITE) and clears it. */
mm_status mm_sync(mm_ctx *c);

/* Static description of the context: out[0..7] = number of evolving
 * magnetic faces, magnetic faces on PEC walls, soft-source edges, padded x
 * pitch, padded y rows, padded z planes, storage bytes per field element,
 * device bytes held by the context. */
mm_status mm_info(const mm_ctx *c, int64_t out[8]);

/* Device layout: out[0..7] = bulk tiles (64 x 4 cells x out[5] planes),
 * tiles near evolving magnetic faces (they take each Faraday half step on
 * its own, in sub-step order), far tiles (within one mm_step call they take
 * the two half steps that use the same curl E, Step 3 of one step and Step
 * 1 of the next, in one fused pass), cells in near tiles, cells in far
 * tiles, planes per tile, the number of distinct (eps_r, sigma) pairs when
 * the E update reads byte material ids instead of the two cell maps (at
 * most 256; 0: dense maps), tiles holding open-boundary layer entries
 * (updated by the layer kernels in every half step; "bulk tiles" above
 * count the others).  The far tiles' lag is invisible at the interface:
 * probes read the level they sample, and every call ends with all tiles at
 * level n. */
mm_status mm_layout(const mm_ctx *c, int64_t out[8]);

/* Adjoint (an addition to the paper's method).  mm_adjoint_enable, called
 * before the first step, makes mm_step save the state (E, H, M) every
 * `checkpoint_every` steps (device memory held by the context).  With
 * 0 < inner_every < checkpoint_every the adjoint is two-level: each
 * segment is recomputed once to save the state every inner_every steps,
 * and per-step storage is held for inner_every steps instead of
 * checkpoint_every (one more forward recompute, far less memory);
 * inner_every = 0 is single-level.  Requires the second-order scheme.
 * mm_adjoint then returns, in host arrays of nx*ny*nz doubles (cell maps,
 * x fastest), the gradient of L = sum_{n=1}^{N} dt P^n -- the
 * time-integrated value of flux probe `probe_id` over the N steps taken --
 * with respect to the eps_r and Ms cell maps.  It is the exact reverse of
 * the computation (same iteration counts; the sub-step iterates are
 * replayed), through the 4-cell edge mean of eps_r and, for Ms, the face
 * mean Ms_f (renormalisation target, alpha/Ms, initial M).  Which faces
 * are magnetic is held fixed: cells with Ms = 0 get 0.  It recomputes each
 * segment from its checkpoint and leaves the context's state, step count
 * and probes as they were.  Requirements: mu_r = 1 everywhere (MM_EINVAL
 * from mm_adjoint_enable otherwise), a flux probe, at most 16 iterations
 * per sub-step (MM_ESTATE otherwise), no hard source or surface current
 * (MM_EINVAL from either side).  Synchronises the stream. */
mm_status mm_adjoint_enable(mm_ctx *c, int32_t checkpoint_every, int32_t inner_every);
mm_status mm_adjoint(mm_ctx *c, int32_t probe_id, double *grad_eps_r, double *grad_Ms);

/* Kernel timing.  mm_profile(c, 1) makes every later mm_step bracket each
 * kernel launch with a pair of HIP events on the context's stream (class
 * 0 e_update, 1 h_bulk (one half step: every tile, or the near tiles),
 * 2 hm_pre or hm_fused, 3 hm_step or hm_more, 4 hm_finish, 5 probes,
 * 6 hm_commit, 7 h_far (the fused two half steps of the far tiles)),
 * mm_profile(c, 0) stops
 * recording.  mm_profile_read synchronises, writes the summed elapsed
 * milliseconds and the launch counts of each class to ms[0..7] /
 * counts[0..7] and discards the records. */
mm_status mm_profile(mm_ctx *c, int32_t enable);
mm_status mm_profile_read(mm_ctx *c, double ms[8], int64_t counts[8]);

/* Text of the last error recorded on this context ("" if none).  The
 * pointer stays valid until the next call on the context. */
const char *mm_last_error(const mm_ctx *c);

/* Free the context and all its device memory (after waiting for the stream). */
void mm_destroy(mm_ctx *c);

#ifdef __cplusplus
}
#endif

#endif /* MM_H */
