/*
 * spect.h - C ABI of the MI355X (gfx950) SPECT projector library.
 *
 * The library computes the parallel-hole SPECT system matrix of the paper
 * (Section 2.1.1, Eq. 1)
 *
 *     H = sum_n v_n (x) ( T_fov P_x T_cdr T_att T_trans T_rot )
 *
 * its transpose H^T (forward projection FP and back projection BP, same
 * section), the subset normalisation H_m^T 1 ("compute_normalization_factor",
 * Section 2.2) and one OSEM subiteration: the preconditioned gradient ascent
 * step of Eq. 5 with the Poisson log-likelihood gradient and the OSEM
 * preconditioner of Table 1.
 *
 * Discretisation (the paper names the operations but not their sampling):
 *   T_rot   bilinear interpolation in each axial slice about the grid centre
 *           c = (N-1)/2; rotated sample (i', j') sits at
 *           X = c + cos(t)(i'-c) - sin(t)(j'-c), Y = c + sin(t)(i'-c) + cos(t)(j'-c);
 *           zero outside the grid.  cos/sin are evaluated in double precision
 *           and magnitudes below 1e-15 are set to 0.
 *   T_trans identity (rotation axis on the grid centre).
 *   T_att   exp(-tau), tau(i') = dx (mu(i')/2 + sum over i'' > i' of mu(i''))
 *           along the rotated depth axis i'; the detector lies beyond i' = N-1.
 *   T_cdr   at depth i': Gaussian of sigma = psf_a d + psf_b (cm), with
 *           d = max(0, R_n - (i'-c) dx), sampled at integer pixel offsets,
 *           truncated at K = ceil(psf_nsigma sigma/dx - 1e-9), normalised to unit
 *           sum, applied along the detector bin axis and the axial axis with
 *           zero padding.
 *   P_x     plain sum over i'.   T_fov  all ones.
 *
 * Layouts (all device arrays are float32, C order, last index fastest):
 *   object       f[i][j][k]  shape (N, N, Nz): i = x, j = y, k = z (axial)
 *   projections  p[n][r][k]  shape (A, N, Nz): n = angle, r = detector bin
 * z is the fastest axis because the rotation acts in the x-y plane: every
 * bilinear corner is then a contiguous run of axial voxels.
 *
 * Conventions for every call:
 *   - Device pointers are caller-owned, must be 4-byte aligned and must not
 *     alias one another unless stated; 16-byte alignment with Nz % 4 == 0
 *     enables vector loads.  The library never frees caller memory.
 *   - Host-side validation runs before any launch; on error nothing is
 *     launched and the call returns a negative status with a message for
 *     spect_last_error().
 *   - Calls are asynchronous on the given stream (a hipStream_t; NULL is the
 *     null stream).  Results are valid once the stream reaches them.
 *   - angle_idx is a host array of angle indices in [0, n_angles); NULL means
 *     all angles in order (n_idx is then ignored).  An index may repeat: a
 *     projection call writes that row (with the same values) once more, a
 *     back projection or sensitivity adds its term once per occurrence.
 *   - The workspace is device memory of at least spect_workspace_size() bytes
 *     for the same op and angle count, 256-byte aligned; it holds nothing
 *     between calls.  Two calls in flight at once need separate workspaces.
 */
#ifndef SPECT_H
#define SPECT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define SPECT_OK 0
#define SPECT_EINVAL (-1)      /* invalid argument (nothing launched) */
#define SPECT_ENOMEM (-2)      /* device allocation failed */
#define SPECT_EHIP (-3)        /* HIP runtime or launch error */
#define SPECT_EUNSUPPORTED (-4) /* valid but outside this build's limits */

/* Workspace queries. */
#define SPECT_OP_FWD 0
#define SPECT_OP_BACK 1
#define SPECT_OP_SENS 2
#define SPECT_OP_OSEM 3
#define SPECT_OP_RECON 4
#define SPECT_OP_BSREM_STEP 5
#define SPECT_OP_BSREM 6
#define SPECT_OP_STEP 7        /* osem_list_step, n_idx = list length */
#define SPECT_OP_STEP_VJP 8    /* osem_list_step_vjp, n_idx = list length */

/* with_mu value of spect_workspace_size for the attenuation-table calls. */
#define SPECT_ATT_TABLE 2

/* Limits of this build. */
#define SPECT_MAX_N 256        /* transverse size N */
#define SPECT_MAX_K 32         /* collimator blur radius in pixels */

typedef struct spect_plan spect_plan;
typedef struct spect_batch spect_batch;

/* Acquisition geometry (Section 2.1.1: projection space V of 2D images, one
 * per angle; object space U of voxelised activity). */
typedef struct {
    int32_t n;                /* transverse grid size N (object N x N x nz, N bins) */
    int32_t nz;               /* axial size Nz (object slices = detector rows) */
    int32_t n_angles;         /* A */
    int32_t flags;            /* reserved, must be 0 */
    double voxel_cm;          /* isotropic voxel and detector pixel size dx > 0 */
    const double *angles_deg; /* host [n_angles]; NULL = n * 360 / A */
    const double *radius_cm;  /* host [n_angles] detector distance R_n >= 0;
                                 NULL = N dx / 2 (detector touching the grid) */
    double psf_a;             /* sigma(d) = psf_a d + psf_b in cm; both >= 0; */
    double psf_b;             /*   psf_a = psf_b = 0 disables T_cdr */
    double psf_nsigma;        /* truncation in sigmas; <= 0 means 4 */
} spect_geometry;

/* Validate the geometry and precompute per-angle trigonometry and per-depth
 * blur kernels (Eq. 1) on the current HIP device.  *out receives a plan that
 * owns a small device table; the plan is immutable and may be used from
 * several streams at once.  The angle and radius arrays are copied.
 * Errors: SPECT_EINVAL (NULL pointers, sizes < 1, flags != 0, non-finite or
 * out-of-range values), SPECT_EUNSUPPORTED (N > SPECT_MAX_N, blur radius >
 * SPECT_MAX_K, an object of 2^29 voxels (2 GiB) or more, a projection set
 * of 2^31 elements or more, Nz >= 2^22), SPECT_ENOMEM, SPECT_EHIP. */
int spect_plan_create(const spect_geometry *geom, spect_plan **out);

/* Free a plan (NULL is accepted).  The caller must make sure no work that
 * uses the plan is still queued. */
int spect_plan_destroy(spect_plan *plan);

/* Workspace bytes needed by op (SPECT_OP_*) over n_idx angles; for
 * SPECT_OP_OSEM and SPECT_OP_RECON n_idx is the number of subsets M.  with_mu:
 * 0 no attenuation, 1 an attenuation map will be passed, SPECT_ATT_TABLE the
 * table calls (spect_fwd_table, spect_back_table with SPECT_OP_FWD /
 * SPECT_OP_BACK; spect_sensitivity_table with SPECT_OP_SENS). */
int spect_workspace_size(const spect_plan *plan, int op, int32_t n_idx, int with_mu,
                         size_t *bytes);

/* Forward projection (FP, Section 2.1.1; Eq. 1): for each listed angle n,
 * proj[n] = P_x T_cdr T_att T_rot f.  f: device (N, N, Nz); mu: device
 * (N, N, Nz) attenuation map in cm^-1, or NULL for no attenuation; proj:
 * device (A, N, Nz), only the listed rows are written.  f and proj must not
 * overlap. */
int spect_fwd(const spect_plan *plan, const float *f, const float *mu, float *proj,
              const int32_t *angle_idx, int32_t n_idx, void *ws, size_t ws_bytes,
              void *stream);

/* Allocation-free forward projection, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid hipMalloc): the same computation as spect_fwd, bitwise, with
 * the scratch taken from a fixed device array of the library
 * (SPECT_STATIC_SCRATCH_BYTES on every device the library runs on, held until
 * the process ends) instead of a caller workspace.  The call allocates
 * nothing.  It returns SPECT_EINVAL, launching nothing, when the listed
 * angles need more scratch than that (spect_workspace_size with SPECT_OP_FWD
 * gives the need; 128^3 with 120 angles and the 0.48 cm blur fits).  Every
 * call on one device uses the same array: calls that overlap in time on one
 * device (several streams, or several host threads) race and must be
 * serialised by the caller, e.g. by issuing them on one stream.  The array
 * needs no clearing between calls (every scratch element a call reads is
 * written earlier in the same call). */
#define SPECT_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
int spect_fwd_static(const spect_plan *plan, const float *f, const float *mu, float *proj,
                     const int32_t *angle_idx, int32_t n_idx, void *stream);

/* Back projection (BP, Section 2.1.1): f_out = sum over listed n of
 * H_n^T proj[n] (accumulate == 0), or f_out += that sum (accumulate != 0).
 * proj: device (A, N, Nz), only listed rows are read; f_out: device
 * (N, N, Nz). */
int spect_back(const spect_plan *plan, const float *proj, const float *mu, float *f_out,
               const int32_t *angle_idx, int32_t n_idx, int accumulate, void *ws,
               size_t ws_bytes, void *stream);

/* Subset normalisation H_S^T 1 (Section 2.2 "compute_normalization_factor";
 * the OSEM denominator of Table 1) for the listed angles S; sens: device
 * (N, N, Nz), overwritten. */
int spect_sensitivity(const spect_plan *plan, const float *mu, float *sens,
                      const int32_t *angle_idx, int32_t n_idx, void *ws, size_t ws_bytes,
                      void *stream);

/* Batched OSEM: many reconstructions of different geometries at once (studies
 * over many patients, noise realisations and algorithms, Section 4; the OSEM
 * of Section 2.1.3, Eq. 5 with the Table 1 preconditioner, as in
 * osem_reconstruct).
 *
 * A batch holds R member geometries (plans, which must outlive it) and a
 * common subset count M.  osem_batch_reconstruct runs, for every member, the
 * computation of osem_reconstruct with the same subsets; subiteration m of all
 * members is one batched launch per stage (forward projection with the ratio,
 * rotated-frame adjoint, gather with the multiplicative update) over a
 * work-list of (member, angle, axial slab, depth chunk) tasks.  Each member's
 * state lives in its own region of one workspace (spect_batch_workspace_size
 * bytes, 256-byte aligned, caller-owned; it also holds copies of the images
 * for osem_batch_autotune).  With schedules 0-3 the results equal
 * osem_reconstruct per member bitwise; schedules 4-7 sum each ray's forward
 * depth contributions over all depths at once, which changes only the FP32
 * rounding.
 *
 * Arrays f, mu, g, s_add are host arrays of R device pointers, laid out as in
 * osem_reconstruct; mu must be given for every member if the batch was created
 * with_mu != 0 (attenuation-factor tables are then kept per member and
 * subset) and must be NULL (or hold NULLs) otherwise; s_add may be NULL.
 *
 * Schedules 0..7 (spect_batch_set_schedule, osem_batch_autotune): bit 0 set =
 * one launch per stage for each group of members with equal block size and
 * blur class, clear = one launch for all members; bit 1 set = persistent
 * grids (workgroups loop over tasks), clear = one task per workgroup; bit 2
 * set = every task walks all depths of its rays, clear = depths split into
 * the chunks a single reconstruction would use.
 *
 * By default one iteration (the M subiterations) is captured once as a HIP
 * graph on an internal stream and replayed on `stream` n_iters times;
 * SPECT_BATCH_EAGER launches the kernels directly instead.  A batch is not
 * reentrant: calls on it must not overlap. */
#define SPECT_BATCH_EAGER 1

int spect_batch_create(const spect_plan *const *plans, int32_t n_members, int32_t n_subsets,
                       int with_mu, spect_batch **out);
int spect_batch_destroy(spect_batch *batch);
int spect_batch_workspace_size(const spect_batch *batch, size_t *bytes);
int osem_batch_reconstruct(spect_batch *batch, float *const *f, const float *const *mu,
                           const float *const *g, const float *const *s_add, int32_t n_iters,
                           int32_t flags, void *ws, size_t ws_bytes, void *stream);

/* Autotuner: times one graph-replayed iteration of every schedule on copies
 * of the images (the sensitivities are computed first; f is not changed),
 * keeps the fastest as the batch's schedule and records the times.
 * Synchronises the stream. */
int osem_batch_autotune(spect_batch *batch, float *const *f, const float *const *mu,
                        const float *const *g, const float *const *s_add, void *ws,
                        size_t ws_bytes, void *stream);

/* The current schedule and, in candidate_ms[0..7] (may be NULL), the
 * autotuner's per-iteration times (-1 where not measured). */
int spect_batch_schedule(const spect_batch *batch, int32_t *schedule, double *candidate_ms);
int spect_batch_set_schedule(spect_batch *batch, int32_t schedule);

/* Reconstruction server with continuous batching: OSEM reconstructions of
 * many studies (Section 4) admitted as they arrive and advanced together.
 *
 * A request is a whole reconstruction (the computation of osem_reconstruct):
 * the sensitivity pass of each subset (with an attenuation map it also fills
 * the subset's attenuation-factor table), then n_iters x n_subsets
 * subiterations; each of these is one step.  A scheduler thread owned by the
 * server launches ticks back to back on up to four lanes (streams of default
 * priority that run concurrently); a lane's tick takes the next step of each
 * of the lane's resident requests, whatever its geometry, subset or
 * iteration, and runs them together as one launch per stage (sensitivity
 * pass, forward projection with the ratio, the rotated-frame adjoint, gather
 * with the update; the forward and adjoint stages once per blur-radius
 * class).  The tick's launch tables are copied on a separate upload stream.
 * At every tick boundary requests are admitted in arrival order, to the lane
 * with the least work left, while fewer than n_slots are resident and the
 * pool (pool_bytes of device memory owned by the server) holds a free block
 * of the request's workspace (spect_workspace_size with SPECT_OP_RECON); a
 * request that does not fit waits, and so do the requests behind it.  One
 * exception: a wide request (one step covers at least 2^24 voxel-angles, so
 * it fills the device on its own) waits while another wide request is
 * resident, unless four or more wide requests are queued; narrow requests
 * behind it may start meanwhile.  A request retires, freeing its block, once
 * the tick holding its last step has finished.  Its state lives in its block, laid out as
 * osem_reconstruct's workspace, and its steps use osem_reconstruct's launch
 * arguments: the result equals osem_reconstruct alone, bitwise, whatever
 * shares its ticks.  With an attenuation map the tables of all subsets must
 * fit in 32 GiB (SPECT_EUNSUPPORTED otherwise).
 *
 * The caller owns f (the initial image on submission, the reconstruction
 * once the request is SPECT_REQ_DONE), mu, g, s_add, and keeps them alive
 * and untouched until then.  Ordering: spect_server_submit records an event
 * on `stream` (the caller's HIP stream; NULL = the null stream) and the
 * request's first tick waits for it on the device, so f, mu, g and s_add may
 * still be being written by work the caller queued on that stream before the
 * call.  A request is finished once spect_server_wait returns or its state
 * reads SPECT_REQ_DONE; the caller may then read f on any stream.
 *
 * The calls may come from any host thread (the server serialises them).
 * spect_server_submit fails with SPECT_EINVAL if the request's workspace can
 * never fit in the pool.  spect_server_progress reports the resident and
 * queued counts (the scheduler thread does the work).  spect_server_status:
 * *state = SPECT_REQ_*; a failed request returns its error code and message.
 * spect_server_wait blocks until the request is done or failed.
 * spect_server_forget drops the record of a finished request.
 * spect_server_destroy finishes every resident request; queued ones are
 * dropped. */
#define SPECT_REQ_QUEUED 0
#define SPECT_REQ_RUNNING 1
#define SPECT_REQ_DONE 2
#define SPECT_REQ_FAILED 3

typedef struct spect_server spect_server;
int spect_server_create(int32_t n_slots, size_t pool_bytes, spect_server **out);
int spect_server_destroy(spect_server *server);
int spect_server_submit(spect_server *server, const spect_plan *plan, float *f, const float *mu,
                        const float *g, const float *s_add, int32_t n_iters, int32_t n_subsets,
                        void *stream, int64_t *request_id);
int spect_server_progress(spect_server *server, int32_t *n_running, int32_t *n_queued);
int spect_server_status(spect_server *server, int64_t request_id, int32_t *state);
int spect_server_wait(spect_server *server, int64_t request_id);
int spect_server_forget(spect_server *server, int64_t request_id);
/* Resident and queued counts, the largest number of requests ever resident
 * at once, and the pool bytes in use. */
int spect_server_stats(const spect_server *server, int32_t *n_running, int32_t *n_queued,
                       int32_t *peak_running, size_t *pool_in_use);

/* Attenuation-factor tables (T_att of Eq. 1 evaluated once).  For a fixed
 * attenuation map and angle list the factors exp(-tau) do not change between
 * projections, so repeated projections of the same list (OSEM iterations,
 * unrolled reconstructions) can read them instead of resampling mu.  A table
 * holds, for list position i, axial slab s of 16 slices, rotated depth i' and
 * bin j', the factors of the slab's 16 axial rows:
 *     table[((i * ceil(Nz/16) + s) * N + i') * N + j'][16]   (float32)
 * (rows past Nz hold unused values).  Tables are device memory owned by the
 * caller, 16-byte aligned.
 *
 * spect_table_size: bytes of a table for n_idx angles, n_idx * ceil(Nz/16) *
 * N * N * 64. */
int spect_table_size(const spect_plan *plan, int32_t n_idx, size_t *bytes);

/* spect_sensitivity for the listed angles (mu required) that also writes the
 * attenuation factors of those angles, in list order, to table. */
int spect_sensitivity_table(const spect_plan *plan, const float *mu, float *sens, float *table,
                            const int32_t *angle_idx, int32_t n_idx, void *ws, size_t ws_bytes,
                            void *stream);

/* spect_fwd / spect_back with the attenuation factors read from a table that
 * spect_sensitivity_table wrote for the same angle list in the same order
 * (results equal spect_fwd / spect_back with that mu up to FP32 rounding of
 * the attenuation sums).  Workspace: spect_workspace_size(..., SPECT_ATT_TABLE). */
int spect_fwd_table(const spect_plan *plan, const float *f, const float *table, float *proj,
                    const int32_t *angle_idx, int32_t n_idx, void *ws, size_t ws_bytes,
                    void *stream);
int spect_back_table(const spect_plan *plan, const float *proj, const float *table, float *f_out,
                     const int32_t *angle_idx, int32_t n_idx, int accumulate, void *ws,
                     size_t ws_bytes, void *stream);

/* One OSEM subiteration (Eq. 5 with Table 1: PoissonLogLikelihood gradient
 * H^T(g/(Hf+s)) - H^T 1, OSEM preconditioner f / (H_m^T 1), no prior) on the
 * interleaved subset S_m = { n : n mod n_subsets == m }:
 *     gbar = H_m f + s_m;  q = g / gbar where gbar > 0, else 0;
 *     f <- f * (H_m^T q) / sens_m where sens_m > 0, else f unchanged.
 * f: device (N, N, Nz), updated in place; g: device (A, N, Nz) measured data;
 * s_add: device (A, N, Nz) additive term or NULL (zero); sens_m: device
 * (N, N, Nz) = H_m^T 1 from spect_sensitivity with the same subset; mu as in
 * spect_fwd.  0 <= m < n_subsets <= n_angles. */
int osem_subset_step(const spect_plan *plan, float *f, const float *mu, const float *g,
                     const float *s_add, const float *sens_m, int32_t m, int32_t n_subsets,
                     void *ws, size_t ws_bytes, void *stream);

/* The subiteration of osem_subset_step over an explicit angle list S (1 to
 * 128 distinct angles; angle_idx NULL = all angles), out of place, with the
 * attenuation from mu or from a table that spect_sensitivity_table wrote for
 * the same list in the same order (at most one of mu and table; both NULL:
 * none):
 *     f_out = f * H_S^T(g / (H_S f + s)) / sens   where sens > 0, f elsewhere,
 * the ratio taken as 0 where H_S f + s <= 0 (Eq. 5 with Table 1).  f, f_out,
 * sens: device (N, N, Nz), f_out == f updates in place, otherwise they must
 * not overlap; sens = H_S^T 1.  g, s_add as in osem_subset_step.  Workspace:
 * SPECT_OP_STEP with n_idx = the list length and with_mu 0, 1 or
 * SPECT_ATT_TABLE.  Errors: SPECT_EINVAL (empty list, an angle listed twice,
 * both mu and table), SPECT_EUNSUPPORTED (more than 128 angles). */
int osem_list_step(const spect_plan *plan, const float *f, float *f_out, const float *mu,
                   const float *table, const float *g, const float *s_add, const float *sens,
                   const int32_t *angle_idx, int32_t n_idx, void *ws, size_t ws_bytes, void *stream);

/* Vector-Jacobian product of osem_list_step in f, for differentiating
 * unrolled reconstructions (the paper's projectors inside learned
 * reconstruction, Section 1):
 *     grad_f = (d f_out / d f)^T grad_out
 *            = u + H_S^T( -g / e^2 * H_S(grad_out * f / sens) )   (e > 0 rows),
 *     e = H_S f + s,  u = grad_out * H_S^T(g / e) / sens  (grad_out where sens = 0),
 * with the branches of the ratio and of sens = 0 differentiated as written
 * (no gradient through a row with e <= 0 or a voxel with sens = 0 other than
 * the identity).  g, s_add and sens are data (not differentiated).  The call
 * recomputes e and the back projection from f (nothing is kept between the
 * step and its product), 4 projector passes over the list.  grad_f may equal
 * grad_out; it must not overlap f.  Workspace: SPECT_OP_STEP_VJP (n_idx and
 * with_mu as for SPECT_OP_STEP).  Other arguments and errors as in
 * osem_list_step. */
int osem_list_step_vjp(const spect_plan *plan, const float *f, const float *mu, const float *table,
                       const float *g, const float *s_add, const float *sens,
                       const int32_t *angle_idx, int32_t n_idx, const float *grad_out, float *grad_f,
                       void *ws, size_t ws_bytes, void *stream);

/* A whole OSEM reconstruction f = A(L) (Section 2.1.3, Eq. 4 and Eq. 5 with
 * the Table 1 OSEM preconditioner and Poisson gradient): computes the subset
 * sensitivities H_m^T 1, then runs n_iters iterations, each visiting the
 * interleaved subsets m = 0 .. n_subsets-1 in order with the update of
 * osem_subset_step.  With an attenuation map, the sensitivity pass of each
 * subset stores that subset's attenuation factors exp(-tau) (64 bytes per
 * angle, 16-slice slab, depth and bin) in the workspace and every
 * subiteration reads them back instead of resampling mu; if the tables of all
 * subsets would exceed 32 GiB, each subset keeps only its depth-chunk
 * attenuation offsets and every pass samples mu.  f: device (N, N, Nz), the
 * initial image on entry (the paper leaves it open; 1 everywhere is the usual
 * choice) and the reconstruction on return; g, s_add, mu as in
 * osem_subset_step.  The workspace (SPECT_OP_RECON, n_idx = n_subsets) also
 * holds the M sensitivity volumes and, when Nz is a multiple of 128 and mu is
 * not resampled, a copy of f with columns Nz + 32 floats apart that the
 * forward reads and every update rewrites (a layout only: the result is the
 * same).  n_iters >= 0.
 *
 * Graph replay: the launches depend only on the plan and the arguments, so
 * the plan captures them into a HIP graph on the second call with the same
 * arguments (f, mu, g, s_add, ws and ws_bytes, n_iters, n_subsets) and
 * replays that graph on `stream` in later calls with the same arguments;
 * the arrays' contents are read at run time, so they may change between
 * calls.  Replays give bitwise the result of eager launches.  The first call
 * with new arguments, and every call while kernel timing
 * (spect_profile_enable) is on, launches eagerly.  A plan keeps its 8 most
 * recently used graphs until spect_plan_destroy, and guards them with a
 * lock, so calls from several host threads may share a plan. */
int osem_reconstruct(const spect_plan *plan, float *f, const float *mu, const float *g,
                     const float *s_add, int32_t n_iters, int32_t n_subsets, void *ws,
                     size_t ws_bytes, void *stream);

/* osem_reconstruct from the start image 1 everywhere (the usual choice for
 * Eq. 5's iteration, Section 2.1.3): f is written, never read, so it may hold
 * anything on entry.  The first sensitivity launch also sets f to 1 (no
 * separate fill launch); the result equals osem_reconstruct's from an f of
 * ones bitwise.  Arguments, workspace, errors and graph replay as
 * osem_reconstruct (the two calls keep separate graphs). */
int osem_reconstruct_ones(const spect_plan *plan, float *f, const float *mu, const float *g,
                          const float *s_add, int32_t n_iters, int32_t n_subsets, void *ws,
                          size_t ws_bytes, void *stream);

/* BSREM with the relative difference prior (Section 2.1.3: Eq. 4 with the
 * Table 1 BSREM preconditioner C = f alpha^(n) / (c^(n) H^T 1), prior
 * weight beta^(n) = c^(n) beta, and the Table 1 RelativeDifferencePrior
 * phi(a, b) = (a - b)^2 / (a + b + gamma |a - b|)).
 *
 * Prior V(f) = sum_r sum_{s in N(r)} w_rs phi(f_r, f_s) over the 26 neighbours
 * s of voxel r inside the grid, w_rs = 1 / (distance in voxels) (the paper:
 * "typically inverse Euclidean distance"); its gradient is
 *     dV/df_r = 2 sum_s w_rs (f_r - f_s)(f_r + 3 f_s + gamma |f_r - f_s|)
 *               / (f_r + f_s + gamma |f_r - f_s|)^2,
 * a pair with a zero denominator contributing 0.
 *
 * spect_rdp_gradient: grad = dV/df.  f, grad: device (N, N, Nz), distinct;
 * gamma >= 0. */
int spect_rdp_gradient(const spect_plan *plan, const float *f, float *grad, float gamma,
                       void *stream);

/* One BSREM subiteration on the interleaved subset S_m:
 *     f <- max(0, f + f alpha / (c S) (H_m^T(g / (H_m f + s)) - H_m^T 1 - c beta dV/df))
 * where S = sens_all = H^T 1 over all angles (spect_sensitivity with all
 * angles), sens_m = H_m^T 1, c = |S_m| / A (the subset's share of the data);
 * voxels with S = 0 keep their value; the clip at 0 keeps the image
 * non-negative (the paper does not state it; BSREM is defined on the
 * non-negative orthant).  alpha > 0, beta >= 0, gamma >= 0.  Workspace:
 * SPECT_OP_BSREM_STEP with n_idx = n_subsets.  Other arguments as in
 * osem_subset_step. */
int bsrem_subset_step(const spect_plan *plan, float *f, const float *mu, const float *g,
                      const float *s_add, const float *sens_m, const float *sens_all, int32_t m,
                      int32_t n_subsets, float alpha, float beta, float gamma, void *ws,
                      size_t ws_bytes, void *stream);

/* A whole BSREM-RDP reconstruction: the subset sensitivities (and, with an
 * attenuation map, the attenuation-factor tables, as in osem_reconstruct),
 * S = their sum, then n_iters iterations of bsrem_subset_step over
 * m = 0 .. n_subsets-1 with alpha = relaxation[k] in iteration k (relaxation:
 * host array of n_iters values > 0, or NULL for 1 / (1 + k), a reading: the
 * paper leaves the sequence open).  The paper's SPECT examples use beta = 0.3,
 * gamma = 2.  Workspace: SPECT_OP_BSREM with n_idx = n_subsets.  Graph
 * replay as in osem_reconstruct; beta, gamma and the relaxation values are
 * part of the arguments that select a graph. */
int bsrem_reconstruct(const spect_plan *plan, float *f, const float *mu, const float *g,
                      const float *s_add, int32_t n_iters, int32_t n_subsets, float beta,
                      float gamma, const float *relaxation, void *ws, size_t ws_bytes,
                      void *stream);

/* Kernel timing, a tracing aid.  While enabled (process-wide), every kernel
 * the library launches is bracketed by two HIP events recorded on the
 * launch's own stream.  spect_profile_query waits for the recorded launches of
 * the named kernel ("tau_prepass", "fwd_main", "fwd_reduce", "back_rot",
 * "back_gather", "fill_zero", "rdp_grad", "vol_sum", "fwd_batch", "reduce_batch",
 * "back_batch", "gather_batch", "sens_line", "pad_columns") and returns their count and summed duration in
 * milliseconds; spect_profile_reset waits for and frees all records.
 * Errors: SPECT_EINVAL (NULL argument, unknown name), SPECT_EHIP. */
int spect_profile_enable(int enable);
int spect_profile_reset(void);
int spect_profile_query(const char *kernel, int32_t *launches, double *total_ms);

/* Message for the last error on the calling thread ("" if none). */
const char *spect_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SPECT_H */
