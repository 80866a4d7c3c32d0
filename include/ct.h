/*
 * ct.h -- C ABI of the MI355X (gfx950) library for the ABBA method:
 * BA-GMRES and AB-GMRES for CT with unmatched projector / back-projector
 * pairs, and CGLS for comparison.
 *
 * Method: Sidky, Hansen, Jorgensen, Pan, "Iterative image reconstruction for
 * CT with unmatched projection matrices using the generalized minimal
 * residual algorithm".
 *   - the linear CT model A x = b after the negative log (Sec. I, Eq. 1);
 *   - CGLS for min ||A x - b|| with A^T replaced by B (Sec. I, Eq. 2);
 *   - AB-GMRES: A B y = b, x = B y (Sec. II, Eq. 4);
 *   - BA-GMRES: B A x = B b (Sec. II, Eq. 5);
 *   - zero initial vector; first basis vector b (AB) or B b (BA); one
 *     orthonormalised basis vector and one least-squares solve per
 *     iteration; the iteration count is the only parameter (Sec. II);
 *   - A ray-driven, B_un voxel-driven with linear interpolation on the
 *     detector, B_FBP = B_un F with F the ramp filter (Sec. III).
 *
 * Conventions (all lengths FP64, in the same unit as the voxel size):
 *   volume   float x[nz][ny][nx] (x fastest); voxel (ix,iy,iz) has centre
 *            ((ix-(nx-1)/2) d, (iy-(ny-1)/2) d, (iz-(nz-1)/2) d), d = voxel.
 *   data     y[n_views][nv][nu] (u fastest); 2D uses nz = nv = 1.
 *   angles   NULL -> uniform: t_p = (pi*p)/P (2D) or (2*pi*p)/P (3D).
 *   2D       parallel beam. View p: n = (cos t, sin t), d = (-sin t, cos t);
 *            bin a at s = (a-(nu-1)/2) du; ray { s n + t d }.
 *   3D       circular cone beam. Source (SOD cos t, SOD sin t, 0); detector
 *            centre = source - SDD (cos t, sin t, 0); e_u = (-sin t, cos t, 0),
 *            e_v = (0,0,1); pixel (au,av) at centre + u e_u + v e_v with
 *            u = (au-(nu-1)/2) du, v = (av-(nv-1)/2) dv.
 *
 * Operators:
 *   A      chosen per geometry (ct_geometry_desc.projector):
 *          CT_JOSEPH: for the dominant axis a of the ray direction r (ties go
 *          to x, then y; for the uniform 2D view set the choice is x-major
 *          iff P <= 4p <= 3P), sample the ray in every voxel-centre plane
 *          along a, interpolate bilinearly (linearly in 2D) in the plane with
 *          zero outside the grid, sum, multiply by d*|r|/|r_a|;
 *          CT_SIDDON: the line-intersection model the paper uses (Sec. III),
 *          A_ij = length of ray i inside voxel j (rays lying exactly on a
 *          voxel boundary plane give their length to either neighbour).
 *   A^T    exact transpose of A's weights.
 *   B_un   voxel-driven: 2D weight d^2/du times the linear interpolation of
 *          view p at s = x.n; 3D weight d^3 M^2/(du dv) times the bilinear
 *          interpolation at the voxel's perspective projection
 *          (M = SDD/U, U = SOD - (x cos t + y sin t)); zero outside the
 *          detector; summed over views.
 *   F      Ram-Lak along u: (F q)[a] = du * sum_a' h[a-a'] q[a'],
 *          h[0] = 1/(4 du^2), h[even] = 0, h[odd j] = -1/(pi^2 j^2 du^2);
 *          zero-padded linear convolution per view and detector row.
 *
 * Memory: every array argument is a DEVICE pointer owned by the caller,
 * contiguous, 256-byte aligned for workspaces.  The library owns only the
 * geometry handle (immutable after creation; may be shared across streams
 * and threads).  Operators and solvers take a caller-provided workspace
 * sized by the matching *_workspace_bytes query; no entry point below
 * allocates device memory except ct_geometry_create.
 *
 * Streams: `stream` is a hipStream_t (NULL = the null stream).  Operators
 * are asynchronous.  Solvers enqueue all their work on `stream` and then
 * synchronise that stream once to return the residual history and the
 * iteration count.
 *
 * Errors: every entry point returns a ct_status; nothing throws or aborts
 * across the ABI.  ct_last_error() returns a thread-local message for the
 * last failure on the calling thread.  A GMRES breakdown is not an error:
 * it shows as *iters_done < opts->iters.
 */
#ifndef CT_ABBA_H
#define CT_ABBA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ct_geometry ct_geometry;

enum {
    CT_OK = 0,
    CT_ERR_ARG = 1,          /* invalid argument, size or workspace          */
    CT_ERR_ALLOC = 2,        /* device allocation failed (create only)      */
    CT_ERR_HIP = 3,          /* a HIP runtime call failed                    */
    CT_ERR_NUMERIC = 4,      /* non-finite value met in a solver             */
    CT_ERR_UNSUPPORTED = 5   /* valid input outside what the kernels cover  */
};

enum { CT_PARALLEL_2D = 0, CT_CONE_CIRCULAR_3D = 1 };
enum { CT_JOSEPH = 0, CT_SIDDON = 1 };   /* forward projector model */
enum { CT_F32 = 0, CT_F16 = 1 };                  /* data storage type    */
enum { CT_B_UNMATCHED = 0, CT_B_RAMP = 1, CT_B_AT = 2 };
enum { CT_SOLVER_BA = 0, CT_SOLVER_AB = 1, CT_SOLVER_CGLS = 2, CT_SOLVER_BA_MONITOR = 3,
       CT_SOLVER_BA_RESTARTED = 4 };
enum { CT_OP_A = 0, CT_OP_B = 1, CT_OP_B_RAMP = 2, CT_OP_AT = 3, CT_OP_FBP = 4 };

typedef struct {
    int kind;                 /* CT_PARALLEL_2D or CT_CONE_CIRCULAR_3D      */
    int nx, ny, nz;           /* nz = 1 for 2D                              */
    double voxel;             /* isotropic voxel size d > 0                 */
    int n_views;
    const double *angles;     /* HOST pointer to n_views radians, or NULL   */
    int nu, nv;               /* detector columns / rows (nv = 1 for 2D)    */
    double du, dv;            /* detector pitch (at the detector, cone)     */
    double sod, sdd;          /* source-isocentre, source-detector (cone)   */
    int projector;            /* CT_JOSEPH or CT_SIDDON (A and A^T)         */
} ct_geometry_desc;

typedef struct {
    int iters;                /* number of iterations K >= 0               */
    int B;                    /* CT_B_UNMATCHED, CT_B_RAMP (B_un F), CT_B_AT */
    int sino_dtype;           /* CT_F32, or CT_F16 storage of the solver's
                                 internal projections (FP32 arithmetic) */
    double breakdown_tol;     /* GMRES: stop when the new vector's norm after
                                 orthogonalisation is <= tol times its norm
                                 before; 0 -> 64 * 2^-24                    */
    int basis_dtype;          /* BA-GMRES (plain and restarted): CT_F32, or
                                 CT_F16 storage of the Krylov basis, whose
                                 size is the method's memory burden (Sec. II).
                                 Each new vector v is stored as FP16 of t v,
                                 t a power of two with t ||v|| in
                                 (sqrt(len)/2, sqrt(len)] (values near 1, no
                                 overflow); orthogonalisation, dots and
                                 norms stay FP32/FP64, and the rounding to
                                 FP16 applies to the FP32 vector.  Halves the
                                 basis memory and the orthogonalisation
                                 traffic.  CT_ERR_UNSUPPORTED for the other
                                 solvers and with the 2D line-intersection
                                 projector.  0 (= CT_F32) keeps FP32.       */
} ct_solver_opts;

/* Validate the descriptor, build per-view tables (FP64 cos/sin, 2D
 * dominant-axis flags, Ram-Lak taps) and upload them to the current device.
 * Errors: CT_ERR_ARG for non-positive sizes or pitches, SDD <= SOD, a volume
 * that reaches the source circle; CT_ERR_UNSUPPORTED for cone angles at
 * which a ray could be z-dominant, or for volumes whose padded copy exceeds
 * 4 GiB; CT_ERR_ALLOC / CT_ERR_HIP on device failures.  *out is NULL on
 * error.  Caller destroys with ct_geometry_destroy. */
int ct_geometry_create(const ct_geometry_desc *desc, ct_geometry **out);

/* Free the handle and its device tables.  NULL is ignored.  The caller must
 * make sure no enqueued work still uses the handle. */
void ct_geometry_destroy(ct_geometry *g);

/* n_vox = nx*ny*nz, n_rays = n_views*nv*nu.  Either pointer may be NULL. */
int ct_geometry_sizes(const ct_geometry *g, size_t *n_vox, size_t *n_rays);

/* Workspace bytes needed by one operator call over `batch` items
 * (op = CT_OP_*).  CT_OP_B needs none (0). */
int ct_op_workspace_bytes(const ct_geometry *g, int op, int batch, size_t *bytes);

/* y = A x (Sec. III, the ray-driven projector; Joseph's discretisation or
 * the line-intersection model, as the geometry says).
 * x: float[batch][nz][ny][nx]; y: float or half (y_dtype)
 * [batch][n_views][nv][nu], round-to-nearest-even for half.
 * ws: >= ct_op_workspace_bytes(CT_OP_A) bytes. */
int ct_project_A(const ct_geometry *g, const float *x, void *y, int y_dtype,
                 int batch, void *ws, size_t ws_bytes, void *stream);

/* y = A x as ct_project_A, for callers that cannot allocate device memory
 * or pass a workspace: code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation.  The padded volume copies live in a
 * static device array of CT_NOALLOC_SCRATCH_BYTES bytes (enough for volumes
 * up to 256^3: 138.4 MB), one per GPU, held from the first call on that GPU
 * until the process ends.  Allocates nothing and records no kernel timing;
 * the results are those of ct_project_A bit for bit.
 * Every call on one GPU shares that GPU's array (it keeps the last call's
 * contents; each call rewrites what it reads): calls that overlap on one
 * GPU, from any stream or thread, race and must be serialised by the
 * caller.  CT_ERR_UNSUPPORTED (with the sizes in ct_last_error) when the
 * geometry's copies need more than CT_NOALLOC_SCRATCH_BYTES; other errors as
 * ct_project_A. */
#define CT_NOALLOC_SCRATCH_BYTES (144u << 20)
int ct_project_A_noalloc(const ct_geometry *g, const float *x, void *y, int y_dtype,
                         int batch, void *stream);

/* x = B_un y, or x = B_un F y when ramp_filter != 0 (Sec. III, B_un and
 * B_FBP).  y: float or half [batch][n_views][nv][nu]; x: float[batch][...].
 * ws: >= ct_op_workspace_bytes(CT_OP_B or CT_OP_B_RAMP) bytes (may be NULL
 * when that is 0). */
int ct_backproject_B(const ct_geometry *g, const void *y, int y_dtype, float *x,
                     int ramp_filter, int batch, void *ws, size_t ws_bytes,
                     void *stream);

/* x = A^T y, the exact transpose of ct_project_A (Sec. I: CGLS requires
 * B = A^T).  Gathered per voxel (each voxel sums the weighted values of the
 * rays whose samples touch it, in a fixed order, without atomics), so the
 * result is the same bits on every run.
 * ws: >= ct_op_workspace_bytes(CT_OP_AT) bytes (cone beam: the data
 * weighted by each ray's step length; 2D: none, ws may be NULL). */
int ct_backproject_AT(const ct_geometry *g, const void *y, int y_dtype, float *x,
                      int batch, void *ws, size_t ws_bytes, void *stream);

/* y = F q, the Ram-Lak filter alone (Sec. III).  q, y: float
 * [batch][n_views][nv][nu]; q == y is not allowed. */
int ct_ramp_filter(const ct_geometry *g, const float *q, float *y, int batch,
                   void *stream);

/* One-shot filtered back-projection, the reference reconstruction the paper
 * compares against (Sec. III), built from B_un and F:
 *   2D parallel beam:  x = (pi/P) (du/d^2) B_un F y;
 *   3D circular cone:  x = (pi/P) (SOD/SDD) (du dv/d^3) B_un F (w . y),
 *     w = SDD / sqrt(SDD^2 + u^2 + v^2) (Feldkamp-Davis-Kress cosine
 *     pre-weighting; B_un's M^2 weight carries the distance weighting).
 * y: float or half [batch][n_views][nv][nu]; x: float[batch][nz][ny][nx].
 * ws: >= ct_op_workspace_bytes(CT_OP_FBP) bytes. */
int ct_fbp(const ct_geometry *g, const void *y, int y_dtype, float *x, int batch,
           void *ws, size_t ws_bytes, void *stream);

/* Workspace bytes for a solver (CT_SOLVER_*, CT_SOLVER_BA_MONITOR for
 * ct_ba_gmres_monitor) with the given options. */
int ct_solver_workspace_bytes(const ct_geometry *g, int solver,
                              const ct_solver_opts *opts, size_t *bytes);

/* BA-GMRES (Sec. II, Eq. 5): x_K minimises ||B b - B A x|| over the Krylov
 * space K_K(B A, B b), x0 = 0.  b: float[n_views][nv][nu]; x: float[nz][ny][nx].
 * Basis FP32 in the workspace; dot products, norms, the Hessenberg matrix,
 * the Givens rotations and the triangular solve in FP64 on the device.
 * res_hist: HOST double[iters+1] or NULL; res_hist[k] = ||B b - B A x_k||
 * as carried by the rotations (res_hist[0] = ||B b||).  iters_done: HOST,
 * may be NULL; < iters after a breakdown, 0 when B b = 0 (then x = 0).
 * CT_ERR_NUMERIC if a non-finite value appears (x is then unspecified). */
int ct_ba_gmres(const ct_geometry *g, const float *b, float *x,
                const ct_solver_opts *opts, void *ws, size_t ws_bytes,
                double *res_hist, int *iters_done, void *stream);

/* BA-GMRES as ct_ba_gmres, plus the per-iteration curves the paper plots
 * (Sec. III, Figs. 2 and 4: data residual and image error against the iteration number),
 * without applying A again: the projections A w_k computed by the
 * iteration are kept (n_views*nv*nu floats per iteration in the
 * workspace; query with solver CT_SOLVER_BA_MONITOR) and combined with the
 * coefficients of each iterate x_k.
 *   x_ref:    DEVICE float[nz][ny][nx] reference image, or NULL.
 *   data_res: HOST double[iters+1] or NULL; data_res[k] = ||b - A x_k||
 *             (data_res[0] = ||b||).
 *   img_rmse: HOST double[iters+1] or NULL; img_rmse[k] =
 *             sqrt(sum (x_k - x_ref)^2 / n) (NaN without x_ref).
 * Entries after a breakdown are NaN.  opts->sino_dtype must be CT_F32
 * (CT_ERR_UNSUPPORTED otherwise).  x and res_hist equal ct_ba_gmres's. */
int ct_ba_gmres_monitor(const ct_geometry *g, const float *b, float *x,
                        const float *x_ref, const ct_solver_opts *opts,
                        void *ws, size_t ws_bytes, double *res_hist,
                        double *data_res, double *img_rmse, int *iters_done,
                        void *stream);

/* Restarted BA-GMRES(m): `cycles` cycles of opts->iters = m BA-GMRES steps
 * (Sec. II, Eq. 5), each on the data residual of the current iterate:
 * x <- x + argmin over K_m(BA, B(b - A x)) of ||B(b - A x) - B A d||.  The
 * basis holds m + 1 vectors instead of K + 1 (the storage the paper names as
 * the method's burden), at the price of the convergence a full Krylov space
 * would give.  Cycle 1 equals ct_ba_gmres with m iterations.
 *   res_hist: HOST double[cycles][m+1] or NULL, each cycle's residual
 *             history as in ct_ba_gmres (NaN after a breakdown);
 *   iters_done: HOST, total iterations over the cycles.
 * Workspace: ct_solver_workspace_bytes(CT_SOLVER_BA_RESTARTED) with
 * opts->iters = m.  Other arguments as ct_ba_gmres. */
int ct_ba_gmres_restarted(const ct_geometry *g, const float *b, float *x,
                          const ct_solver_opts *opts, int cycles, void *ws,
                          size_t ws_bytes, double *res_hist, int *iters_done,
                          void *stream);

/* AB-GMRES (Sec. II, Eq. 4): y_K minimises ||b - A B y|| over
 * K_K(A B, b), x = B y.  Basis in data space.  res_hist[k] = ||b - A x_k||
 * as carried by the rotations.  Other arguments as ct_ba_gmres. */
int ct_ab_gmres(const ct_geometry *g, const float *b, float *x,
                const ct_solver_opts *opts, void *ws, size_t ws_bytes,
                double *res_hist, int *iters_done, void *stream);

/* CGLS (Sec. I, Eq. 2) with A^T replaced by opts->B (CT_B_AT gives the
 * textbook method; CT_B_UNMATCHED / CT_B_RAMP give the unmatched variant the
 * paper shows diverging).  res_hist[k] = ||b - A x_k|| from the recurrence.
 * Scalars stay on the device in FP64. */
int ct_cgls(const ct_geometry *g, const float *b, float *x,
            const ct_solver_opts *opts, void *ws, size_t ws_bytes,
            double *res_hist, int *iters_done, void *stream);

/* Batched BA-GMRES (Sec. II, Eq. 5) over `count` independent 2D parallel-beam
 * problems of any sizes, solved together: each step of the iteration runs
 * as one launch over all problems, and the whole chain is replayed from a
 * captured hipGraph (see ct_batched_config).  Every problem gets the result
 * ct_ba_gmres would give it up to the order of FP64 sums.
 *   g:  HOST array of `count` geometry handles (CT_PARALLEL_2D, all on the
 *       current device; the same handle may appear more than once).
 *   b:  HOST array of `count` DEVICE pointers, float[n_views][nu] each.
 *   x:  HOST array of `count` DEVICE pointers, float[ny][nx] each (outputs).
 *   opts: as ct_ba_gmres; B = CT_B_UNMATCHED or CT_B_RAMP, sino_dtype CT_F32,
 *       CT_JOSEPH geometries (others: CT_ERR_UNSUPPORTED); the same
 *       iteration count for all.
 *   ws: DEVICE workspace of ct_ba_gmres_batched_workspace_bytes bytes.  It
 *       holds the per-problem tables, so a cached graph is tied to it: do
 *       not use one workspace from two calls at once.
 *   res_hist: HOST double[count][iters+1] or NULL (per problem as in
 *       ct_ba_gmres; NaN after a problem's breakdown).
 *   iters_done: HOST int[count] or NULL.
 * The call synchronises `stream` once at the end.  CT_ERR_NUMERIC if any
 * problem met a non-finite value (the others' results are valid).
 * count == 0 is a no-op. */
int ct_ba_gmres_batched_workspace_bytes(const ct_geometry *const *g, int count,
                                        const ct_solver_opts *opts, size_t *bytes);
int ct_ba_gmres_batched(const ct_geometry *const *g, int count,
                        const float *const *b, float *const *x,
                        const ct_solver_opts *opts, void *ws, size_t ws_bytes,
                        double *res_hist, int *iters_done, void *stream);

/* Execution choices of ct_ba_gmres_batched (process-wide):
 *   use_graph: 1 (default) capture the solve into a hipGraph on the first
 *       call for a batch shape / workspace / options and replay it; 0 launch
 *       the kernels directly on the stream.
 *   a_variant, b_variant: -1 (default) pick by timing every variant on the
 *       first solve of a batch shape (cached); otherwise force the 2D
 *       projector variant (0, 1: plane loop unrolled by 4, 8) or the 2D
 *       back-projector variant (0, 1, 2: 1, 2, 4 pixels per work-item).
 *       All variants give identical results.
 * ct_batched_last_config reports the choices of the last batched solve. */
int ct_batched_config(int use_graph, int a_variant, int b_variant);
int ct_batched_last_config(int *use_graph, int *a_variant, int *b_variant);

/* Launch setting of the cone-beam forward projector (the staged Joseph and
 * line-intersection kernels behind ct_project_A and the solvers).  Its
 * workgroups are 16 x 16 ray tiles of one view; a setting picks the order
 * they are dealt to the eight XCDs and how many stay resident per CU:
 *   vgrp in 1..64: XCD-contiguous order, groups of vgrp views (the same
 *       tile of a group's views on one XCD, sharing its L2);
 *   vgrp in -16..-1: band order, groups of -vgrp views (all XCDs on one
 *       band of detector rows, for volumes beyond the last-level cache);
 *   wg_per_cu in 1..8: at most that many resident workgroups per CU
 *       (dynamic LDS), 0: as many as fit.
 * Every setting gives bit-identical results; only the time differs.
 * ct_projector_config stores a setting in the geometry handle (0, 0: the
 * size heuristic, which is the default: groups of 10 views in XCD order
 * while both padded volume copies fit the 256 MB last-level cache, else
 * the band order in groups of 4 at 4 workgroups per CU); it may be called
 * while other threads use the handle (they see the old or the new
 * setting).  ct_projector_get_config returns the setting in use (0, 0 for
 * 2D geometries, which have no such setting).
 * Errors: CT_ERR_ARG (NULL, out of range), CT_ERR_UNSUPPORTED (a non-zero
 * setting for a 2D geometry). */
int ct_projector_config(ct_geometry *g, int vgrp, int wg_per_cu);
int ct_projector_get_config(const ct_geometry *g, int *vgrp, int *wg_per_cu);

/* Autotuner of that setting: times each candidate on this geometry (one
 * warm-up and `reps` timed launches of the forward projector, hipEvents on
 * `stream`, on a scratch volume of pseudo-random values and a scratch
 * sinogram that this call allocates with hipMalloc and frees before it
 * returns; `stream` is synchronised) and stores the fastest with
 * ct_projector_config.  Candidates: groups of 4, 6, 8, 10, 12 and 16 views
 * in XCD order at full occupancy, and where the padded copies exceed the
 * last-level cache also the band order with groups of 2, 4 and 6 views at
 * 3, 4 and 5 workgroups per CU.  Launches made by other threads with this
 * handle meanwhile run with one of the candidates.
 *   reps: 1..100.
 *   cap, vgrp, wg_per_cu, ms: HOST arrays of `cap` entries (may be NULL
 *       when cap == 0) receiving the first min(cap, count) candidates'
 *       settings and mean milliseconds per launch.
 *   count: HOST, may be NULL: the number of candidates (0 for 2D
 *       geometries, which are left as they are).
 * Not for graph capture (kernel timing with events, allocation).  On an
 * error the previous setting is kept.  Errors: CT_ERR_ARG, CT_ERR_ALLOC,
 * CT_ERR_HIP. */
int ct_tune_projector(ct_geometry *g, int reps, int cap, int *vgrp, int *wg_per_cu, double *ms, int *count,
                      void *stream);

/* Kernel timing (opt-in tracing).  When enabled, every projector,
 * back-projector, filter and orthogonalisation kernel launched by the
 * library is bracketed by two hipEvents recorded on the stream it runs on.
 * ct_profile_read synchronises those events and returns, for the kernel
 * class `name` ("A", "AT", "B", "F", "CGS", "ARNOLDI"), the number of
 * launches and their summed duration in milliseconds since the last reset.
 * Recording stops when 65536 launches are held.  Not for graph capture.
 * Errors: CT_ERR_ARG for an unknown name or NULL outputs, CT_ERR_HIP. */
int ct_profile_enable(int on);
int ct_profile_reset(void);
int ct_profile_read(const char *name, long *launches, double *total_ms);

/* Measured ceilings of the device the calling thread has current, the
 * constants the kernels' rooflines are measured against (measurement
 * infrastructure for callers that report a roofline; not an operation of
 * the method).  Each figure is the best of five timed launches after a
 * warm-up:
 *   hbm_copy_gbs:      device-to-device copy of 512 MiB, bytes read plus
 *                      bytes written per second, in GB/s;
 *   hbm_read_gbs:      streaming read (sum) of 1 GiB, GB/s;
 *   fp32_fma_tflops:   independent v_fma_f32 chains, 2 FLOP each, TFLOP/s;
 *   fp32_add_tflops:   independent v_add_f32 chains, TFLOP/s;
 *   lds_bilinear_gsps: bilinear samples per second (1e9) of the kind the
 *                      projectors take (two plane coordinates, integer and
 *                      fraction parts, four taps, three linear
 *                      interpolations, an accumulate), taps from an LDS tile;
 *   l2_bilinear_gsps:  the same samples with the taps gathered from a 1 MiB
 *                      array resident in L2;
 *   lds_gather_gbs:    the taps alone (four floats per sample, the address
 *                      stepping by a row and/or a column), bytes read from
 *                      LDS per second, GB/s: the gather bandwidth;
 *   l2_gather_gbs:     the same taps gathered from the L2-resident array;
 *   lds_peak_gbs:      LDS read bandwidth without bank conflicts (each lane
 *                      16 consecutive bytes per read), GB/s.
 *   out: HOST, filled on success (left as it is on an error).
 *   stream: hipStream_t the kernels run on (NULL: the null stream).
 * Allocates and frees 1 GiB plus 4 MiB of device memory; takes about a
 * second.  Not for graph capture.  Errors: CT_ERR_ARG for a NULL out,
 * CT_ERR_ALLOC, CT_ERR_HIP. */
typedef struct ct_ceilings {
    double hbm_copy_gbs;
    double hbm_read_gbs;
    double fp32_fma_tflops;
    double fp32_add_tflops;
    double lds_bilinear_gsps;
    double l2_bilinear_gsps;
    double lds_gather_gbs;
    double l2_gather_gbs;
    double lds_peak_gbs;
} ct_ceilings;
int ct_measure_ceilings(ct_ceilings *out, void *stream);

/* Thread-local description of the last error on this thread ("" if none). */
const char *ct_last_error(void);

/* Library version string. */
const char *ct_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CT_ABBA_H */
