/*
 * fks.h - C ABI of the MI355X (gfx950) fast spectral Boltzmann collision library.
 *
 * The library evaluates, independently in every spatial cell, the fast spectral
 * approximation of the variable-hard-sphere (VHS) Boltzmann collision operator
 * Q(f,f) of Dimarco, Loubere, Narski and Rey (Section 3.3: eqs. ode, FKM and the
 * decoupled 3D formula), applies the L2 conservation projection of Section 3.2
 * (eq. minim1) and the forward-Euler collision update of Section 3.1
 * (eq. f_coll, with the 1/tau rescaling of Part 2), and performs the exact FKS
 * transport shift of piecewise-constant data (Section 3.1 eq. f_bar, particle
 * form of Section 4.1), whole-grid or on one z slab of a decomposed grid with
 * the halo messages between slabs (Section 4.2).
 *
 * Conventions shared by every entry point
 *   - Velocity grid: n points per axis on [-T, T), nodes v_j = -T + j*2T/n.
 *     A cell's distribution is n^3 FP64 values in C order f[x][y][z].
 *   - Batches are cell-major: f[cell][x][y][z], contiguous.
 *   - Pointers documented as "device" must be device memory of the current
 *     HIP device; "host" pointers are ordinary host memory.  The caller owns
 *     every array; the library never frees caller memory.
 *   - hip_stream is a hipStream_t passed as void* (NULL = default stream).
 *     All device work of a call is enqueued on that stream; calls return
 *     after enqueueing (asynchronously) unless stated otherwise.
 *   - Every function returns fks_status; nothing throws across the ABI.
 *     Argument validation happens before anything is enqueued, so an
 *     FKS_ERR_INVALID / FKS_ERR_UNSUPPORTED return leaves all buffers untouched.
 */
#ifndef FKS_H
#define FKS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FKS_OK = 0,
    FKS_ERR_INVALID = -1,      /* bad argument, size or pointer */
    FKS_ERR_UNSUPPORTED = -2,  /* valid request outside the implemented set (e.g. odd n) */
    FKS_ERR_NOMEM = -3,        /* device allocation failed (plan creation only) */
    FKS_ERR_DEVICE = -4,       /* a HIP runtime call or kernel launch failed */
    FKS_ERR_NUMERIC = -5       /* non-finite Q_c recorded by the numeric guard (fks_numeric_status) */
} fks_status;

typedef enum {
    FKS_PREC_F64 = 0,          /* plain FP64 path: transforms, products and fix in FP64 */
    FKS_PREC_F32_FIX64 = 1     /* FP32 transforms/products, FP64 moments + projection + update */
} fks_precision;

typedef enum {
    FKS_RULE_GAUSS = 0,        /* cos(theta_p) Gauss-Legendre, uniform azimuth (default) */
    FKS_RULE_MIDPOINT = 1      /* theta_p = (p+1/2)pi/n_polar with sin(theta) Jacobian */
} fks_dir_rule;

/* Path selection flags (fks_plan_desc.flags). */
#define FKS_FLAG_FORCE_GENERIC 0x1u  /* use the multi-pass path even where the fused kernel exists */
#define FKS_FLAG_NUMERIC_GUARD 0x2u  /* record the first cell whose Q_c is not finite (fks_numeric_status) */
/*
 * De-aliased convolution: only pairs l + m = k exactly (k in the band
 * -n/2 < k_i < n/2) enter Qhat_k, instead of the n-periodic sum of eq. ode.
 * Every inverse transform and product runs on a 3n/2 grid of the same box and
 * the band coefficients of the products are kept (zero-padding, the 3/2 rule);
 * the FP64 fix and update are unchanged.  Multi-pass path only; dim = 3 and
 * n in {4, 8, 12, 16, 24, 32}, else FKS_ERR_UNSUPPORTED.
 */
#define FKS_FLAG_DEALIAS 0x4u

/*
 * Operator description (Section 3.3).  Zero / non-positive optional fields
 * take the documented defaults.
 */
typedef struct {
    int32_t n;            /* velocity points per axis; even, 4 <= n <= 48, n = 2^a 3^b */
    double  T;            /* velocity half-box: grid on [-T, T) (T > 0) */
    double  R;            /* Carleman truncation radius; <= 0 -> 2T/(3+sqrt 2) */
    double  gamma;        /* VHS exponent, 0 <= gamma <= 1 (1 = hard spheres) */
    double  c_gamma;      /* kernel constant C_gamma; <= 0 -> 1/(4 pi) */
    int32_t n_polar;      /* polar nodes A1 (>= 1) */
    int32_t n_azim;       /* azimuthal nodes A2 (>= 1); M = A1*A2 directions on the half sphere */
    int32_t rule;         /* fks_dir_rule */
    int32_t radial_terms; /* K for gamma != 1; 0 -> smallest K with lambda_K/lambda_0 < radial_tol */
    double  radial_tol;   /* <= 0 -> 1e-4 */
    int32_t precision;    /* fks_precision */
    uint32_t flags;       /* FKS_FLAG_* */
    int32_t dim;          /* velocity dimension d_v: 3 (0 -> 3) or 2 (see below) */
} fks_plan_desc;

/*
 * dim = 2: Maxwell molecules in two velocity dimensions, the decoupled
 * two-dimensional formula of Section 3.3 (eq. dfor0): B_F(l, m) =
 * 2 C_0 (pi/A) sum_p phi(kappa l.e_p) phi(kappa m.e_p^perp), phi(s) = 2R Sinc(Rs),
 * e_p = (cos t_p, sin t_p), t_p = pi p / A, p = 1..A.  Fields: n in
 * {8, 12, 16, 24, 32, 48, 64} (FP64: n <= 32); n_polar = A (angles);
 * n_azim must be 1; gamma must be 0 (FKS_ERR_UNSUPPORTED otherwise);
 * c_gamma = C_0, <= 0 -> 1/(2 pi) (then the loss term is rho f);
 * radial_terms 0 or 1; rule and radial_tol are ignored; FKS_FLAG_FORCE_GENERIC
 * is unsupported.  Arrays are [ncell][n][n] FP64 (x-major), the invariants are
 * (1, v_x, v_y, |v|^2), and fks_collide_batch needs no workspace for them.
 */

typedef struct fks_plan fks_plan;   /* opaque: owns device tables; immutable after creation except
                                       for the schedule cache that fks_autotune fills */

typedef struct {
    int32_t n;                 /* as described */
    int32_t M;                 /* directions n_polar*n_azim */
    int32_t K;                 /* radial terms actually used */
    int32_t J;                 /* convolution terms per cell: M*K gain terms + 1 loss term */
    double  R;                 /* truncation radius actually used */
    double  c_gamma;           /* kernel constant actually used */
    int32_t precision;         /* fks_precision */
    int32_t fused;             /* 1 if fks_collide_batch uses the fused kernels (FP32, dim 3, n in
                                  {8, 16, 24, 32, 48}; at n = 48 three workgroups per cell) */
    size_t  table_bytes;       /* device bytes held by the plan */
    double  flops_per_cell;    /* algorithmic flops of one Q evaluation: (2J'+2) 2.5 N log2 N + 7J' N + 3N,
                                  N = n^3 (n^2 for dim 2), J' = J - 1 (a real FFT counts 2.5 N log2 N);
                                  the de-aliased variant counts its zero-padded transforms instead */
    int32_t dim;               /* velocity dimension (2 or 3) */
    int32_t fused_grid;        /* workgroups the fused terms kernel keeps resident (0 if not fused) */
    int32_t queue_items_per_wg; /* work queues led by this plan: items per resident workgroup
                                   kept by fks_autotune (0: the cost model's 4) */
} fks_plan_info;

/*
 * Creates a plan: directions, radial expansion and the 5x5 Gram matrix of the
 * collision invariants are computed on the host in FP64; the kernel-mode
 * tables alpha_{e,r}(k), beta_{e,r}(k) (half spectrum, kz in [0, n/2]) and the
 * loss table L(k) = B_F(k,k) are computed on the device in FP64, then rounded
 * to FP32 for the FP32 path.  Blocks until the tables are built.
 * Errors: FKS_ERR_INVALID (NULL pointers, out-of-range fields),
 * FKS_ERR_UNSUPPORTED (n odd or not 2^a 3^b, n > 48), FKS_ERR_NOMEM, FKS_ERR_DEVICE.
 * On error *out is set to NULL.
 */
fks_status fks_plan_create(const fks_plan_desc* desc, void* hip_stream, fks_plan** out);

/* Frees the plan's device memory (on the device the plan was created on; hipFree
 * waits for work pending there, so no explicit synchronisation is made).  The caller
 * must not destroy a plan that another host thread is using.  NULL is a no-op. */
fks_status fks_plan_destroy(fks_plan* plan);

/* Fills *info (host).  FKS_ERR_INVALID on NULL. */
fks_status fks_plan_query(const fks_plan* plan, fks_plan_info* info);

/*
 * Numeric guard of a plan created with FKS_FLAG_NUMERIC_GUARD: every segment of
 * the plan in fks_collide_batch records, in a device word the plan owns, the
 * smallest cell index (within its segment) whose Q_c has a non-finite moment sum.
 * This call synchronises the device, then returns FKS_ERR_NUMERIC with
 * *first_bad_cell = that index if one was recorded since the last reset, else
 * FKS_OK with *first_bad_cell = -1; reset = 1 clears the word afterwards.  Calls
 * that overlap on one plan share the word.  FKS_ERR_INVALID for NULL arguments
 * or a plan without the flag.
 */
fks_status fks_numeric_status(const fks_plan* plan, int64_t* first_bad_cell, int32_t reset);

/*
 * Copies the plan's FP64 tables to host memory, for inspection and tests.
 * ab_host: [J][n/2+1][n][n][2] doubles = (omega_j * alpha_j(k), beta_j(k)) with
 * k = (kx, ky, kz) in FFT storage order, kz in [0, n/2]; the last term
 * (j = J-1) is the loss term (-L(k), 1).  Either pointer may be NULL.
 * dirs_host: [M][4] doubles = (e_x, e_y, e_z, w_e).  Synchronous.
 * dim = 2: ab_host is [J][n][n][2] = (sqrt(w) alpha_p(k), sqrt(w) alpha'_p(k)),
 * w = 2 C_0 pi / A, k = (kx, ky) in FFT storage order, and the loss term is
 * (-L(k)/s, s) with s = sqrt(L(0)); dirs_host rows are (cos t_p, sin t_p, 0, pi/A).
 */
fks_status fks_plan_copy_tables(const fks_plan* plan, double* ab_host, double* dirs_host);

/*
 * One homogeneous run of cells sharing a plan.
 *   f      device, const, [ncell][n][n][n] FP64: the post-transport distribution f*.
 *   q_out  device, [ncell][n^3] FP64, or NULL: receives Q_c, the collision
 *          operator after the conservation projection (Section 3.2).
 *   f_out  device, [ncell][n^3] FP64, or NULL: receives f_base + dt_over_tau * Q_c
 *          (eq. f_coll).  May alias f or f_base (in-place update); must not
 *          overlap q_out.
 *   f_base device, [ncell][n^3] FP64, or NULL (= f): the state the update starts
 *          from.  With f_base != f one call is a stage of a Runge-Kutta step,
 *          e.g. the midpoint rule f + dt Q(f + dt/2 Q(f)) is two calls.
 *   At least one of q_out, f_out must be non-NULL.  ncell >= 0 (0 = nothing).
 *   f, q_out and f_out must be 16-byte aligned (every cell boundary of an
 *   array from hipMalloc is).
 */
typedef struct {
    const fks_plan* plan;
    const double*   f;
    double*         q_out;
    double*         f_out;
    int64_t         ncell;
    double          dt_over_tau;
    const double*   f_base;
} fks_segment;

/* Device workspace bytes needed by fks_collide_batch for these segments (host call). */
fks_status fks_workspace_size(const fks_segment* segs, int32_t nseg, size_t* bytes);

/*
 * Evaluates Q(f,f) for every cell of every segment (fast spectral form with
 * Nyquist planes zeroed: the n-periodic convolution, or the de-aliased one for
 * plans with FKS_FLAG_DEALIAS), projects it onto the kernel of the collision
 * invariants in FP64 and writes q_out / f_out.  workspace: device memory of at
 * least fks_workspace_size bytes for the same segments (the size depends on
 * ncell: large FP32 batches run one workgroup per cell, small ones pairs of
 * workgroups with partial sums), 256-byte aligned, owned by the caller, not
 * used concurrently by another call.  No device allocation, host
 * synchronisation or memset happens inside, so the call can be captured in a
 * HIP graph.  Results are deterministic (no floating-point atomics).
 *   Launch groups: segments of fused FP32 plans (fks_plan_info.fused) that share
 *   n, two or more in one call (up to 16 per group), run together: at n <= 32 one
 *   work queue whose items are a cell's terms or a range of them (cells with many
 *   terms are cut into ranges so that items have similar lengths; longest
 *   first), FP32 partial sums, then one FP64 fix over all the group's cells; at
 *   n = 48 one launch of the three-workgroup kernel over all their cells.  Other
 *   segments run alone, in call order.  The grouping depends only on the
 *   segments' plans and sizes (and the queue's items per workgroup, which
 *   fks_autotune may keep in the first segment's plan), so results are
 *   reproducible call to call.
 * Errors: FKS_ERR_INVALID (NULL plan/f, both outputs NULL, ncell < 0,
 * misaligned arrays, small or misaligned workspace), FKS_ERR_DEVICE (launch
 * failure).
 */
fks_status fks_collide_batch(const fks_segment* segs, int32_t nseg, void* workspace,
                             size_t ws_bytes, void* hip_stream);

/*
 * fks_collide_batch without a workspace argument, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same segments, kernels, schedules and
 * results (bit for bit) as fks_collide_batch with a caller workspace; the
 * workspace is instead a static device array of FKS_STATIC_WORKSPACE_BYTES that
 * the library holds on every GPU it runs on until the process ends (its address
 * is looked up once per device, at plan creation).  Nothing is allocated or
 * freed and no allocating library routine is called.
 *   Segments whose workspace (fks_workspace_size) exceeds
 *   FKS_STATIC_WORKSPACE_BYTES are rejected with FKS_ERR_INVALID before anything
 *   is enqueued.  64 MiB holds the fused path's largest layout at n = 32 (one
 *   128 KiB spectrum slot per resident workgroup) and the small-batch pair layout
 *   up to about 170 cells of 32^3; the multi-pass path (FP64, n = 48) needs more
 *   for large batches and is then rejected.
 *   Every call on one GPU shares that GPU's array and leaves its contents behind
 *   (the kernels write every workspace location before reading it, so nothing
 *   needs clearing): calls that overlap on one GPU, on different streams or from
 *   different host threads, race and must be serialised by the caller.
 * Errors: as fks_collide_batch.
 */
#define FKS_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
fks_status fks_collide_batch_static(const fks_segment* segs, int32_t nseg, void* hip_stream);

/*
 * Autotuner.  For each segment, times the schedules fks_collide_batch can use
 * for it and keeps the fastest in the segment's plan, keyed by ncell: for
 * fused plans one workgroup per cell or pairs of workgroups per cell; for the
 * multi-pass path (FP64, n = 48, FKS_FLAG_FORCE_GENERIC, FKS_FLAG_DEALIAS) the
 * cells per pass batch (32, 64, 128, 256, 512 or ncell), which sets how much of
 * the work arrays stays in the on-chip caches, and the consecutive terms per
 * launch of the per-term kernels (1, 2 or 4; not for FKS_FLAG_DEALIAS), which
 * trades launches and accumulator traffic for work-array space.  Later fks_workspace_size and
 * fks_collide_batch calls with the same (plan, ncell) use the kept schedule when
 * the segment runs alone (not in a work queue with other segments of its n, see
 * fks_collide_batch); other sizes keep the built-in cost model.  Segments that
 * fks_collide_batch would run as one work queue (two or more fused segments of one
 * n <= 32) are also timed as that queue with 1, 2, 4 or 8 items per resident
 * workgroup (fewer items carry more terms each: the direction batch of an item); the
 * fastest is kept in every plan of the group, and a later queue uses the value of
 * its first segment's plan (fks_plan_info.queue_items_per_wg; 0 = the cost model's
 * 4).  fks_workspace_size must be asked again after tuning.  Schedules change the
 * summation order of the FP32 partial sums only, never the operator.
 *   Each segment is evaluated several times (its outputs are overwritten): its
 *   f_out must not overlap f or f_base.  workspace: at least
 *   fks_autotune_workspace_size bytes for the same segments (candidates that do
 *   not fit are skipped), 256-byte aligned.  choice_out: host [nseg][3] or
 *   NULL, receives (one workgroup per cell 1 / pairs 0 / -1, cells per pass
 *   batch or 0, terms per launch or 0) per segment.  Synchronises hip_stream; not for graph capture;
 *   no other call may use the same plans meanwhile.
 * Errors: FKS_ERR_INVALID (as fks_collide_batch, or overlapping outputs),
 * FKS_ERR_DEVICE.
 */
fks_status fks_autotune_workspace_size(const fks_segment* segs, int32_t nseg, size_t* bytes);
fks_status fks_autotune(const fks_segment* segs, int32_t nseg, void* workspace, size_t ws_bytes,
                        void* hip_stream, int32_t* choice_out);

/*
 * Moments U = C f (eq. i5 on the grid, C of Section 3.2): for each cell
 * U[cell] = dv^3 * sum_j f_j (1, v_x, v_y, v_z, |v|^2)  (FP64).
 * f device [ncell][n^3]; U device [ncell][5].  FP64 throughout.
 */
fks_status fks_moments(const double* f, int64_t ncell, int32_t n, double T, double* U,
                       void* hip_stream);

/*
 * L2 projection of every cell onto prescribed moments (eq. minim1):
 * f <- f + C^T (C C^T)^{-1} (U_target - C f).  f device [ncell][n^3] in/out;
 * U_target device [ncell][5] in the units of fks_moments.  FP64.
 */
fks_status fks_conserve(double* f, const double* U_target, int64_t ncell, int32_t n, double T,
                        void* hip_stream);

/* Spatial grid of the transport step: cells f[iz][iy][ix][n^3]. */
#define FKS_BC_PERIODIC 0
#define FKS_BC_DIRICHLET 1
typedef struct {
    int32_t nx, ny, nz;        /* cells per axis (>= 1) */
    double  dx;                /* cell width (> 0), equal on every axis */
    int32_t bc[3];             /* per axis (x, y, z): FKS_BC_PERIODIC or FKS_BC_DIRICHLET */
} fks_space_desc;

/*
 * Exact transport of piecewise-constant data (Section 3.1 eq. f_bar) in the
 * particle form of Section 4.1: per velocity component the accumulated
 * displacement s is advanced by v dt, and every velocity's mass moves by the
 * change of d = floor(s/dx + 1/2) cells.
 *   f_in   device, const [nz][ny][nx][n^3] FP64.
 *   f_out  device [nz][ny][nx][n^3] FP64; must not overlap f_in.
 *   offsets host [3][n] FP64, in/out: accumulated displacement of each 1D
 *          velocity index along x, y, z; updated by this call.
 *   bc_f   device [6][n^3] FP64 inflow states (faces x-, x+, y-, y+, z-, z+),
 *          read where a Dirichlet axis pulls mass from outside; may be NULL
 *          if no axis is Dirichlet.
 * Any integer shift is handled (periodic wrap or inflow); CFL <= 1 keeps it
 * within one cell.  Errors: FKS_ERR_INVALID.
 */
fks_status fks_transport_shift(const double* f_in, double* f_out, const fks_space_desc* space,
                               int32_t n, double T, double dt, double* offsets,
                               const double* bc_f, void* hip_stream);

/*
 * z-slab decomposition of the transport step (Section 4.2: the spatial domain is
 * cut into slices along z, one per process; each process collides its own cells
 * and exchanges the particle masses that cross a slice boundary with its
 * neighbours).  These calls are the per-GPU part of that exchange; moving the
 * messages between GPUs (point-to-point send/receive) is the caller's.
 *
 * A slab owns slab->nz consecutive z planes of a grid of slab->nx x slab->ny
 * cells:
 *   f      device [slab->nz][ny][nx][n^3] FP64 (no ghost planes).
 * Under CFL <= 1 the only masses that cross a z face in one step are those of
 * the velocities moving through it: v_z < 0 (kz < n/2, ceil(n/2) values of kz)
 * leave through z-, v_z > 0 (kz > n/2, n - 1 - floor(n/2) values) through z+.
 * A message holds those velocities of every cell of the boundary plane:
 *   buf    device [ny][nx][n][n][h] FP64, h the count of kz above; contiguous.
 */
#define FKS_FACE_ZLO 0   /* the z- face of a slab */
#define FKS_FACE_ZHI 1   /* the z+ face */

/* Bytes of the message that leaves a slab through `face` (and enters the
 * neighbour beyond it through the opposite face).  Host only.
 * Errors: FKS_ERR_INVALID (NULL pointer, bad slab, n outside 2..64, bad face). */
fks_status fks_halo_size(const fks_space_desc* slab, int32_t n, int32_t face, size_t* bytes);

/* Packs the message that leaves through `face`: the outgoing velocities of the
 * first (FKS_FACE_ZLO) or last (FKS_FACE_ZHI) plane of f into buf.  f is only
 * read.  Enqueued on hip_stream.  Errors: FKS_ERR_INVALID, FKS_ERR_DEVICE. */
fks_status fks_halo_pack(const double* f, const fks_space_desc* slab, int32_t n, int32_t face,
                         double* buf, void* hip_stream);

/* fks_transport_shift on a slab, f_in -> f_out (both [nz][ny][nx][n^3]), where
 * what enters through the z faces comes from the neighbours' messages:
 *   from_below  device, the message the slab below packed at its FKS_FACE_ZHI;
 *   from_above  device, the message the slab above packed at its FKS_FACE_ZLO
 * (for a periodic z axis the bottom slab's neighbour below is the top slab; a
 * single slab may pass its own messages).  x and y take slab->bc[0..1] as in
 * fks_transport_shift; slab->bc[2] is not read.  offsets, dt and bc_f as in
 * fks_transport_shift; every slab of a grid advances the same offsets.  The z
 * shift of the step must stay within what the messages hold: +1 only for
 * v_z > 0, -1 only for v_z < 0 (CFL <= 1, dt >= 0), else FKS_ERR_INVALID before
 * anything is enqueued and offsets unchanged.  f_in and f_out must not overlap;
 * the messages must not overlap f_out.  Errors: FKS_ERR_INVALID, FKS_ERR_DEVICE. */
fks_status fks_transport_shift_slab(const double* f_in, double* f_out, const fks_space_desc* slab,
                                    int32_t n, double T, double dt, double* offsets,
                                    const double* from_below, const double* from_above,
                                    const double* bc_f, void* hip_stream);

/*
 * Per-kernel timing of fks_collide_batch, for measurement tools.  While
 * enabled, the library records HIP events on the call's stream around each
 * kernel of the fused path: one kernel when a workgroup takes whole cells
 * (large batches), else the terms kernel, then the finish kernel.
 * fks_profile_last waits for the last recorded call to finish and writes up
 * to `capacity` durations in milliseconds (host array), in launch order;
 * *count receives how many kernels the last call timed (0 if none).
 * Calls must not overlap while profiling is enabled.
 */
fks_status fks_profile_enable(int32_t enable);
fks_status fks_profile_last(double* kernel_ms, int32_t capacity, int32_t* count);

/* Static string for a status code. */
const char* fks_status_string(fks_status status);

/*
 * Spectrum of a batch of cells (Section 3.3, eq. FC on the grid), in FP64: the
 * optional forward transform of Q (or of f) for a spectral-space update.
 *   xhat_k = n^-3 sum_j x_j exp(-i kappa k.v_j),  kappa = pi/T,  v_j = -T + j dv,
 * which does not depend on T: exp(-i kappa k.v_j) = (-1)^k exp(-2 pi i k.j / n).
 *   x      device, const, [ncell][n][n][n] FP64 (x-major, as f)
 *   xhat   device, [ncell][n][n][n/2+1][2] FP64: (re, im) at (kx, ky, kz), kx and
 *          ky in FFT storage order (0..n/2-1, -n/2..-1), kz in [0, n/2]; the rest
 *          of the spectrum is xhat(-k) = conj xhat(k).
 *   zero_nyquist  1: every mode with a component equal to n/2 is set to 0 (what
 *          the collision operator uses); 0: the plain transform.
 *   workspace  device, 256-byte aligned, at least one cell (16 n^3 bytes); cells
 *          are processed in chunks of up to min(512, ws_bytes / (16 n^3)).
 *          fks_spectrum_workspace_size gives the size for the largest chunk.
 * n as for fks_plan_desc (dim 3).  No overlap between x, xhat and workspace.
 * Errors: FKS_ERR_INVALID, FKS_ERR_UNSUPPORTED (n), FKS_ERR_DEVICE.
 */
fks_status fks_spectrum_workspace_size(int64_t ncell, int32_t n, size_t* bytes);
fks_status fks_spectrum(const double* x, double* xhat, int64_t ncell, int32_t n, int32_t zero_nyquist,
                        void* workspace, size_t ws_bytes, void* hip_stream);

/*
 * BGK relaxation operator with the conservative discrete Maxwellian
 * (Section 2 eq. ibgk; Section 3.2 eq. minimMax), FP64, per cell:
 *   U = C f;  (rho, u, theta) with d_v rho theta = sum |v|^2 f dv^d - rho |u|^2;
 *   M~ = rho (2 pi theta)^{-d/2} exp(-|v-u|^2 / (2 theta)) at the nodes;
 *   E = M~ + C^T (C C^T)^{-1} (U - C M~), so that C E = U exactly;
 *   Q = nu' (E - f) with nu' = nu (nu_rho = 0) or nu * rho (nu_rho = 1).
 * Outputs: q_out = Q; f_out = f + dt_over_tau Q (step FKS_BGK_EULER, eq. f_coll)
 * or E + exp(-nu' dt_over_tau) (f - E) (FKS_BGK_EXACT, the exact solution of
 * df/dt = nu'(E - f) with E fixed).  A cell with rho <= 0 or theta <= 0 has no
 * Maxwellian and is left unchanged (Q = 0).
 *   f      device, const, [ncell][n^dim] FP64 (same layout as fks_collide_batch)
 *   q_out  device [ncell][n^dim] or NULL; must not overlap f or f_out
 *   f_out  device [ncell][n^dim] or NULL; may alias f
 * dim 3: 2 <= n <= 64; dim 2: 2 <= n <= 512.  No workspace.  Asynchronous on
 * hip_stream.  Errors: FKS_ERR_INVALID (NULL desc or f, both outputs NULL,
 * overlaps, out-of-range fields, ncell < 0), FKS_ERR_DEVICE.
 */
typedef enum { FKS_BGK_EULER = 0, FKS_BGK_EXACT = 1 } fks_bgk_step;

typedef struct {
    int32_t dim;      /* 2 or 3 */
    int32_t n;        /* velocity points per axis */
    double  T;        /* grid on [-T, T)^dim */
    double  nu;       /* collision frequency, or its factor when nu_rho = 1 (>= 0) */
    int32_t nu_rho;   /* 0: nu' = nu; 1: nu' = nu * rho */
    int32_t step;     /* fks_bgk_step */
} fks_bgk_desc;

fks_status fks_bgk(const fks_bgk_desc* desc, const double* f, double* q_out, double* f_out,
                   int64_t ncell, double dt_over_tau, void* hip_stream);

/*
 * Scalars of the split scheme (host, no device needed).
 *   fks_stable_dt: the time step bound min(dx / T, tau / mu) of one split step,
 *     transport CFL (|v| <= T on the grid) and collision stability with
 *     mu = 4 pi C_gamma (2R)^gamma rho_max, the loss frequency of the truncated
 *     kernel at the largest density (Section 3.1; the paper states the bound for
 *     T = pi).  All arguments > 0 except gamma in [0, 1]; else FKS_ERR_INVALID.
 *   fks_exp_euler_step: the step length h = (1 - exp(-mu dt_over_tau)) / mu of the
 *     exponential Euler collision step f + h Q_c(f) for stiff collisions (the
 *     penalised form Q = [Q + mu (f - M)] - mu (f - M) with the linear part
 *     integrated exactly); h -> dt_over_tau as mu dt_over_tau -> 0 and h <= 1/mu.
 *     mu > 0 and dt_over_tau >= 0, finite; else FKS_ERR_INVALID.
 */
fks_status fks_stable_dt(double dx, double T, double tau, double R, double gamma, double c_gamma,
                         double rho_max, double* dt);
fks_status fks_exp_euler_step(double mu, double dt_over_tau, double* h);

/*
 * Host-only helpers (no device needed), exposed so that the host precompute
 * can be checked without a GPU.
 *   fks_desc_validate: the validation fks_plan_create performs.
 *   fks_host_sphere_rule: directions and weights of the half-sphere rule,
 *     e_w [n_polar*n_azim][4] = (e_x, e_y, e_z, w).
 *   fks_host_radial_terms: radial expansion for gamma (K requested, 0 -> by tol);
 *     *K_out receives K; nodes [nq], coef [nq][K] (row-major) may be NULL to query K.
 *   fks_host_tables_2d: the FP64 tables a dim = 2 plan uploads, ab [J][n][n][2]
 *     laid out as fks_plan_copy_tables describes; *J_out receives J = A + 1 and
 *     ab may be NULL to query it.
 */
fks_status fks_desc_validate(const fks_plan_desc* desc);
fks_status fks_host_sphere_rule(int32_t n_polar, int32_t n_azim, int32_t rule, double* e_w);
fks_status fks_host_radial_terms(double gamma, double R, int32_t K, double tol, int32_t nq,
                                 int32_t* K_out, double* nodes, double* coef);
fks_status fks_host_tables_2d(const fks_plan_desc* desc, int32_t* J_out, double* ab);

#ifdef __cplusplus
}
#endif

#endif /* FKS_H */
