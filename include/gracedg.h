/*
 * gracedg.h -- C ABI of the MI355X (gfx950) collision-operator library.
 *
 * The operator is the DG right-hand side of the coagulation-fragmentation
 * equation of Yang, Chen & Bai, "GRACE-DG: A Discontinuous Galerkin
 * Method-Based Code for General Nonlinear Coagulation-Fragmentation
 * Equations": the truncated coagulation flux and the paper's conservative
 * fragmentation flux (Sec. 2, Eqs. Fcoag and Ffrag; Sec. 3.3, Eqs. Fcoagtrun
 * and Ffragtrun; App. B, Eqs. inte1/inte2), assembled into the per-bin
 * Legendre right-hand side L[g] (Sec. 3.1, Eq. evo), the scaling limiter
 * (Sec. 3.2, Eqs. recon/gamma) and the SSP-RK3 step (Eq. RK3).
 *
 * Conventions shared by every call
 *  - Every call returns an int status: GD_OK (0) or a negative GD_E* code;
 *    gd_last_error() returns a thread-local message for the last failure.
 *  - Device pointers are plain HIP device addresses owned by the caller; the
 *    library never frees caller memory.  Host pointers are read during the
 *    call only.
 *  - State layout: hydro cells are contiguous, each cell holds P = bins*(order+1)
 *    doubles, coefficient index p = j*(order+1) + i for bin j and Legendre
 *    degree i (Eq. 2.3).  Cells of a plan are ordered group by group.
 *  - Calls on a plan are asynchronous on the plan's HIP stream unless stated.
 *  - A plan holds workspaces, work lists and captured graphs: calls on one plan
 *    must not overlap from several host threads.  Distinct plans share no writable device
 *    memory and may run on different streams at once.  A tensor is read only once
 *    its device layouts exist; the calls that build them on first use
 *    (gd_tensor_upload and gd_plan_create: the forward layouts; a plan's first
 *    gd_adjoint or gd_collision_vjp: the transposed layout) must not run
 *    concurrently on the same tensor.
 *  - Invalid arguments return GD_EINVAL before any launch; HIP failures return
 *    GD_EHIP with the HIP error string in gd_last_error().
 */
#ifndef GRACEDG_H
#define GRACEDG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    GD_OK = 0,
    GD_EINVAL = -1,   /* bad argument (shape, enum, null pointer)              */
    GD_EHIP = -2,     /* HIP runtime error                                      */
    GD_ENOMEM = -3,   /* device or host allocation failed                       */
    GD_EUNSUPPORTED = -4, /* combination not built (e.g. P above the kernels' limit) */
    GD_EPOSITIVITY = -5   /* returned after a step call that was given a violation counter
                             completed: the state is advanced (every step taken), but the
                             limiter found bins with a negative (or non-finite) average,
                             which it flattened keeping their mass (Sec. 3.2, Eq. gamma);
                             the counter holds how many.  A step beyond the CFL bound of
                             Eq. dt is the usual cause.                                 */
};

/* Collision kernel K(u,v) (Secs. 4.2-4.5). */
enum {
    GD_KERNEL_CONST = 0,          /* K = 1                                        */
    GD_KERNEL_ADDITIVE = 1,       /* K = u + v                                    */
    GD_KERNEL_MULTIPLICATIVE = 2, /* K = u v                                      */
    GD_KERNEL_BALLISTIC = 3,      /* K = (u^1/3 + v^1/3)^2 dv, dv = v0(u^-1/6+v^-1/6) */
    GD_KERNEL_MAXWELL = 4         /* Sec. 4.5: relative speeds Maxwellian with the
                                     constant rms v0; with the cross section
                                     sigma = pi (u^1/3 + v^1/3)^2 the coagulation
                                     rate is sigma v0 beta_coag(v_bounce) and the
                                     fragmentation rate sigma v0 beta_frag(v_frag),
                                     beta_* the probabilities of a speed below the
                                     bouncing threshold / above the fragmentation
                                     threshold (no sharp split of node pairs)       */
};

/* Fragment distribution b(w,u,v) of a fragmenting collision (Sec. 2.2, Sec. 4.4,
 * Eq. break).  A node pair (u,v) fragments when dv(u,v) = v0(u^-1/6 + v^-1/6)
 * exceeds the threshold v_frag, otherwise it coagulates. */
enum {
    GD_FRAG_NONE = 0,            /* pure coagulation                                */
    GD_FRAG_POWERLAW = 1,        /* b = A w^alpha on [x_min, u+v], no remnant       */
    GD_FRAG_UNIFORM_BINARY = 2,  /* b = 2/u 1[w<=u] + 2/v 1[w<=v] (Sec. 4.4)         */
    GD_FRAG_REMNANT_ONLY = 3,    /* b = delta(w-(u+v)): fragmentation == coagulation */
    GD_FRAG_GENERAL = 4          /* Eq. break with Eq. mfrag: b = A w^alpha on
                                    [x_min, m_frag] + delta(w - m_left), m_frag(u,v)
                                    set by the mass ratio (destructive, transition,
                                    cratering, transition, mass transfer), m_left =
                                    u + v - m_frag, A from local mass conservation;
                                    inner integrals of App. B (Eqs. inte1/inte2)   */
};

/* Arithmetic of the contraction. */
enum {
    GD_PREC_FP64 = 0,        /* FP64 MFMA, the plain double-precision form          */
    GD_PREC_MIXED_F16X3 = 1  /* FP16 hi+lo split of T and of the scaled state,
                                three FP16 MFMA products, FP32 accumulation; the
                                mass bookkeeping, limiter and RK update stay FP64 */
};

typedef struct {
    int kind;        /* GD_KERNEL_*                                     */
    double v0;       /* velocity scale of dv (and of the ballistic K);
                        GD_KERNEL_MAXWELL: the rms relative speed       */
    double v_bounce; /* GD_KERNEL_MAXWELL: bouncing threshold v_b       */
} gd_kernel;

typedef struct {
    int kind;              /* GD_FRAG_*                                        */
    double alpha;          /* power-law index (-11/6 in the paper)             */
    int n_levels;          /* number of threshold levels (>= 1)                */
    const double* levels;  /* host array, ascending.  n_levels == 1: the sharp
                              threshold levels[0] for every cell (with
                              GD_KERNEL_MAXWELL: the fragmentation threshold v_f
                              of beta_frag).  n_levels > 1: a cell with threshold
                              v uses the linear blend of the two neighbouring
                              level operators (clamped)                         */
} gd_frag_law;

typedef struct {
    double x_min, x_max;  /* mass domain                                           */
    int conservative;     /* 1: dx = -u + x_min (F(x_min)=F(x_max)=0); 0: dx = 0     */
    int quad_points;      /* Gauss points per (sub)interval; 0 -> order+1 (Sec. 3.3) */
} gd_grid;

typedef struct gd_tensor gd_tensor;
typedef struct gd_plan gd_plan;

typedef struct {
    int bins, order, P;         /* P = bins*(order+1)                               */
    int n_out;                  /* rows of the raw flux vector                        */
    int n_levels;
    long long nnz_folded;       /* structurally nonzero entries of the folded T (p<=q),
                                   summed over rows, level 0                          */
    double flops_per_eval;      /* 2 * nnz_folded: algorithmic flops per cell-eval    */
    size_t device_bytes;        /* device memory held by the tensor                   */
} gd_tensor_info_t;

/*
 * gd_init_tensor -- build the collision tensor once per kernel, fragment law,
 * grid and order (Sec. 3.3; App. B).  The raw flux vector of a cell is
 *     Y_o = sum_{p,q} T[o][p][q] g_p g_q ,
 *     Y = (F(e_1),...,F(e_{N-1}), [F(e_N) if non-conservative],
 *          V_{0,1..k}, ..., V_{N-1,1..k}),
 *     V_{j,i} = sum_theta w_theta P_i'(s_theta) F(c_j + h_j s_theta / 2),
 * with the log grid e_j = x_min (x_max/x_min)^(j/N) and Gauss-Legendre sums
 * split at every bin edge.  T is built in FP64 on the host and uploaded in the
 * layouts of both contraction precisions.  Synchronous.  *out receives a handle
 * that the caller releases with gd_free_tensor.  Limits: 2 <= bins <= 256,
 * 0 <= order <= 4, P = bins*(order+1) <= 208; GD_EINVAL otherwise.
 */
int gd_init_tensor(const gd_kernel* kernel, const gd_frag_law* frag, int bins, int order,
                   const gd_grid* grid, gd_tensor** out);
int gd_tensor_info(const gd_tensor* t, gd_tensor_info_t* info);
/* Copy level `level` of the unfolded FP64 tensor to host memory [n_out][P][P]. */
int gd_tensor_export(const gd_tensor* t, int level, double* host_out);
/* Copy the bin edges (bins+1 doubles) to host memory. */
int gd_tensor_edges(const gd_tensor* t, double* host_out);
/* Upload the device layouts of both contraction precisions now (otherwise the first
 * plan on the tensor does it).  Allocates device memory; synchronous; idempotent. */
int gd_tensor_upload(gd_tensor* t);
void gd_free_tensor(gd_tensor* t);

/*
 * gd_plan_create -- bind groups of hydro cells to tensors.  Group g has
 * cells_per_group[g] cells evaluated with tensors[g]; a tensor may serve several
 * groups.  precision is GD_PREC_*.
 *  vfrag  : host [total cells] per-cell fragmentation threshold, or NULL.  Used only
 *           for tensors built with more than one level: a cell with threshold v is
 *           evaluated with (1-theta) T_r + theta T_{r+1}, levels[r] <= v < levels[r+1],
 *           theta = (v - levels[r]) / (levels[r+1] - levels[r]) clamped to [0,1];
 *           NULL means v = levels[0].  The plan sorts cells into brackets of
 *           constant r internally; the caller's cell order is kept in every array.
 *  stream : hipStream_t (NULL = the null stream).
 * The plan allocates its own device workspace (stage states, split-state fragments,
 * raw flux buffers).  The tensors must outlive the plan.  Synchronous.
 */
int gd_plan_create(const gd_tensor* const* tensors, const int* cells_per_group, int n_groups,
                   int precision, const double* vfrag, void* stream, gd_plan** out);
/*
 * gd_plan_set_vfrag -- new per-cell fragmentation thresholds for an existing plan (a
 * hydro driver whose thresholds change from step to step keeps its plan): the cells
 * are sorted into threshold brackets again and the blend weights recomputed exactly as
 * gd_plan_create does with this vfrag (host [total cells], or NULL = levels[0]).  The
 * plan's buffers were sized at creation for any bracketing, so nothing is allocated;
 * the work items are rebuilt, captured graphs dropped.  Synchronous (waits for the
 * plan's stream first).  A non-finite value returns GD_EINVAL and leaves the plan as
 * it was.  Groups whose tensor has one level are unaffected.
 */
int gd_plan_set_vfrag(gd_plan* plan, const double* vfrag);
/* total cells and total state doubles (sum over groups of cells * P) */
int gd_plan_sizes(const gd_plan* plan, long long* n_cells, long long* n_values);
/* total bins (sum over groups of cells * bins): the length of a limiter-factor array */
int gd_plan_bins(const gd_plan* plan, long long* n_bins);
/* stored contraction fragments of a group's tensor (split-FP16 and FP64 layouts,
 * all levels) and the group's slot count (cells plus bracket padding) */
int gd_plan_schedule_stats(const gd_plan* plan, int group, long long* frags_mixed, long long* frags_fp64,
                           int* n_slots);
/* Waits for the plan's work in flight (its stream and its lanes' streams), then frees it. */
void gd_plan_destroy(gd_plan* plan);

/*
 * gd_collision_rhs -- L[g] for every cell (Eq. evo), no limiting.
 *  g       : device, state layout, read only.
 *  kscale  : device [n_cells] per-cell kernel factor, or NULL (1).
 *  rhs     : device, state layout, written.
 *  raw     : device [n_cells][n_out of the cell's group] FP64 raw flux vector Y, or NULL.
 */
int gd_collision_rhs(gd_plan* plan, const double* g, const double* kscale, double* rhs, double* raw);
/* A plan whose groups hold no cell computes nothing: gd_collision_rhs, gd_rk_step,
 * gd_rk_advance, gd_rk_forward, gd_adjoint, gd_collision_vjp, gd_advect, gd_split_step
 * and gd_plan_autotune (which reports the plan's variant) return GD_OK, with zero
 * counts, after their scalar argument checks, and accept NULL arrays then. */

/*
 * gd_collision_rhs_noalloc -- gd_collision_rhs for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses that forbid
 * hipMalloc): L[g] (Eq. evo) of n_cells cells of tensor t, level 0 of its threshold
 * table for every cell (theta = 0), with no plan.  It allocates nothing: its
 * workspace (group descriptor, work items, split operands and weights, per-cell
 * exponents, raw flux vector) lives in a 16 MiB static device array that each GPU the
 * library runs on holds until the process ends.  The caller passes inputs and outputs:
 *  t        : a tensor whose device layouts exist (gd_tensor_upload, or a plan on it);
 *             GD_EINVAL otherwise.
 *  precision: GD_PREC_FP64 or GD_PREC_MIXED_F16X3.
 *  g, kscale, rhs, raw : device, as gd_collision_rhs with n_cells cells (raw may be NULL).
 *  stream   : hipStream_t (NULL = the null stream); asynchronous.
 * Limit: the workspace of n_cells must fit in the 16 MiB.  Per cell, split FP16:
 * 64 KS + 4 P + 4 ystride + 4 bytes (KS = ceil(P/16), ystride = 32 ceil(n_out/32)),
 * i.e. 1156 B at P = 96 (about 14,000 cells) and 2564 B at P = 208 (about 6,500);
 * FP64: 8 ystride bytes (ystride = 16 ceil(n_out/16)), 768 B at P = 96.  Beyond it:
 * GD_EINVAL, nothing launched.  Every call on a GPU shares that GPU's array
 * and leaves its contents behind; calls that overlap on one GPU (several streams or
 * threads) race and must be serialised by the caller.
 */
int gd_collision_rhs_noalloc(const gd_tensor* t, int precision, int n_cells, const double* g,
                             const double* kscale, double* rhs, double* raw, void* stream);

/*
 * gd_rk_step -- n_steps of SSP-RK3 (Eq. RK3) in place on g, with the scaling
 * limiter applied to the start state and after every stage (Sec. 3.2):
 *     y1 = g + dt L(g), y2 = 3/4 g + 1/4 (y1 + dt L(y1)), g = 1/3 g + 2/3 (y2 + dt L(y2)).
 *  kscale      : device [n_cells] or NULL.
 *  dt          : time step (no CFL check is made on the device).
 *  violations  : host pointer or NULL; if non-NULL the call synchronises the
 *                stream and stores the number of bins found with a negative
 *                average by the limiter (such a bin is flattened, its mass kept),
 *                or with a non-finite coefficient; a nonzero count makes the call
 *                return GD_EPOSITIVITY (after completing every step).
 * Asynchronous otherwise, on the plan's stream; a plan with lanes (gd_plan_set_lanes)
 * steps them on their own streams and joins them to the plan's stream first.
 */
int gd_rk_step(gd_plan* plan, double* g, const double* kscale, double dt, int n_steps, long long* violations);

/*
 * Operator splitting with a hydro step (Sec. 5.2: the grain-growth step is split from
 * the evolution of the hydrodynamics).  The cells of every group of the plan form
 * one row of hydro cells of width dx, in the plan's cell order.
 *
 * gd_advect -- the transport step: every Legendre coefficient of mass bin j moves
 *   between neighbouring cells with the bin's velocity vel[j] by first-order upwind
 *   finite volumes, Courant number c_j = vel[j] dt / dx:
 *       g_c <- (1 - |c_j|) g_c + |c_j| g_up,  up = c - 1 (vel >= 0) or c + 1 (vel < 0),
 *   a convex combination of bin polynomials (positivity kept).  periodic = 1 wraps the
 *   row (the mass of every bin is kept to round-off); 0: nothing flows in at the ends
 *   and what leaves is lost.
 *    vel : host [sum over groups of bins] (groups concatenated); |vel| dt / dx <= 1
 *          for every bin, else GD_EINVAL before any launch.
 *   Synchronises the plan's stream before copying the Courant numbers; the transport
 *   itself is asynchronous.
 * gd_split_step -- n_steps of Strang splitting: transport over dt/2, one SSP-RK3
 *   collision step over dt (as gd_rk_step, start limiter included), transport over
 *   dt/2.  |vel| dt / (2 dx) <= 1.  violations as in gd_rk_step (counted over all
 *   collision steps; GD_EPOSITIVITY when given and nonzero).
 */
int gd_advect(gd_plan* plan, double* g, const double* vel, double dt, double dx, int periodic);
int gd_split_step(gd_plan* plan, double* g, const double* kscale, const double* vel, double dx, int periodic,
                  double dt, int n_steps, long long* violations);

/*
 * gd_rk_advance -- per-cell time steps under the CFL bound of Eq. dt (Sec. 3.2):
 * n_substeps sub-steps of SSP-RK3 (Eq. RK3, the limiter on the start state and
 * after every stage, as gd_rk_step), every cell with its own step, toward the
 * common end time t_end.  In each sub-step a cell c with t[c] < t_end takes
 *     dt_c = min(dt_max, t_end - t[c], cfl * B_c),
 *     B_c  = min over bins j with F(e_{j+1}) - F(e_j) > flux_floor * max_i |F(e_i)|
 *            and g_j^0 > 0 of h_j g_j^0 / (F(e_{j+1}) - F(e_j)),
 * with the fluxes of its state at the start of the sub-step (only a bin that loses
 * mass can turn negative in a forward-Euler stage; a bin with zero average cannot
 * be helped by any step).  flux_floor = 0 is the bound as printed; a positive floor
 * leaves out near-empty bins whose outflow is below that fraction of the cell's
 * largest edge flux (their positivity is left to the limiter).  With split-FP16
 * plans the fluxes carry an absolute error of ~1e-7 of the largest one, so such
 * outflows are rounding noise there: use a floor well above it (e.g. 1e-4).
 * Then t[c] = t_end if dt_c = t_end - t[c], else
 * t[c] + dt_c.  A cell with t[c] >= t_end (or a zero bound) keeps its state bit for
 * bit during the call (the start limiter aside).  The bound covers the first stage
 * of a sub-step: cfl well below 1 keeps the later stages positive too (the
 * violation count reports when it does not).
 *  g          : device, state layout, in place.
 *  kscale     : device [n_cells] or NULL.
 *  t          : device [n_cells] (caller's cell order, groups concatenated), the
 *               time each cell has reached: in/out.
 *  t_end      : finite end time; cfl > 0, dt_max > 0 and flux_floor >= 0 finite
 *               (else GD_EINVAL).
 *  violations : host pointer or NULL, as in gd_rk_step.
 *  unfinished : host pointer or NULL; if non-NULL, the number of cells with
 *               t[c] < t_end after the call.
 * Returns GD_EPOSITIVITY when violations is given and nonzero (the sub-steps are all taken).
 * Either host pointer makes the call synchronise the stream.  With graphs on
 * (gd_plan_use_graph) one sub-step (three contractions and three stage kernels) is
 * captured into a HIP graph and replayed n_substeps times; it is captured again when
 * g, kscale, t, t_end, cfl, dt_max, flux_floor or the variant change.  Off, or while
 * timing, the launches are issued one by one.  The first call on a plan allocates a
 * per-cell step array (synchronous).
 */
int gd_rk_advance(gd_plan* plan, double* g, const double* kscale, double* t, double t_end, double cfl,
                  double dt_max, double flux_floor, int n_substeps, long long* violations, long long* unfinished);

/*
 * Reverse mode (the adjoint of gd_rk_step), FP64 whatever the plan's precision.
 *
 * gd_rk_forward -- gd_rk_step (same steps, limiter placement and results) that also
 *   records what the reverse pass needs, launch by launch (no graph):
 *     states : device, (1 + 3 n_steps) states of n_values doubles: [0] the limited
 *              start state, then per step n the limited stage outputs y1, y2 and
 *              g_{n+1} at [3n+1], [3n+2], [3n+3];
 *     gammas : device, (1 + 3 n_steps) arrays of n_bins doubles (n_bins = sum over
 *              groups of cells * bins, cell-major per group): the factor the limiter
 *              applied to each bin when it wrote the state of the same index.
 *   g is overwritten with the final state, as gd_rk_step does; violations as in
 *   gd_rk_step (GD_EPOSITIVITY when given and nonzero, the record complete).
 * gd_adjoint -- the vector-Jacobian product of the whole gd_rk_forward call:
 *     lam      : device, state layout; in: dLoss/dg(final), out: dLoss/dg(input)
 *                (the caller's state before the start limiter);
 *     dkscale  : device [n_cells] or NULL: dLoss/dkscale (written);
 *     dvfrag   : device [n_cells] or NULL: dLoss/dv_frag through the blend weight of
 *                Eq. (level blend), 0 outside the level table (written);
 *   states, gammas, kscale, dt and n_steps as given to gd_rk_forward.  The steps run
 *   backwards through the stage combinations of Eq. RK3, the limiter of Eq. gamma
 *   (envelope theorem at the minimiser of the bin polynomial; a flattened bin passes
 *   nothing to its higher coefficients) and the collision operator: with the raw
 *   flux vector Y_o = sum_{p<=q} Tf[o][p][q] g_p g_q (Sec. 3.3), a cotangent nu on Y
 *   gives dg_p = sum_{q>=p} M_p[q] g_q + sum_{q<=p} M_q[p] g_q, M_p[q] = sum_o nu_o
 *   Tf[o][p][q], computed on the FP64 MFMA from a transposed copy of the tensor.
 *   The first call on a plan allocates the reverse-mode workspace (synchronous).
 * gd_collision_vjp -- one right-hand-side product: grad += (dL/dg)^T mu at state g,
 *   dkscale/dvfrag (device [n_cells] or NULL) written with d(mu . L)/dkscale and
 *   d(mu . L)/dv_frag.  mu, grad: device, state layout (mu read only).
 */
int gd_rk_forward(gd_plan* plan, double* g, const double* kscale, double dt, int n_steps, double* states,
                  double* gammas, long long* violations);
int gd_adjoint(gd_plan* plan, const double* states, const double* gammas, const double* kscale, double dt,
               int n_steps, double* lam, double* dkscale, double* dvfrag);
int gd_collision_vjp(gd_plan* plan, const double* g, const double* kscale, const double* mu, double* grad,
                     double* dkscale, double* dvfrag);

/*
 * Batching of the contraction (uneven batches of several groups in one launch).
 * Every contraction is ONE launch over all groups of the plan: a list of work items
 * (group, threshold level, a range of output row blocks, a chunk of 4 or 8 tiles of
 * cells), sorted by cost, largest first.  The stage kernels between contractions
 * are likewise one launch over all groups.
 *
 * gd_plan_set_variant -- choose the contraction variant: waves (4 or 8) per
 *   workgroup; tiles_per_wave (1, or 2 for split-FP16 plans with 4 waves and
 *   P <= 96: one A fragment read feeds two independent MFMA chains), a tile being
 *   32 cells (split FP16) or 16 cells (FP64); rows = row blocks per work item (0 =
 *   all of the group's row blocks); xcd = 1 orders the items in 8 contiguous
 *   cost-balanced ranges, one per XCD (workgroup b runs on XCD b % 8), so that the
 *   workgroups sharing an L2 stream the fragments of few iteration lists; xcd = 0
 *   orders all items largest first.  Every variant gives bit-identical results.
 *   Rebuilds the item list (synchronous).
 * gd_plan_variant -- the current variant, the number of workgroups of one
 *   contraction launch (items plus padding) and the MFMA flops one launch executes
 *   (every stored fragment, all products, for every tile of an item); any pointer
 *   may be NULL.
 * gd_plan_autotune -- time every variant on state g (device, state layout, read
 *   only; kscale as in gd_rk_step; the fastest of five samples of three contraction
 *   launches per variant) and keep the fastest (XCD-ordered items win ties
 *   within 5%: they move less than half the HBM traffic, which lanes share with the
 *   other lane's stage kernels).  On a plan of several groups, then the row
 *   blocks per work item group by group (costliest first; a group keeps another
 *   choice where the whole launch gets 1% faster).  cache_path (or NULL) names a text
 *   file of "key waves tiles_per_wave rows xcd [g:rows_0,rows_1,...]" lines (-1: the
 *   plan's rows): a plan of the same shape (precision,
 *   bins, order, levels, cells, brackets and stored fragments of every group) on
 *   the same device (architecture and compute units) takes its stored choice
 *   without timing; a newly timed choice is appended.  Synchronous.
 * gd_plan_use_graph -- (default on) gd_rk_step captures one RK step (three
 *   contractions and three stage kernels) into a HIP graph on a private stream and
 *   replays it once per step on the plan's stream.  The graph is captured again
 *   when g, kscale, dt or the variant change.  Off: the launches are issued one by
 *   one.  Timing (gd_plan_timing) also issues them one by one.
 */
int gd_plan_set_variant(gd_plan* plan, int waves, int tiles_per_wave, int rows, int xcd);
/* gd_plan_group_rows -- the row blocks per work item of every group (rows[n_groups];
 * the autotuner may set them group by group, gd_plan_set_variant resets them to rows). */
int gd_plan_group_rows(const gd_plan* plan, int* rows);
int gd_plan_variant(const gd_plan* plan, int* waves, int* tiles_per_wave, int* rows, int* xcd, int* n_items,
                    double* exec_flops);
/*
 * gd_plan_algorithmic_flops -- the flops one right-hand-side evaluation of every
 * cell of the plan must do, whatever the precision or blocking: per cell
 * 2 nnz of the folded tensor of its threshold level (Sec. 3.3), plus 2 nnz of the
 * difference to the next level for a cell between two levels (the blend of the
 * level tensors).  Host value into *flops.
 */
int gd_plan_algorithmic_flops(const gd_plan* plan, double* flops);
int gd_plan_autotune(gd_plan* plan, const double* g, const double* kscale, const char* cache_path, int* waves,
                     int* tiles_per_wave, int* rows, int* xcd);
int gd_plan_use_graph(gd_plan* plan, int enable);
/*
 * gd_plan_set_lanes -- split the cells of the plan into `lanes` lanes (contiguous
 * ranges of 32-slot tiles of equal contraction cost) for gd_rk_step, gd_rk_advance
 * and gd_collision_rhs: every lane takes all the call's steps or sub-steps (or its
 * evaluation) on a stream of its own (lane 0 on the plan's stream, the others on
 * private streams forked from it and joined back to it before the call returns), so
 * that the kernels of one lane fill the tail of another lane's contraction and its
 * memory-bound stage kernels overlap the other's contractions.  Cells are
 * independent (Eq. evo acts cell by cell), so the results are bit for bit those of
 * one lane.  lanes: 0 = by size (two once the plan has 1024 tiles of 32 slots or
 * more, else one), 1..8.  Plans with fewer tiles than lanes take one lane per tile.
 * The adjoint calls run one lane; while timing (gd_plan_timing) every call does.
 * Synchronous (waits for the plan's work in flight); drops the captured graphs.
 * gd_plan_lanes -- the lanes in use, and (first_tiles, if given, room for 8) the
 * first tile of each.
 */
/*
 * gd_plan_checks -- the device checks of the checked build (libgracedg_checks.so,
 * compiled with -DGD_CHECKS): before using them, the kernels test the work items,
 * iteration descriptors, fragment and iteration ranges and slot -> cell indices
 * against the sizes of the plan's groups, skip the work on a failure (the results
 * are then incomplete) and set a bit of the plan's check word; the stage kernel also
 * flags non-finite new states.  *flags receives the word (GD_CHECK_* bits) of the
 * calls since the last read, which clears it; synchronous.  The regular build
 * returns GD_EUNSUPPORTED with *flags = 0.
 */
#define GD_CHECK_ITEM 1u        /* a work item outside its group's levels, row blocks or tiles */
#define GD_CHECK_DESC 2u        /* an iteration list or descriptor outside the schedule */
#define GD_CHECK_SLOT 4u        /* a slot mapped to a cell outside its group */
#define GD_CHECK_NONFINITE 8u   /* a stage produced a non-finite coefficient */
int gd_plan_checks(gd_plan* plan, unsigned* flags);
int gd_plan_set_lanes(gd_plan* plan, int lanes);
int gd_plan_lanes(const gd_plan* plan, int* lanes, int* first_tiles);

/*
 * gd_projection_points / gd_project -- initial coefficients (Sec. 3.2, Eq. init):
 *     g_j^i = (2i+1)/2 sum_a w_a g0(c_j + h_j s_a / 2) P_i(s_a)
 * with a 16-point Gauss-Legendre rule per bin.  gd_projection_points writes the
 * sample masses to host memory [bins][16]; the caller evaluates its profile g0 there
 * for every cell and passes the device array samples [n_cells][bins][16]; coef
 * [n_cells][P] (device) receives the coefficients.  Synchronous on stream.
 */
int gd_projection_points(const gd_tensor* t, double* host_x);
int gd_project(const gd_tensor* t, int n_cells, const double* samples, double* coef, void* stream);

/*
 * gd_plan_timing / gd_plan_contraction_time / gd_plan_stage_time -- measurement
 * support.  While timing is enabled the plan records a HIP event pair on its stream
 * around every contraction launch and every stage-kernel launch (limiter, flux
 * assembly, RK combination and state split), and issues the RK step launch by
 * launch instead of as a graph.  The _time calls synchronise the stream, return the
 * summed event time (ms) and the number of launches of that kernel since timing was
 * enabled or last read, and reset that count.
 */
int gd_plan_timing(gd_plan* plan, int enable);
int gd_plan_contraction_time(gd_plan* plan, double* total_ms, int* launches);
int gd_plan_stage_time(gd_plan* plan, double* total_ms, int* launches);

const char* gd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GRACEDG_H */
