/* sem.h -- C ABI of the MI355X spectral-element operator library (libsem.so).
 *
 * The library evaluates the matrix-free Poisson/Helmholtz stiffness operator of
 * a spectral-element solver on lx^3 Gauss-Lobatto-Legendre (GLL) hexahedra
 * (arXiv 2506.20994, Sec. 3 and Sec. 4.2, Listing 2), the gather-scatter sum
 * that assembles it (Sec. 2.1), and the set-up and solver steps around them.
 *
 * Conventions shared by every entry point
 *  - Element-local fields are [nel][lx][lx][lx] with i fastest (the index order
 *    of Listing 2), contiguous, no padding.  "n_local" = nel * lx^3.
 *  - Pointers named "device" must point to device memory of the GPU that was
 *    current when the context was created; the caller owns them and the library
 *    never frees them.  Pointers named "host" are ordinary host memory.
 *  - Calls that take a context run asynchronously on the context's stream
 *    unless documented as synchronous.  No call allocates device memory except
 *    sem_create and the *_setup / *_create calls.
 *  - Every call returns a status: SEM_OK (0), a positive informational code, or
 *    a negative error code.  On error nothing has been launched and
 *    sem_last_error() returns a message.
 *  - lx must be in [2, 12] (SEM_EUNSUPPORTED_LX otherwise).
 */
#ifndef SEM_H
#define SEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sem_ctx_s* sem_ctx_t;
typedef struct sem_gs_s* sem_gs_t;
typedef struct sem_cg_s* sem_cg_t;
typedef struct sem_lp_s* sem_lp_t;
typedef struct sem_mg_s* sem_mg_t;

typedef enum { SEM_F64 = 0, SEM_F32 = 1, SEM_BF16 = 2 } sem_dtype_t;

enum {
    SEM_OK = 0,
    SEM_NOT_CONVERGED = 1,   /* solver stopped at maxit; results are valid but not converged */
    SEM_FELL_BACK = 2,       /* learned preconditioner was abandoned for Jacobi */
    SEM_EINVAL = -1,         /* bad argument (null pointer, size, alias, dtype) */
    SEM_EUNSUPPORTED_LX = -2,
    SEM_EHIP = -3,           /* a HIP runtime call failed */
    SEM_EBREAKDOWN = -4,     /* solver breakdown: non-finite or non-positive curvature */
    SEM_ENOMEM = -5,
    SEM_EGEOMETRY = -6       /* folded mesh: det J <= 0 somewhere */
};

#define SEM_LX_MIN 2
#define SEM_LX_MAX 12

/* ---------------------------------------------------------------- context */

/* Create a context on the current HIP device.  `hip_stream` is a hipStream_t
 * (NULL = the null stream) that the context borrows; it is not destroyed by
 * sem_destroy.  Allocates a small device workspace (reduction partials).
 * Plans, solvers and networks made from a context must be destroyed before
 * the context. */
int sem_create(sem_ctx_t* ctx, void* hip_stream);
int sem_destroy(sem_ctx_t ctx);
/* Switch the stream later calls are launched on (borrowed, as above). */
int sem_set_stream(sem_ctx_t ctx, void* hip_stream);
/* Message for the last error on this context (ctx = NULL: last error of a call
 * that had no valid context).  Never NULL. */
const char* sem_last_error(sem_ctx_t ctx);
/* Block the host until all work queued on the context's stream is done. */
int sem_sync(sem_ctx_t ctx);

/* ----------------------------------------------------------------- set-up */

/* GLL nodes xi[0..lx), weights w[0..lx) and the derivative matrix of the
 * Lagrange basis (Sec. 3, Eq. 2-3), written in the layout of the operator's
 * argument list (Listing 1/2):  dx[l*lx + i] = l_l'(xi_i) (the factor that
 * multiplies u_l in the r-derivative at node i) and dxt[l*lx + i] = dx[i*lx + l].
 * All outputs are host arrays; any of them may be NULL.  Synchronous, needs no
 * context or GPU. */
int sem_gll(int lx, double* xi, double* w, double* dx, double* dxt);

/* Periodic box of n^3 elements on the unit cube with the cyclic sine
 * deformation x = X + amp sin(2 pi Y) sin(2 pi Z) (y, z cyclically), where X is
 * the position of the node on the undeformed uniform grid.  Elements are
 * numbered e = ex + n (ey + n ez).  Writes node coordinates x, y, z (device
 * float64, n_local each) and global node ids (device int64, n_local), the id
 * being the node's position on the periodic (n (lx-1))^3 lattice.  Any output
 * may be NULL. */
int sem_box_mesh(sem_ctx_t ctx, int n, int lx, double amp,
                 double* x, double* y, double* z, int64_t* ids);

/* The same box and deformation without the periodic identification, with
 * homogeneous Dirichlet conditions on the whole boundary (u = 0 on the six
 * faces of the undeformed cube; a case the paper's Poisson setting (Sec. 3)
 * leaves to the solver around the operator).  Boundary nodes get id -1 (no
 * unknown); interior nodes get their position on the (M - 1)^3 lattice of
 * interior points, M = n (lx - 1):
 * id = ((K - 1) (M - 1) + (J - 1)) (M - 1) + (I - 1), I = ex (lx - 1) + i etc.
 * Outputs and rules as in sem_box_mesh. */
int sem_box_mesh_dirichlet(sem_ctx_t ctx, int n, int lx, double amp,
                           double* x, double* y, double* z, int64_t* ids);

/* Geometric factors of the operator from node coordinates (isoparametric:
 * the GLL derivative matrix applied to x, y, z gives the Jacobian).  With
 * 1 = r, 2 = s, 3 = t and W = w_i w_j w_k |J|:
 *   g_ab = W sum_c (dr_a/dx_c)(dr_b/dx_c),   bm = W (diagonal mass).
 * All arrays device float64 of n_local.  bm may be NULL.  The call is
 * synchronous: it returns SEM_EGEOMETRY when det J <= 0 at some node; if
 * `min_detj` (host) is non-NULL it receives the minimum det J. */
int sem_geometry(sem_ctx_t ctx, const double* x, const double* y, const double* z,
                 int64_t nel, int lx,
                 double* g11, double* g22, double* g33,
                 double* g12, double* g13, double* g23, double* bm,
                 double* min_detj);

/* out_local[L] = in_unique[ids[L]] for L < n_local (the scatter Q; any dtype,
 * in and out of the same dtype).  ids device int64 in [0, n_unique), or
 * negative for a Dirichlet node, which receives 0. */
int sem_scatter(sem_ctx_t ctx, void* out_local, const void* in_unique,
                const int64_t* ids, int64_t n_local, sem_dtype_t dtype);

/* Element-local diagonal of the operator (before gather-scatter):
 *   d = sum_l D_li^2 V11(l,j,k) + sum_l D_lj^2 V22(i,l,k) + sum_l D_lk^2 V33(i,j,l)
 *     + 2 D_ii D_jj V12 + 2 D_ii D_kk V13 + 2 D_jj D_kk V23,   V_ab = h1 g_ab,
 * with D_il = dx[l*lx + i].  h1 may be NULL (h1 = 1).  Device float64. */
int sem_ax_diag(sem_ctx_t ctx, double* d, const double* dx, const double* h1,
                const double* g11, const double* g22, const double* g33,
                const double* g12, const double* g13, const double* g23,
                int64_t nel, int lx);

/* f[L] = scale[L] * sum_m amp[m] cos(2 pi (k[m].x_L) + phase[m]) for a sum of
 * nmodes <= 64 Fourier modes (k host int64 [nmodes][3], amp and phase host
 * float64).  scale may be NULL (1).  Device float64 in/out. */
int sem_fourier(sem_ctx_t ctx, double* f, const double* x, const double* y,
                const double* z, const double* scale, int64_t n_local,
                const int64_t* k, const double* amp, const double* phase, int nmodes);

/* Element-wise precision conversion dst = src, round-to-nearest-even; float64
 * to bfloat16 rounds through float32.  Device arrays of n entries. */
int sem_convert(sem_ctx_t ctx, void* dst, sem_dtype_t dst_dtype,
                const void* src, sem_dtype_t src_dtype, int64_t n);

/* ---------------------------------------------------------------- operator */

/* w = A_e u on every element (Sec. 4.2, Listing 2; argument order of
 * Listing 1, with nel and lx passed by value):
 *   ur = sum_l dx[l,i] u[k,j,l],  us = sum_l dy[l,j] u[k,l,i],
 *   ut = sum_l dz[l,k] u[l,j,i]
 *   [vr vs vt] = h1 * [[g11 g12 g13] [g12 g22 g23] [g13 g23 g33]] [ur us ut]
 *   w[k,j,i] = sum_l dxt[l,i] vr[k,j,l] + dyt[l,j] vs[k,l,i] + dzt[l,k] vt[l,j,i]
 * field_dtype is the storage type of u, h1 and g.. (SEM_F64, SEM_F32 or
 * SEM_BF16); the six lx*lx matrices are float64 for SEM_F64 and float32
 * otherwise; arithmetic is float64 for SEM_F64 and float32 (accumulation
 * included) otherwise.  out_dtype is SEM_F64 (only with field_dtype SEM_F64)
 * or SEM_F32.  h1 may be NULL (h1 = 1).  w must not overlap any input.
 * All pointers device.  Asynchronous. */
int sem_ax(sem_ctx_t ctx, void* w, const void* u,
           const void* dx, const void* dy, const void* dz,
           const void* dxt, const void* dyt, const void* dzt,
           const void* h1, const void* g11, const void* g22, const void* g33,
           const void* g12, const void* g13, const void* g23,
           int64_t nel, int lx, sem_dtype_t field_dtype, sem_dtype_t out_dtype);

/* Helmholtz form of the operator: w = A_e u + h2b .* u on every element, the
 * stiffness of sem_ax plus the diagonal mass term h2 B u of the velocity
 * (Helmholtz) solves.  The paper's routine bears that name (ax_helm, Listing
 * 1) while its arithmetic (Listing 2) carries only the h1 stiffness; this is
 * the adjacent step.  h2b = h2 * bm per local node (bm: the diagonal mass of
 * sem_geometry; h2: the Helmholtz coefficient), stored in field_dtype like u;
 * it must not be NULL.  Every other argument, type and rule as in sem_ax; the
 * extra stream makes it 80 B per local node in float64. */
int sem_ax_helmholtz(sem_ctx_t ctx, void* w, const void* u,
                     const void* dx, const void* dy, const void* dz,
                     const void* dxt, const void* dyt, const void* dzt,
                     const void* h1, const void* g11, const void* g22, const void* g33,
                     const void* g12, const void* g13, const void* g23, const void* h2b,
                     int64_t nel, int lx, sem_dtype_t field_dtype, sem_dtype_t out_dtype);

/* Kernel variants of the float64 operator (sem_ax and sem_ax_helmholtz with
 * field dtype SEM_F64), all computing the same sums (results agree to
 * rounding):
 *   SEM_AX_COLUMN     one thread per (i, j) column, u's column in registers,
 *                     the element's slices and fluxes in LDS (Sec. 4.2, the
 *                     per-(i, j) thread mapping with a k loop);
 *   SEM_AX_COLUMN_PF  the same with the opposite choice of fetching the next
 *                     slice's factors one slice ahead;
 *   SEM_AX_SLICE      the column mapping with the element passing through LDS
 *                     one slice at a time (double-buffered, one barrier per
 *                     slice; 6 lx^2 LDS values per element instead of ~3 lx^3);
 *   SEM_AX_3D         one thread per node (lx <= 10);
 *   SEM_AX_WAVE       the column mapping with each element's lx^2 columns on
 *                     16, 32 or 64 lanes of one wave (lx = 3, 5, 6, 7), so an
 *                     element never spans two waves and needs no workgroup
 *                     barrier (as the column mapping has at lx = 2, 4, 8).
 * SEM_AX_DEFAULT (-1) is the built-in choice: SEM_AX_COLUMN.  The paper picks among kernel variants by timing them at run
 * time (Sec. 4); sem_ax_tune does that for one lx and element count. */
enum { SEM_AX_DEFAULT = -1, SEM_AX_COLUMN = 0, SEM_AX_COLUMN_PF = 1, SEM_AX_SLICE = 2, SEM_AX_3D = 3,
       SEM_AX_WAVE = 4 };
#define SEM_AX_VARIANTS 5
/* Select the variant for lx on this context (SEM_EINVAL if it does not
 * exist at that lx). */
int sem_ax_set_variant(sem_ctx_t ctx, int lx, int variant);
int sem_ax_get_variant(sem_ctx_t ctx, int lx, int* variant);
/* Time every variant that exists at lx on nel elements of synthetic inputs
 * (allocated and freed here; `reps` launches each after two warm-ups, HIP
 * events on the context's stream; two rounds over the variants, each
 * variant's faster round kept, so that the clock ramp of an idle GPU does not
 * penalise the variant timed first), select the fastest for lx on this
 * context and return it in *best.  us (host, SEM_AX_VARIANTS entries, may be
 * NULL) receives the average launch time of each variant in microseconds, -1
 * where a variant does not exist.  Synchronous. */
int sem_ax_tune(sem_ctx_t ctx, int lx, int64_t nel, int reps, double* us, int* best);
/* The same timing on the caller's own float64 operands (the arguments of
 * sem_ax, h1 may be NULL; w is overwritten, no allocation), as the paper's
 * autotuning times the variants on the call it serves (Sec. 4).  SEM_EINVAL
 * for null arrays or an output that overlaps an input. */
int sem_ax_tune_on(sem_ctx_t ctx, void* w, const void* u, const void* dx, const void* dy, const void* dz,
                   const void* dxt, const void* dyt, const void* dzt, const void* h1, const void* g11,
                   const void* g22, const void* g33, const void* g12, const void* g13, const void* g23,
                   int64_t nel, int lx, int reps, double* us, int* best);

/* ---------------------------------------------------------- gather-scatter */

/* Build the gather-scatter plan (Sec. 2.1) for a local numbering: ids (host
 * int64, n_local entries) names the global node of each local node.  A
 * negative id marks a Dirichlet node (homogeneous Dirichlet condition): it is
 * no unknown, sem_gs sets it to 0, its multiplicity is 1 and its owner weight
 * 0, and the solver keeps it at 0.  Nodes whose (non-negative) id occurs once
 * are left alone by sem_gs.  The plan lives on the context's device until
 * sem_gs_destroy.  Synchronous.  n_local must be < 2^31. */
int sem_gs_setup(sem_ctx_t ctx, const int64_t* ids, int64_t n_local, sem_gs_t* gs);
int sem_gs_destroy(sem_gs_t gs);
/* Number of distinct non-negative ids, and of ids that occur more than once
 * (host outs). */
int sem_gs_info(sem_gs_t gs, int64_t* n_unique, int64_t* n_shared);
/* Number of local nodes with a negative id (Dirichlet nodes; host out). */
int sem_gs_dirichlet_count(sem_gs_t gs, int64_t* n_dirichlet);
/* In place u <- Q Q^T u: each local copy of a node receives the sum over all
 * copies, added in a fixed order (deterministic); Dirichlet nodes receive 0.
 * dtype SEM_F64 or SEM_F32 (float32 fields are summed in float32).  Device
 * array of n_local. */
int sem_gs(sem_gs_t gs, void* u, sem_dtype_t dtype);
/* mult[L] = number of local copies of node L's id, 1 on Dirichlet nodes
 * (device float64). */
int sem_gs_mult(sem_gs_t gs, double* mult);

/* Owner weights for dot products of continuous fields: wgt[L] = 1 for the
 * first local copy (lowest local index) of each id and 0 for the others and
 * for Dirichlet nodes, so sum_L wgt_L u_L v_L = u_G . v_G for u = Q u_G,
 * v = Q v_G (device float64). */
int sem_gs_owner(sem_gs_t gs, double* wgt);
/* In place x <- x - mean_G(x) for a continuous field: the mean over unique
 * nodes (owner-weighted sum / number of distinct ids) is subtracted from every
 * local node, making sum_G x_G = 0 (the solvability condition of the periodic
 * Poisson problem).  Device float64, n_local.  Asynchronous.  A plan with
 * Dirichlet nodes has no such null space: SEM_EINVAL. */
int sem_remove_mean(sem_gs_t gs, double* x);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * operation as sem_remove_mean, same arguments, rules and result, with its
 * reduction partials in a fixed file-scope device array of the library
 * (8194 float64 slots, 64 KiB per GPU, held until the process ends) instead of
 * the context's workspace.  It calls no hipMalloc, hipFree or other allocating
 * routine; the first call on a device looks up that device's copy of the
 * array (hipGetSymbolAddress).  A plan whose reduction would need more than
 * the array's partial slots is refused with SEM_EINVAL (never the case for
 * plans sem_gs_setup accepts: the reduction grid is capped at 8192 blocks).
 * Every call on one GPU shares that GPU's array: calls that overlap in time on
 * one GPU (different streams or host threads) race and give wrong means; calls
 * serialised on one stream are safe.  Asynchronous. */
int sem_remove_mean_static(sem_gs_t gs, double* x);

/* ------------------------------------------------------------------ solver */

/* The assembled Poisson operator A_G = sum_e Q_e^T A_e Q_e in the local
 * layout: y = gs(Ax(x)).  Float64 device arrays, the layout of sem_ax; h1 may
 * be NULL (h1 = 1, the Poisson case).  With h2b non-NULL the operator is the
 * Helmholtz form of sem_ax_helmholtz, A_e + diag(h2b) on every element
 * (h2b = h2 * bm per local node, h2 > 0: the velocity-type solves), whose
 * assembled matrix is positive definite. */
typedef struct {
    const double* dx; const double* dy; const double* dz;
    const double* dxt; const double* dyt; const double* dzt;
    const double* h1;
    const double* g11; const double* g22; const double* g33;
    const double* g12; const double* g13; const double* g23;
    int64_t nel;
    int lx;
    const double* h2b;
} sem_operator_t;

typedef enum {
    SEM_SOLVE_F64 = 0,      /* float64 Jacobi-PCG throughout */
    SEM_SOLVE_F32_IR = 1,   /* float64 refinement around float32 inner PCG */
    SEM_SOLVE_BF16_IR = 2   /* as F32_IR, inner operator with bfloat16 h1 and G */
} sem_solve_precision_t;

typedef struct {
    double tol;          /* stop at ||b - A x||_2 <= tol ||b||_2 over unique dofs (e.g. 1e-10) */
    int maxit;           /* limit on operator applications of the outer float64 loop
                            (F64) or on inner iterations summed over all outer steps (IR) */
    int precision;       /* sem_solve_precision_t */
    double inner_tol;    /* IR: inner relative residual target (0: 1e-6 F32, 1e-2 BF16) */
    int inner_maxit;     /* IR: iterations per inner solve (0: 500) */
    int max_outer;       /* IR: outer refinement steps (0: 60) */
    int check_every;     /* iterations between host convergence checks (0: 16; 4 with mg) */
    sem_lp_t learned;    /* NULL: Jacobi-PCG.  Otherwise flexible CG (Notay's FCG(1))
                            preconditioned by this network, bound to the same operator
                            (sem_lp_bind), with the Jacobi fallback described below */
    int ir_mode;         /* IR modes: 0 restarted refinement (each outer step runs a fresh
                            inner PCG on r / ||r||), 1 residual replacement ("reliable
                            updates"): one reduced-precision Krylov iteration whose
                            residual is replaced by the float64 b - A x, and whose
                            accumulated update is added to the float64 x, each time its
                            residual has fallen by the factor `delta`; the search
                            direction is kept */
    double delta;        /* ir_mode 1: replacement trigger (0: 0.1; 1e-3 with mg) */
    sem_mg_t mg;         /* NULL: none.  Otherwise flexible CG preconditioned by this
                            multigrid V-cycle (sem_mg_create on the same operator and
                            plan); not together with `learned` */
} sem_solve_opts_t;

typedef struct {
    int iterations;      /* operator applications in the Krylov loops (all levels) */
    int outer;           /* IR refinement steps (0 for F64) */
    double relres;       /* final ||b - A x||_2 / ||b||_2, recomputed in float64 */
    double relres_hist[64]; /* relres after each outer step (IR) */
    int converged;       /* 1 if relres <= tol */
    int breakdown;       /* 1 if a Krylov loop met a non-positive or non-finite curvature */
    int jacobi_steps;    /* learned: iterations whose network output was replaced by Jacobi */
    int fell_back;       /* learned: 1 if the solve switched to Jacobi for good */
} sem_solve_stats_t;

/* Create a solver for A on the plan gs: allocates the work vectors, the
 * assembled Jacobi diagonal (sem_ax_diag + sem_gs), and for the IR modes the
 * reduced-precision copies of h1, G and D.  `opts` fixes the precision mode.
 * Synchronous.  The operator arrays must stay valid while the solver lives. */
int sem_cg_setup(sem_ctx_t ctx, sem_gs_t gs, const sem_operator_t* A,
                 const sem_solve_opts_t* opts, sem_cg_t* cg);
int sem_cg_destroy(sem_cg_t cg);

/* Solve A x = b (Jacobi-preconditioned CG; Hestenes-Stiefel; Saad Alg. 9.1),
 * or float64 iterative refinement around reduced-precision inner PCG solves.
 * With opts->learned set, every Krylov loop is flexible CG with one stored
 * direction (Notay 2000): z = P(r) is the network's output; an iteration whose
 * z is non-finite or has r.z <= 0 uses the Jacobi z instead, and a solve whose
 * relative residual has not halved over 256 iterations switches to Jacobi for
 * good (stats->fell_back, return SEM_FELL_BACK when it then converges).
 * b: device float64, local layout, continuous (b = Q b_G) with sum_G b_G = 0
 * (the periodic operator's null space is the constants).  x: device float64
 * output, local layout, continuous, with sum_G x_G = 0.  Starts from x = 0.
 * On a plan with Dirichlet nodes the operator is the assembled one restricted
 * to the free nodes (their rows and columns only), which has no null space:
 * b needs no projection (its Dirichlet entries are ignored), no mean is
 * removed, and x is 0 on the Dirichlet nodes.  The same holds without
 * projection for the Helmholtz operator (A->h2b set at sem_cg_setup); the
 * Jacobi diagonal then includes h2b.  A plan without free nodes is
 * refused by sem_cg_setup (SEM_EINVAL).
 * Returns SEM_OK, SEM_NOT_CONVERGED (limit reached; x is the last iterate) or
 * SEM_EBREAKDOWN.  Synchronous (reads convergence flags every check_every
 * iterations). */
int sem_cg_solve(sem_cg_t cg, double* x, const double* b, const sem_solve_opts_t* opts,
                 sem_solve_stats_t* stats);

/* ------------------------------------------------ multigrid preconditioner */

/* A multigrid V-cycle for the operators of the box meshes (sem_box_mesh and
 * sem_box_mesh_dirichlet): the preconditioner whose iteration count does not
 * grow with the mesh, for the Poisson (and Helmholtz) solve the operator
 * serves (Sec. 3).  Levels: the caller's operator (n^3 elements, lx), then
 * lx -> max(2, lx / 2) on the same elements down to lx = 2 (p-coarsening),
 * then the lx = 2 box n^3 -> (n/2)^3 while n is even and n/2 >= n_coarse
 * (h-coarsening).  Each level below the first is re-discretised by the
 * library's set-up calls on the same deformed box (h1 = 1; h2 times that
 * level's mass for Helmholtz operators); a level whose geometry would fold
 * (det J <= 0 at a node: coarse trilinear elements of a strongly deformed box)
 * takes the amplitude halved until it does not (or, with opts->galerkin, every
 * lx = 2 level below the first is P^T A P of the level above).  Transfer: the coarse level's field
 * evaluated at the fine level's nodes (the coarse Lagrange basis on the same
 * element; the parent's trilinear basis); restriction by its transpose.
 * Smoothing: `degree` steps of the Chebyshev semi-iteration in D^-1 A (D the
 * assembled diagonal) on [lo lmax, hi lmax] (defaults 2, 0.15, 1.1: the fastest
 * 32^3 lx = 8 solve of a sweep over degree 1-4 and lo 0.15-0.3), lmax of every level estimated by
 * `lanczos_steps` Lanczos steps at creation.  The coarsest level is solved
 * with a dense inverse (at most 2048 unknowns; of A + c 1 1^T on the singular
 * periodic box, c = mean diagonal / unknowns).  V(b): pre-smoothing from 0,
 * coarse correction of the residual, post-smoothing: a fixed symmetric positive
 * definite map.  Vectors and operators of the V-cycle are float32. */
typedef struct {
    int n;               /* elements per side of the box the operator lives on */
    double amp;          /* the box's deformation amplitude (sem_box_mesh) */
    int dirichlet;       /* 1: the Dirichlet box (its plan has Dirichlet nodes), 0: periodic */
    double h2;           /* Helmholtz coefficient (> 0 exactly when A->h2b is set; 0: Poisson) */
    int degree;          /* Chebyshev steps per smoothing (0: 2) */
    double lo, hi;       /* smoothing interval in units of lmax (0: 0.15 and 1.1) */
    int n_coarse;        /* h-coarsening keeps n >= n_coarse (0: 2) */
    int lanczos_steps;   /* Lanczos steps per level for lmax (0: 20) */
    int fine_bf16;       /* 1: the finest level's smoothing operator stores its factors (and
                            h2 B) in bfloat16, as SEM_SOLVE_BF16_IR does (half the bytes of
                            its four applications per V-cycle); 0: float32 */
    int galerkin;        /* 1: every lx = 2 level below the first is the Galerkin product
                            P^T A P of the level above (float64 set-up from the float64
                            operators, kept as one dense 8 x 8 float32 matrix per element;
                            no geometry of its own, amplitude reported 0), instead of a
                            re-discretised box: the coarse correction stays an A-orthogonal
                            projection where coarse boxes of a strongly deformed mesh fold;
                            0: re-discretised */
} sem_mg_opts_t;

/* Build the hierarchy for the operator A (h1 must be NULL) on the plan gs of
 * the n^3 box: allocates every level's factors, plans and work vectors, and
 * estimates each lmax.  Synchronous.  SEM_EINVAL if the sizes do not match
 * n^3 elements, the plan's Dirichlet nodes do not match opts->dirichlet, or
 * the coarsest level would exceed 2048 unknowns (choose n_coarse).  The
 * operator arrays must stay valid while the hierarchy lives. */
int sem_mg_create(sem_ctx_t ctx, sem_gs_t gs, const sem_operator_t* A, const sem_mg_opts_t* opts,
                  sem_mg_t* mg);
int sem_mg_destroy(sem_mg_t mg);
/* Number of levels (host out). */
int sem_mg_levels(sem_mg_t mg, int* count);
/* Level `level` (0 = the caller's): elements per side, lx, unknowns, the
 * estimated lmax of D^-1 A (0 on the coarsest level) and the deformation
 * amplitude of the level's box.  Any out may be NULL. */
int sem_mg_level_info(sem_mg_t mg, int level, int* n, int* lx, int64_t* n_unique, double* lmax,
                      double* amp);
/* Replace the lmax of a smoothed level (every level but the coarsest). */
int sem_mg_set_lmax(sem_mg_t mg, int level, double lmax);
/* Launch mode of the V-cycle (default off): replay it as a HIP graph captured
 * on first use for each set of (z, r) pointers (the V-cycle's pointers and
 * the sequence of its launches are fixed), or launch its kernels one by one
 * (off).  Both give the same result bit for bit.  Graphs are kept until
 * sem_mg_destroy; a graph captured for pointers whose memory is later freed
 * is never replayed unless the same pointers are passed again. */
int sem_mg_set_graphs(sem_mg_t mg, int on);
/* z = V(r) on unique-node vectors of the finest plan (the layout of
 * sem_lp_apply_unique); dtype SEM_F64 or SEM_F32 for both; z must not alias r.
 * Asynchronous; the hierarchy's work vectors are shared by all calls on mg. */
int sem_mg_apply(sem_mg_t mg, void* z, const void* r, sem_dtype_t dtype);

/* --------------------------------------------- learned preconditioner */

/* A per-element network for elements of n = lx^3 nodes (lx even, 4..12; the
 * workload's network is lx = 8, n = 512): inputs are the element's residual
 * r_e / s_e (n values, s_e = ||r_e||_2) and six geometric features
 * mean(h1 g_ab) / kappa_e (kappa_e = mean(h1 (g11 + g22 + g33)) / 3); layers
 * Linear(n + 6, 256)-ReLU-Linear(256, 256)-ReLU-Linear(256, n).  Applied as
 *   z = Q Q^T (mult^-1 (s_e / kappa_e) NN(x_e)).
 * Training minimises the mean squared error against t_e = err_e kappa_e / s_e
 * with Adam.  Products run on bf16 MFMA with float32 accumulation; weights,
 * moments, loss and bias gradients are float32.
 * Parameter slots for sem_lp_set/get: 0 W1 (256 x (n + 6), row-major, out x
 * in), 1 b1 (256), 2 W2 (256 x 256), 3 b2, 4 W3 (n x 256), 5 b3 (n); add 6 for
 * Adam's first moments, 12 for the second moments, 18 for the gradients.
 * Feature rows (sem_lp_samples, sem_lp_forward, sem_lp_gradients) are n + 6
 * values zero padded to a multiple of 16 (528 at lx = 8); target and output
 * rows are n wide.  The sizes below are those of lx = 8. */
#define SEM_LP_IN 518
#define SEM_LP_IN_PAD 528      /* row width of feature matrices (zero padded) */
#define SEM_LP_HIDDEN 256
#define SEM_LP_OUT 512

/* Allocate a network for lx = 8 elements with zero weights and workspace for
 * up to max_rows rows (elements per inference, or batch rows per training
 * step). */
int sem_lp_create(sem_ctx_t ctx, int64_t max_rows, sem_lp_t* lp);
/* The same for elements of lx^3 nodes, lx even in [4, 12] (SEM_EUNSUPPORTED_LX
 * otherwise), with hidden layers of width `hidden` (a multiple of 16 in
 * [16, 1024]; 0: 256, the workload's).  The linear form's block then has rank
 * at most `hidden`.  At lx = 8 the linear form's product runs in a
 * weight-stationary kernel written for 512 x 512 blocks; at other lx in the
 * general MFMA product.  Slot sizes follow: W1 hidden x (n + 6), W2 hidden x
 * hidden, W3 n x hidden. */
int sem_lp_create_lx(sem_ctx_t ctx, int lx, int hidden, int64_t max_rows, sem_lp_t* lp);
/* The element size lx and hidden width (may be NULL) the network was created for. */
int sem_lp_lx(sem_lp_t lp, int* lx, int* hidden);
int sem_lp_destroy(sem_lp_t lp);
/* Copy `count` float32 values (host) into / out of slot `which`; count must
 * equal the slot's size.  Synchronous. */
int sem_lp_set(sem_lp_t lp, int which, const float* host, int64_t count);
int sem_lp_get(sem_lp_t lp, int which, float* host, int64_t count);
/* Adam's step counter (the number of updates taken). */
int sem_lp_set_step(sem_lp_t lp, int64_t step);
int sem_lp_get_step(sem_lp_t lp, int64_t* step);
/* Checkpoint of the network: its form (linear, Jacobi base), training metric,
 * Adam step, parameters and Adam moments, to a binary file ("SEMLP001",
 * version 1, little-endian: int32 version, linear, jacobi_base; double mu;
 * int64 step; then for each of slots 0..17 an int64 count and that many
 * float32 values).  sem_lp_load reads and checks the whole file before it
 * changes anything (SEM_EINVAL for a missing, truncated or foreign file);
 * loading then equals sem_lp_set_linear / _set_jacobi_base / _set_metric /
 * sem_lp_set of slots 0..17 / sem_lp_set_step, so training resumes bitwise
 * and the Jacobi base takes effect at the next sem_lp_bind.  Synchronous. */
int sem_lp_save(sem_lp_t lp, const char* path);
int sem_lp_load(sem_lp_t lp, const char* path);
/* Training loss.  mu < 0: mean squared error (the default).  mu >= 0: the
 * batch mean of (y - t)^T K (y - t) with K = A_ref + mu B_ref, where A_ref is
 * the stiffness matrix of the undeformed reference element [-1, 1]^3 divided
 * by its kappa (mean of w_i w_j w_k) and B_ref = diag(w_i w_j w_k) / kappa:
 * the energy norm CG minimises, plus a mass term that fixes the element-wise
 * constant.  K is held in bfloat16. */
int sem_lp_set_metric(sem_lp_t lp, double mu);
/* Linear form (on != 0): identity activations, biases unused (their
 * gradients are zero), geometric inputs zeroed.  The network output is then
 * W x with W = W3 W2 W1 (the first n input columns), and inference applies
 * the symmetric additive preconditioner
 *     z = sum_e Q_e S_e W_s S_e Q_e^T r / kappa_e  (+ Minv r with the Jacobi base),
 * W_s = (W + W^T) / 2 held in bfloat16, S_e = diag(mult^-1/2) on the element's
 * nodes, kappa_e the element's stiffness scale: a fixed symmetric map of r, so
 * CG's conjugacy holds.  Trained with the energy-norm loss
 * (sem_lp_set_metric) on white-noise residual/error pairs it approximates
 * the element block of the inverse operator.  Applies to training and
 * inference from the next call on. */
int sem_lp_set_linear(sem_lp_t lp, int on);
/* Set the linear form's n x n element block directly (host float32,
 * row-major, count = n * n) instead of folding it from the weights: the
 * preconditioner becomes z = sum_e Q_e S_e W_s S_e Q_e^T r / kappa_e (+ Minv r
 * with the Jacobi base), W_s the symmetric part of W, applied by the same
 * kernels.  For classical (non-learned) element blocks used as a comparison.
 * Switches the network to its linear form; the block holds until the weights
 * change (sem_lp_set, a training step or sem_lp_load), which folds them
 * again. */
int sem_lp_set_block(sem_lp_t lp, const float* W, int64_t count);
/* The kernel of the linear form's product on unique-node vectors (the
 * solver's apply): 0 automatic (the weight-stationary kernel at lx = 8, the
 * general MFMA product otherwise), 1 the weight-stationary kernel (lx = 8
 * only, SEM_EINVAL otherwise), 2 the general product, whose epilogue scales by
 * 1/kappa_e and scatters to CSR order.  Both compute the same sums. */
int sem_lp_set_product(sem_lp_t lp, int kind);
/* Jacobi base (on != 0): the preconditioner becomes z = Minv r + P_net(r),
 * Minv the inverse assembled diagonal of the bound operator, and training
 * targets become (err - Minv r) kappa / s, so the network learns the
 * correction to Jacobi (a network that outputs zero is exactly Jacobi).
 * Takes effect at the next sem_lp_bind. */
int sem_lp_set_jacobi_base(sem_lp_t lp, int on);
/* Bind to an operator (the network's lx, nel <= max_rows) and its plan: computes the
 * per-element geometric features and keeps the operator's arrays for
 * sem_lp_snapshot (they must stay valid while bound).  Needed by sem_lp_samples / sem_lp_apply.
 * Only the stiffness is read (A->h2b is ignored): with a Helmholtz solve the
 * Jacobi base uses the stiffness diagonal. */
int sem_lp_bind(sem_lp_t lp, const sem_operator_t* A, sem_gs_t gs);
/* Training rows for `count` elements elems[] (device int64) of the bound
 * operator: X[row0 + q] = inputs (bf16, the padded feature width) from the residual
 * r, and, if T != NULL, T[row0 + q] = err_e kappa_e / s_e (float32, n wide)
 * from the error err.  r, err: device float64 fields of the bound operator. */
int sem_lp_samples(sem_lp_t lp, const double* r, const double* err, const int64_t* elems,
                   int64_t count, uint16_t* X, float* T, int64_t row0);
/* One snapshot of a solve A x_k = b with reference solution xstar on the
 * bound operator: forms the residual r = b - Q Q^T A x_k and the error
 * err = xstar - x_k (float64, into the caller's work arrays r_out and err_out,
 * n_local each, which must not alias the inputs), then writes the training
 * rows of sem_lp_samples for the `count` elements elems[].  x, xstar, b:
 * device float64 continuous fields of the bound operator.  The bound
 * operator's arrays must still be valid.  Asynchronous. */
int sem_lp_snapshot(sem_lp_t lp, const double* x, const double* xstar, const double* b,
                    double* r_out, double* err_out, const int64_t* elems, int64_t count,
                    uint16_t* X, float* T, int64_t row0);
/* The classical element block the learned one is compared with: kappa times
 * the inverse of the assembled operator restricted to the lx^3 nodes of one
 * element (the local solve of one-level additive Schwarz with minimal
 * overlap), on the undeformed periodic 3^3 box, where every element has the
 * same matrix; kappa = mean(g11 + g22 + g33) / 3 of that element.  The
 * columns come from the library's operator and gather-scatter applied to unit
 * vectors; the (lx^3)^2 matrix is symmetrised and inverted by Cholesky on the
 * host.  W: host float64, (lx^3)^2, row-major.  Allocates and frees
 * temporary device memory; synchronous.  Pass it (rounded to float32) to
 * sem_lp_set_block of a network of the same lx. */
int sem_lp_reference_block(sem_ctx_t ctx, int lx, double* W);
/* Y = NN(X) for `rows` rows (X device bf16 rows x the padded feature width, Y device
 * float32 rows x n). */
int sem_lp_forward(sem_lp_t lp, const uint16_t* X, int64_t rows, float* Y);
/* Gradients of the batch MSE into the gradient slots; *loss (host) receives
 * the loss.  X, T device, B rows (B % 8 == 0). */
int sem_lp_gradients(sem_lp_t lp, const uint16_t* X, const float* T, int64_t B, float* loss);
/* One Adam step from the gradient slots (increments the step counter). */
int sem_lp_adam(sem_lp_t lp, double lr, double beta1, double beta2, double eps);
/* Gather rows[0..B) of (X, T) (device), gradients, Adam (beta 0.9/0.999,
 * eps 1e-8).  *loss is a device float32 that receives the batch loss.
 * Asynchronous. */
int sem_lp_train_step(sem_lp_t lp, const uint16_t* X, const float* T, const int64_t* rows,
                      int64_t B, double lr, float* loss);
/* z = P(r) on the bound operator; dtype SEM_F64 or SEM_F32 for both.
 * z and r are continuous fields in the local layout (nel * n values). */
int sem_lp_apply(sem_lp_t lp, void* z, const void* r, sem_dtype_t dtype);
/* The same on unique-node vectors of the bound plan (sem_gs_info's n_unique
 * values, the layout sem_cg_solve iterates in): unique nodes are numbered in
 * the order in which their global ids first appear in the local layout
 * (Dirichlet nodes excluded).  The linear form runs a gather kernel (S r to
 * bfloat16), the weight-stationary bf16 MFMA product (CSR-ordered output) and
 * an assembly pass.  Asynchronous; the network's workspace is shared with the
 * other calls on lp, so calls on one lp must not overlap. */
int sem_lp_apply_unique(sem_lp_t lp, void* z, const void* r, sem_dtype_t dtype);

#ifdef __cplusplus
}
#endif

#endif /* SEM_H */
