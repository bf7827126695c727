/*
 * moto.h -- C ABI of the MI355X (gfx950) bilayer minimum-mode kernel.
 *
 * Method: Xu & Delin, "A general optimization framework for mapping local
 * transition-state networks" (arXiv 2509.26269).  The library implements the
 * data-parallel hot path of its bilayer minimum-mode-following (MMF) kernel
 * for atomistic spin systems:
 *   - energy and gradient of the spin Hamiltonian (Methods, Eq.
 *     param-hamiltonian; Methods, "Gradient, HVP, and Hessian");
 *   - the tangent-space Hessian-vector product (Methods, "HVP operator mode");
 *   - the inner layer: k smallest eigenpairs of the (masked) tangent Hessian
 *     by block LOBPCG from HVPs only (Results, "Bilayer MMF"; Knyazev 2001);
 *   - the outer layer: reflected force F_mmf = F - 2 (F.v) v and a rotation
 *     step of every spin (Results, "Bilayer MMF" equation; Supplementary
 *     Note 1, Algorithm 1, bilayer-kernel loop);
 *   - certification lambda_1 < 0 < lambda_2 and the two-sided +-min-mode
 *     descent (Results, "Deterministic bidirectional saddle descent";
 *     Supplementary Note 1, item iii).
 *
 * CONVENTIONS (every entry point)
 *   Lattice: periodic rhombic Lx x Ly triangular lattice, a1 = (1,0),
 *     a2 = (1/2, sqrt3/2), nearest-neighbour distance 1, site s = x + Lx*y,
 *     N = Lx*Ly.  Shell s = all lattice offsets at the s-th smallest distance.
 *   Energy: E = -sum_i sum_delta J_delta m_i.m_{i+delta}
 *               - sum_i sum_{delta in NN} D_delta.(m_i x m_{i+delta})
 *               - sum_i B.m_i - K sum_i m_iz^2,
 *     sums over ORDERED pairs (every bond counted twice, as the i != j sums
 *     of the paper read literally), mu_i = 1, D_delta = D[s] (z x dhat).
 *   Spins and ambient vectors: SoA, m = [3][N] (all mx, then my, then mz).
 *   Tangent frame layout: a tangent vector v_i is stored as two coordinates
 *     (v_i.e1_i, v_i.e2_i) in the orthonormal tangent basis of Duff et al.,
 *     "Building an Orthonormal Basis, Revisited" (JCGT 2017) built from m_i:
 *       s = copysign(1, m_z); a = -1/(s + m_z); b = m_x m_y a;
 *       e1 = (1 + s m_x^2 a, s b, -s m_x);  e2 = (b, s + m_y^2 a, -m_y),
 *     computed in the precision of the call; V = [n][2][N].
 *   Tangent (Riemannian) Hessian on the product of unit spheres:
 *       (H v)_i = P_i (A v)_i - c_i v_i,  P_i = I - m_i m_i^T,  c_i = m_i.g_i,
 *     A the constant Euclidean Hessian, g = A m - B the Euclidean gradient.
 *   Mask: uint8 per site, nonzero = active; NULL = all active.  The masked
 *     operator is the principal submatrix on the active sites, M H M.
 *   Batches: `batch` independent lattices of the plan's size stored back to
 *     back (m = [batch][3][N], V = [batch][n][2|3][N], c = [batch][N], ...).
 *
 * OWNERSHIP AND ERRORS
 *   Every array argument is a DEVICE pointer owned by the caller unless
 *   marked "host".  No call keeps a pointer after it returns and no call
 *   allocates device memory: scratch comes from a caller workspace whose size
 *   the matching *_workspace function returns.  Calls are ordered on the
 *   given stream (NULL = default stream).  moto_energy_grad,
 *   moto_tangent_hvp, moto_hessian_apply and moto_reflected_step do not
 *   synchronise; the iterative drivers (moto_min_modes, moto_descend,
 *   moto_saddle_search, moto_saddle_search_batched) synchronise with the
 *   stream at their convergence checks and report through host structs,
 *   except moto_min_modes and moto_descend with the MOTO_ASYNC flag, which
 *   queue every iteration up to the cap, report to device memory and can be
 *   captured into a HIP graph.
 *   Return value: MOTO_OK or a negative error detected before any launch
 *   (outputs untouched) or from the HIP runtime (MOTO_EHIP).  A plan holds
 *   pinned host memory for convergence read-back: use one plan from one host
 *   thread at a time.
 *
 * GPU SCOPE: up to MOTO_MAX_SHELLS exchange shells (the shells of the
 * triangular lattice by increasing distance, 6, 12, 18 or 24 bonds each; the
 * paper's Pd/Fe/Ir(111) parameters, Supplementary Note 4, use 35) and DMI on
 * the nearest-neighbour shell (D[1..] must be 0); other Hamiltonians return
 * MOTO_EUNSUPPORTED.  Up to 3 shells the lattice kernels are specialised
 * (row march, register rings); beyond, a general-shell tile kernel stages a
 * halo of up to 12 rows and sums the shells from LDS.  With more than 3
 * shells, moto_hessian_apply, moto_param_mixed, moto_param_grad_apply and
 * the batched search return MOTO_EUNSUPPORTED, and energy partials carry E
 * only (no parameter derivatives).
 */
#ifndef MOTO_H
#define MOTO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t moto_status;

/* host return codes */
#define MOTO_OK 0
#define MOTO_EINVAL (-1)
#define MOTO_EHIP (-2)
#define MOTO_EWORKSPACE (-4)
#define MOTO_EUNSUPPORTED (-6)

/* outcome codes reported in the result structs (device-detected) */
#define MOTO_SADDLE 0        /* certified index-1 saddle (lambda_1 < -tau < tau < lambda_2) */
#define MOTO_CONVERGED 0     /* eigen-solve: all k residuals below tolerance */
#define MOTO_NOT_CONVERGED 1 /* iteration cap reached (or an unconverged certifying solve) */
#define MOTO_DEGENERATE 2    /* |lambda_1| or |lambda_2| within tau of zero */
#define MOTO_HIGHER_INDEX 3  /* lambda_2 < -tau */
#define MOTO_NAN 4           /* non-finite value met */
#define MOTO_BREAKDOWN 5     /* LOBPCG basis lost rank below the block size */

typedef enum { MOTO_F32 = 0, MOTO_F64 = 1 } moto_dtype;
typedef enum { MOTO_AMBIENT = 0, MOTO_FRAME = 1 } moto_layout;

#define MOTO_MAX_SHELLS 36

/* Spin Hamiltonian (Methods, Eq. param-hamiltonian), reduced units. */
typedef struct {
    int32_t Lx, Ly;            /* lattice size, >= 1 each                   */
    int32_t n_shells;          /* exchange shells in use, 1..MOTO_MAX_SHELLS */
    int32_t reserved;          /* must be 0                                 */
    double J[MOTO_MAX_SHELLS]; /* exchange per shell (J > 0 ferromagnetic)  */
    double D[MOTO_MAX_SHELLS]; /* DMI magnitude per shell, D_delta = D (z x dhat) */
    double K;                  /* uniaxial anisotropy along e_z             */
    double B[3];               /* Zeeman field (mu_i = 1)                   */
} moto_hamiltonian;

typedef struct moto_plan_s *moto_plan;
typedef void *moto_stream; /* a hipStream_t */

/* Plan: validated Hamiltonian, stencil coefficients, pinned read-back
 * buffer.  Immutable after creation.  Returns MOTO_EINVAL for bad sizes,
 * MOTO_EUNSUPPORTED outside the GPU scope above. */
moto_status moto_plan_create(const moto_hamiltonian *h /* host */, moto_plan *out /* host */);
moto_status moto_plan_destroy(moto_plan p);
const char *moto_status_string(moto_status s);
/* Rigorous bound on ||H||: 4 sum_delta (|J_delta| + |D_delta|) + 4|K| + |B|;
 * all relative tolerances below are multiples of it. */
double moto_hessian_norm_bound(moto_plan p);
/* Replays of the eigen-solvers' captured iteration graphs made with this plan
 * so far (diagnostic: 0 means every chunk ran as plain launches). */
int64_t moto_plan_graph_replays(moto_plan p);
/* Number of Hamiltonian parameters theta = (J_0..J_{ns-1}, D_0..D_{ns-1}, K, Bx, By, Bz). */
int32_t moto_n_params(moto_plan p);

/* ---------------------------------------------------------------------
 * Energy and gradient (Methods, Eq. param-hamiltonian; "Gradient, HVP,
 * and Hessian").  FP64 or FP32 spins (dt); reductions always in FP64,
 * deterministic (fixed order).
 *   m        [batch][3][N] unit spins, dtype dt
 *   mask     [batch][N] or NULL; zeroes F on inactive sites only
 *   E        [batch] FP64 energies (or NULL)
 *   grad     [batch][3][N] Euclidean gradient g = dE/dm, dtype dt (or NULL)
 *   c        [batch][N] c_i = m_i.g_i, dtype dt (or NULL)
 *   F        [batch][3][N] force F_i = -(I - m_i m_i^T) g_i, dtype dt (or NULL)
 *   dE_dtheta [batch][n_params] FP64 partials of E with respect to theta (or NULL)
 * Workspace: moto_energy_grad_workspace(p, batch) bytes. */
size_t moto_energy_grad_workspace(moto_plan p, int32_t batch);
moto_status moto_energy_grad(moto_plan p, moto_dtype dt, int32_t batch, const void *m,
                             const uint8_t *mask, double *E, void *grad, void *c, void *F,
                             double *dE_dtheta, void *ws, size_t ws_bytes, moto_stream stream);

/* Allocation-free variant of moto_energy_grad, for callers that cannot
 * allocate or pass a workspace: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  Same arguments, outputs and
 * results (bit for bit) as moto_energy_grad, minus the workspace: its
 * per-tile partial sums go to a static device array of
 * MOTO_NOALLOC_SCRATCH_BYTES that every GPU the library runs on holds until
 * the process ends (its address is looked up on the first call on each
 * device).  Calls that need more, moto_energy_grad_workspace(p, batch) >
 * MOTO_NOALLOC_SCRATCH_BYTES (about 95 000 tiles of 32 x 8 sites: e.g. 1024
 * lattices of 128 x 128, or one of 2048 x 2048), return MOTO_EWORKSPACE
 * before any launch.  No device or host memory is allocated.  All calls on
 * one GPU share that array: calls that overlap in time on one GPU (two
 * streams, two host threads) race and must be ordered by the caller.
 * Nothing needs clearing between calls (every partial is written before it
 * is read). */
#define MOTO_NOALLOC_SCRATCH_BYTES ((size_t)8 << 20)
moto_status moto_energy_grad_noalloc(moto_plan p, moto_dtype dt, int32_t batch, const void *m,
                                     const uint8_t *mask, double *E, void *grad, void *c, void *F,
                                     double *dE_dtheta, moto_stream stream);

/* ---------------------------------------------------------------------
 * Tangent Hessian-vector product, the operator of the inner layer (Methods,
 * "HVP operator mode"): W_j = M H(m) M V_j for n_vec vectors per lattice.
 *   m     [batch][3][N] unit spins, dtype dt
 *   c     [batch][N] Weingarten scalars c_i = m_i.g_i (from moto_energy_grad)
 *   V, W  frame layout [batch][n_vec][2][N], ambient [batch][n_vec][3][N]
 *         (ambient inputs must be tangent); W must not alias V.
 * No workspace.  Does not synchronise. */
moto_status moto_tangent_hvp(moto_plan p, moto_dtype dt, moto_layout layout, int32_t batch,
                             const void *m, const void *c, const uint8_t *mask, int32_t n_vec,
                             const void *V, void *W, moto_stream stream);

/* Autotuner of the frame-layout HVP (tile shape / staging variant): times
 * every variant `reps` times on the caller's buffers (W is overwritten),
 * remembers the fastest in the plan for this (dt, batch, n_vec) -- later
 * moto_tangent_hvp and moto_min_modes calls with that key use it -- and
 * returns its index in *chosen.  times_ms (host, may be NULL) receives
 * moto_tangent_hvp_variants() entries, -1 for variants not applicable to dt.
 * Synchronises with the stream. */
int32_t moto_tangent_hvp_variants(void);
const char *moto_tangent_hvp_variant_name(int32_t variant);
/* Pin a variant for (dt, batch, n_vec) without timing (MOTO_EINVAL if the
 * variant does not exist for dt). */
moto_status moto_plan_set_hvp_variant(moto_plan p, moto_dtype dt, int32_t batch, int32_t n_vec, int32_t variant);
moto_status moto_tangent_hvp_autotune(moto_plan p, moto_dtype dt, int32_t batch, const void *m, const void *c,
                                      const uint8_t *mask, int32_t n_vec, const void *V, void *W, int32_t reps,
                                      int32_t *chosen /* host */, float *times_ms /* host */,
                                      moto_stream stream);

/* Euclidean Hessian (constant) applied to ambient vectors: W_j = A V_j,
 * [batch][n_vec][3][N] (the double-backward of the energy). */
moto_status moto_hessian_apply(moto_plan p, moto_dtype dt, int32_t batch, int32_t n_vec,
                               const void *V, void *W, moto_stream stream);

/* Mixed second derivatives for the double backward: out[b][q] =
 * d(g(m_b) . U_b)/d theta_q, FP64, deterministic.  U ambient [batch][3][N].
 * Workspace: moto_energy_grad_workspace(p, batch). */
moto_status moto_param_mixed(moto_plan p, moto_dtype dt, int32_t batch, const void *m,
                             const void *U, double *out, void *ws, size_t ws_bytes,
                             moto_stream stream);

/* Adjoint of the parameter partials, for the double backward:
 * out[b] = sum_q w[b][q] d g(m_b) / d theta_q  (g is linear in theta), i.e.
 * J_s: -2 sum_{delta in s} m_{i+delta};  D_s: 2 sum_{delta in s} (z x dhat) x m_{i+delta};
 * K: -2 m_iz z;  B: -1.  w FP64 [batch][n_params]; out [batch][3][N] dtype dt. */
moto_status moto_param_grad_apply(moto_plan p, moto_dtype dt, int32_t batch, const void *m, const double *w,
                                  void *out, moto_stream stream);

/* ---------------------------------------------------------------------
 * Inner layer: k smallest eigenpairs of the masked tangent Hessian at m by
 * block LOBPCG (Knyazev 2001) with HVPs only, Rayleigh-Ritz on [X W P] in
 * FP64 (SVQB orthonormalisation, Stathopoulos & Wu 2002, then a Householder-QL eigen-solve), block
 * width k + guard.  HVP and blocks in `hvp` precision; Gram, Rayleigh-Ritz
 * and the returned vectors in FP64.
 * Stopping rule: ||H v_j - lambda_j v_j||_2 <= tol * moto_hessian_norm_bound
 * for all j < k, or max_iter iterations (Results: iteration cap 200).
 *   m      [3][N] FP64 unit spins (batch 1)
 *   evals  [k] FP64 ascending
 *   V      [k][3][N] FP64 ambient unit tangent vectors; input warm start when
 *          opts.warm == 1; output sign rule: the entry of largest magnitude
 *          (first in [3][N] order) is positive
 *   resid  [k] FP64 residual norms (or NULL)
 *   info   host (device with MOTO_ASYNC): outcome (MOTO_CONVERGED /
 *          NOT_CONVERGED / NAN / BREAKDOWN), iterations, HVP columns applied
 *          (or NULL).  NaN or infinite spins end the solve at once with NAN.
 * opts.warm == 2 reuses the full block left in ws by the previous call on
 * the same workspace (transported to the new tangent spaces).
 * Workspace: moto_min_modes_workspace(p, hvp, k, guard) bytes. */
typedef struct {
    double tol;          /* relative residual tolerance (default 1e-5 F32, 1e-10 F64) */
    int32_t max_iter;    /* default 200 */
    int32_t guard;       /* extra block vectors; <0 = 2 for k <= 2, 2k for k = 3, 4, else max(4, ceil(k/2)), at most 16 - k */
    int32_t warm;        /* 0 random start, 1 V holds k start vectors, 2 reuse block */
    int32_t check_every; /* iterations between host convergence checks (default 8) */
    uint64_t seed;       /* start-block seed (SplitMix64 counter generator) */
    int32_t use_graph;   /* 1: replay the iteration chunk as a captured HIP graph (default) */
    int32_t flags;       /* 0 (default) or MOTO_ASYNC */
} moto_eig_opts;

/* MOTO_ASYNC (moto_eig_opts.flags of moto_min_modes and
 * moto_min_modes_population; moto_descend_opts.flags of moto_descend): the
 * call does no host synchronisation and writes its outcome to DEVICE memory
 * (moto_info / moto_descend_result pointers are then device pointers, or
 * NULL).  Every iteration up to the cap is queued: the kernels of iterations
 * after convergence return at once (the device done flag), so the results
 * equal those of the synchronous call bit for bit.  The call is then
 * stream-ordered and may be captured into a HIP graph by the caller (no
 * allocation, no memset node, no host read-back); when the stream is being
 * captured the library queues plain launches instead of replaying its own
 * iteration graph. */
#define MOTO_ASYNC 1

typedef struct {
    int32_t status;
    int32_t iters;
    int64_t n_hvp;
} moto_info;

size_t moto_min_modes_workspace(moto_plan p, moto_dtype hvp, int32_t k, int32_t guard);
moto_status moto_min_modes(moto_plan p, moto_dtype hvp, const double *m, const uint8_t *mask,
                           int32_t k, const moto_eig_opts *opts /* host */, double *evals,
                           double *V, double *resid, moto_info *info /* host */, void *ws,
                           size_t ws_bytes, moto_stream stream);

/* ---------------------------------------------------------------------
 * Inner layer over a population (Methods, multi-objective explorer: the
 * spectral-gap objective needs the two lowest modes of every candidate of
 * a population; Results: population size 24): P independent block-LOBPCG
 * solves, exactly the method of moto_min_modes, on P states of the plan's
 * lattice, run in lock step -- every kernel launch covers the whole
 * population and the dense per-member steps run side by side, so P solves
 * take about the time of one.  Each member stops by its own test; the call
 * returns once all have stopped.
 *   P      1 <= P <= MOTO_MAX_POPULATION
 *   m      [P][3][N] FP64 device, unit spins
 *   mask   [P][N] device (1 = active) or NULL
 *   evals  [P][k] FP64 device;  V [P][k][3][N] FP64 device (input warm
 *          starts when opts.warm == 1);  resid [P][k] FP64 device or NULL
 *   info   host [P] or NULL: outcome of every member
 * Errors: MOTO_EINVAL for P or k out of range; MOTO_EWORKSPACE when ws_bytes
 * is below moto_min_modes_population_workspace(p, hvp, P, k, guard). */
#define MOTO_MAX_POPULATION 256
size_t moto_min_modes_population_workspace(moto_plan p, moto_dtype hvp, int32_t P, int32_t k,
                                           int32_t guard);
moto_status moto_min_modes_population(moto_plan p, moto_dtype hvp, int32_t P, const double *m,
                                      const uint8_t *mask, int32_t k,
                                      const moto_eig_opts *opts /* host */, double *evals, double *V,
                                      double *resid, moto_info *info /* host */, void *ws,
                                      size_t ws_bytes, moto_stream stream);

/* ---------------------------------------------------------------------
 * Outer layer, one step (Results, "Bilayer MMF"; Algorithm 1 bilayer loop):
 *   F_mmf = F - 2 sum_{r < k_reflect} (F.v_r) v_r;   G = -F_mmf;
 *   direction d from L-BFGS on G (memory `mem`, stored pairs transported by
 *   projection onto the current tangent spaces, pairs with s.y <= sy_min
 *   skipped, initial scaling s.y/y.y of the newest valid pair or alpha0,
 *   reset to d = -alpha0 G whenever d.G >= 0), the fixed step d = -alpha0 G,
 *   or nonlinear conjugate gradients (the paper's second outer optimiser:
 *   d = alpha0 p, p = -G + beta P p_prev with the Fletcher-Reeves beta =
 *   |G|^2 / |P G_prev|^2, beta = 0 every 50 steps and whenever p.G >= 0);
 *   d scaled so that max_i |d_i| <= theta_max; each spin rotated by d_i
 *   (m_i <- cos|d_i| m_i + sin|d_i| d_i/|d_i|, renormalised).
 * If ||F_mmf||_2 <= tau_F the step is not taken and the stop flag is set.
 * k_reflect = 0 gives the plain downhill step of the descent.
 *   m      [3][N] FP64, updated in place
 *   F      [3][N] FP64 tangent force at m (moto_energy_grad)
 *   V      [k_reflect][3][N] FP64 unit min modes (NULL if k_reflect = 0)
 *   state  optimiser state, moto_step_state_bytes(p, mem) bytes, zeroed by
 *          the caller before the first step of a run
 *   out    [2] FP64 device: out[0] = ||F_mmf||_2 at m, out[1] = 1 if stopped */
typedef struct {
    int32_t rule;      /* 0 = L-BFGS, 1 = fixed step, 2 = conjugate gradients */
    int32_t mem;       /* L-BFGS memory, 1..16 (default 8) */
    double theta_max;  /* rotation cap, rad (default 0.1) */
    double alpha0;     /* initial / fixed step; <= 0 means 1 / moto_hessian_norm_bound */
    double sy_min;     /* curvature-pair threshold (default 1e-12) */
    double tau_F;      /* stop threshold on ||F_mmf||_2 */
} moto_step_opts;

size_t moto_step_state_bytes(moto_plan p, int32_t mem);
moto_status moto_reflected_step(moto_plan p, double *m, const double *F, const double *V,
                                int32_t k_reflect, const moto_step_opts *opts /* host */,
                                void *state, double *out, moto_stream stream);

/* ---------------------------------------------------------------------
 * Two-sided descent, one side (Supplementary Note 1, item iii): rotate the
 * saddle m by sign*eta*v1/max_i|v1_i| (largest spin rotation eta), then relax
 * with the step rule on F (k_reflect = 0) until ||F||_2 <= tau_F or
 * max_iter steps; finally one k = 1 eigen-solve at the minimum.
 *   m   [3][N] FP64: saddle in, relaxed state out
 *   v1  [3][N] FP64 unit min mode at the saddle
 *   res host (device with MOTO_ASYNC): energy, topological charge
 *       (Berg-Luescher), ||F||, lambda_1. */
typedef struct {
    double eta;          /* default 0.1 rad */
    double tau_F;        /* default 1e-6 */
    int32_t max_iter;    /* default 5000 */
    int32_t check_every; /* steps between host checks (default 16) */
    moto_step_opts step;
    moto_eig_opts eig;   /* final lambda_1 solve */
    int32_t flags;       /* 0 (default) or MOTO_ASYNC (res is then a device pointer) */
    int32_t reserved;
} moto_descend_opts;

typedef struct {
    int32_t converged;
    int32_t iters;
    double E;
    double Q;
    double fnorm;
    double lambda1;
} moto_descend_result;

size_t moto_descend_workspace(moto_plan p, moto_dtype hvp, const moto_descend_opts *o);
moto_status moto_descend(moto_plan p, moto_dtype hvp, double *m, const double *v1, int32_t sign,
                         const moto_descend_opts *opts /* host */,
                         moto_descend_result *res /* host */, void *ws, size_t ws_bytes,
                         moto_stream stream);

/* ---------------------------------------------------------------------
 * Second inner solver: the k smallest eigenpairs of the (masked) tangent
 * Hessian by thick-restart band Lanczos with full reorthogonalisation
 * (Results, "Bilayer MMF": HVP-Lanczos as the alternative Krylov solver;
 * Discussion: Krylov depth and reorthogonalisation are the solver's
 * hyperparameters).  The Krylov space grows from a block of `block`
 * orthonormal start vectors (Ruhe's band Lanczos): step j applies one HVP to
 * basis vector j and orthogonalises the image against the whole basis twice
 * (classical Gram-Schmidt, FP64 coefficients).  After m_max steps one
 * wavefront diagonalises the projected matrix in FP64 and the solve either
 * stops (every residual norm |T[m..m+b)[0..m) y_i|, i < k, at most tol *
 * moto_hessian_norm_bound) or restarts from the `keep` lowest Ritz vectors
 * and the residual block.  A single start vector (block = 1) may leave the
 * second member of a close eigenvalue pair out of the space after the first
 * has met the stopping rule, and holds one direction per exactly degenerate
 * eigenspace; a block of b vectors brings up to b such directions in
 * together.  A breakdown (a new Krylov vector of negligible norm) ends the
 * cycle; the solve never reports CONVERGED with fewer than k Ritz pairs, and
 * the restart replaces the dependent direction by a fresh random one.  Same
 * arguments, outputs, stopping rule and sign rule as moto_min_modes;
 * info->iters counts restarts; MOTO_BREAKDOWN if the start block has no
 * independent direction.  The cycles after the first are replayed as a HIP
 * graph.
 *   m_max   Krylov depth, 3 <= m_max <= 64 and m_max + block <= 2N
 *   keep    Ritz vectors kept at a restart, k <= keep <= m_max - block
 *           (0: max(k + 2, m_max / 2))
 *   block   start-block size b, 1..4 (0: 2)
 *   warm    1: the first start vector is the sum of the k vectors in V
 *           (ambient FP64), the others random
 * k <= 16.  Errors: MOTO_EINVAL for out-of-range sizes or options,
 * MOTO_EWORKSPACE if ws is NULL or short, MOTO_EHIP on a runtime error.
 * Workspace: moto_min_modes_lanczos_workspace(p, hvp, m_max) bytes. */
typedef struct {
    double tol;           /* relative to the norm bound (default 1e-10 F64, 1e-5 F32) */
    int32_t m_max;        /* default 32 */
    int32_t keep;         /* default 0 = max(k + 2, m_max / 2) */
    int32_t max_restarts; /* default 200 */
    int32_t warm;         /* default 0 */
    uint64_t seed;        /* start block when not warm */
    int32_t use_graph;    /* default 1 */
    int32_t block;        /* start-block size, default 0 = 2 */
} moto_lanczos_opts;

void moto_default_lanczos_opts(moto_dtype hvp, moto_lanczos_opts *o);
size_t moto_min_modes_lanczos_workspace(moto_plan p, moto_dtype hvp, int32_t m_max);
moto_status moto_min_modes_lanczos(moto_plan p, moto_dtype hvp, const double *m, const uint8_t *mask, int32_t k,
                                   const moto_lanczos_opts *opts /* host */, double *evals, double *V,
                                   double *resid, moto_info *info /* host */, void *ws, size_t ws_bytes,
                                   moto_stream stream);

/* ---------------------------------------------------------------------
 * Driver of the five calls: one saddle search (Algorithm 1, bilayer-kernel
 * loop).  Repeat {energy_grad; min_modes(k, warm-started); reflected_step}
 * until ||F_mmf||_2 <= tau_F, then certify with a k_cert >= 2 solve:
 * MOTO_SADDLE if lambda_1 < -tau_lam and lambda_2 > tau_lam, else
 * MOTO_HIGHER_INDEX / MOTO_DEGENERATE; MOTO_NOT_CONVERGED after max_outer,
 * and also when the certifying solve itself stops unconverged (its Ritz
 * values only bound the eigenvalues from above, so they cannot exclude a
 * second negative mode).
 *   m    [3][N] FP64: start in, final point out
 *   evals_out [k_cert] FP64 device (or NULL), V_out [k_cert][3][N] FP64 device (or NULL) */
typedef struct {
    double tau_F;        /* default 1e-6 */
    double tau_lam;      /* <= 0: 1e-6 (F64) or 1e-4 (F32) times the norm bound */
    int32_t k;           /* modes during the climb (default 1) */
    int32_t k_cert;      /* modes for certification (default 2) */
    int32_t k_reflect;   /* reflected modes (default 1) */
    int32_t max_outer;   /* default 5000 */
    moto_step_opts step;
    moto_eig_opts eig;
} moto_search_opts;

typedef struct {
    int32_t status;
    int32_t iters;
    int64_t n_hvp;
    double E;
    double fnorm;
    double lambda1, lambda2;
} moto_search_result;

size_t moto_saddle_search_workspace(moto_plan p, moto_dtype hvp, const moto_search_opts *o);
moto_status moto_saddle_search(moto_plan p, moto_dtype hvp, double *m, const uint8_t *mask,
                               const moto_search_opts *opts /* host */,
                               moto_search_result *res /* host */, double *evals_out,
                               double *V_out, void *ws, size_t ws_bytes, moto_stream stream);

/* ---------------------------------------------------------------------
 * Searches over a population: P saddle searches on states of the plan's
 * lattice (same method, options and results as moto_saddle_search) run in
 * lock step: every outer iteration is one batched energy/gradient launch,
 * one population eigen-solve (moto_min_modes_population, warm-started) and
 * one reflected step per member still climbing; a member stops by its own
 * test and is left in place while the others go on.  This is the form for
 * many starts of one size (an explorer's Pareto front, Results): all steps
 * of all members share each launch, where the persistent batched kernel
 * below gives each search one workgroup.
 *   m      [P][3][N] FP64 device: starts in, final points out
 *   mask   [P][N] device or NULL
 *   res    host [P] results
 *   evals_out [P][k_cert] FP64 device or NULL; V_out [P][k_cert][3][N] or NULL
 * The call synchronises with the stream at every outer iteration.
 * Errors: MOTO_EINVAL (P outside 1..MOTO_MAX_POPULATION, bad options),
 * MOTO_EWORKSPACE below moto_saddle_search_population_workspace(p, hvp, P, opts). */
size_t moto_saddle_search_population_workspace(moto_plan p, moto_dtype hvp, int32_t P,
                                               const moto_search_opts *o);
moto_status moto_saddle_search_population(moto_plan p, moto_dtype hvp, int32_t P, double *m,
                                          const uint8_t *mask, const moto_search_opts *opts /* host */,
                                          moto_search_result *res /* host */, double *evals_out,
                                          double *V_out, void *ws, size_t ws_bytes, moto_stream stream);

/* ---------------------------------------------------------------------
 * Batching form: n independent saddle searches on periodic square lattices
 * of uneven sides L[b] (5 <= L <= 4096) in ONE persistent launch, one
 * workgroup per search (largest lattices first), FP32 HVP with FP64 state.
 * Same method as moto_saddle_search (k <= 2 climb modes, k_reflect = 1,
 * L-BFGS rule, certification with k = 2); every search runs to its own
 * stopping rule, so uneven convergence costs no host round trips.
 *   h      host: Hamiltonian (Lx, Ly ignored)
 *   L      host [n] lattice sides
 *   m_all  device FP64: the n starts back to back, [3][L_b^2] each; final points out
 *   mask_all device uint8 [sum_b L_b^2] active sites of every lattice, back
 *          to back (or NULL: all active): the climb, its eigen-solves and the
 *          certification then work in the masked tangent subspace
 *          (Algorithm 1: the minimum mode of the masked tangent Hessian;
 *          Methods: masked perturbation x0 + P_Omega delta), and the spins
 *          of inactive sites stay fixed
 *   res    device [n] results (status, iterations, HVP columns, E, ||F_mmf||, lambda_1, lambda_2)
 * The call uploads the small descriptor arrays (synchronising once before
 * the launch) and returns after queueing the launch.
 * Workspace: moto_saddle_search_batched_workspace(n, L, opts) bytes. */
#define MOTO_TILE_32x8 0  /* tile shapes of the lattice loops: 32 x 8 output sites */
#define MOTO_TILE_16x16 1 /* 16 x 16 */
#define MOTO_TILE_64x4 2  /* 64 x 4 */
size_t moto_saddle_search_batched_workspace(int32_t n, const int32_t *L /* host */, const moto_search_opts *o);
/*   tiles  host [n] tile shape of each lattice (MOTO_TILE_*), e.g. from
 *          moto_saddle_search_batched_autotune; NULL: 32 x 8 everywhere */
moto_status moto_saddle_search_batched(const moto_hamiltonian *h, int32_t n, const int32_t *L /* host */,
                                       double *m_all, const uint8_t *mask_all, const int32_t *tiles /* host */,
                                       const moto_search_opts *opts /* host */, moto_search_result *res, void *ws,
                                       size_t ws_bytes, moto_stream stream);

/* Autotuner of the batching form's tile shapes (systems; the paper runs its
 * searches one by one): the lattices are grouped by side into buckets 8
 * apart; for each bucket up to 4 members run 2 outer steps of the batched
 * search from copies of their starts (m_all and mask_all are not changed)
 * with each tile shape, timed on the stream with events, and the fastest
 * shape is written to tiles[] (host [n]) for every member of the bucket.
 * Synchronises with the stream.  Same arguments as the batched search
 * otherwise.  Workspace: moto_saddle_search_batched_autotune_workspace. */
size_t moto_saddle_search_batched_autotune_workspace(int32_t n, const int32_t *L /* host */,
                                                     const moto_search_opts *o);
moto_status moto_saddle_search_batched_autotune(const moto_hamiltonian *h, int32_t n, const int32_t *L /* host */,
                                                const double *m_all, const uint8_t *mask_all,
                                                const moto_search_opts *opts /* host */, int32_t *tiles /* host */,
                                                void *ws, size_t ws_bytes, moto_stream stream);

/* ---------------------------------------------------------------------
 * Explorer objectives (Methods, "Multi-objective initial-configuration
 * explorer"; Algorithm 1, population loop; Results, "Multi-objective explorer
 * over generations"): for a population of P candidates on the plan's lattice,
 *   x_p = x0 + P_Omega delta_p, each active spin then projected onto the
 *         unit sphere (an active site whose sum vanishes keeps x0; inactive
 *         sites keep x0),
 * and per candidate the three objectives an evolutionary selector ranks:
 *   diversity:      l1 distances to the other candidates and to an archive
 *                   A of n_archive configurations (sum over the population,
 *                   minimum over population and archive);
 *   feasibility:    |Q(x_p) - Q_target| with the Berg-Luescher charge;
 *   separability:   lambda_2 - lambda_1 of the tangent Hessian, restricted
 *                   to the masked subspace when a mask is given, from the
 *                   population eigen-solve (moto_min_modes_population).
 * The selector itself (NSGA-II) is not part of the library.
 *   x0      [3][N] FP64 device: the reference minimum
 *   mask    [N] device (1 = active) or NULL (all active)
 *   delta   [P][3][N] FP64 device: ambient perturbations
 *   archive [n_archive][3][N] FP64 device (NULL when n_archive == 0)
 *   x_out   [P][3][N] FP64 device: the candidates
 *   res     [P] device: objectives and the eigen-solve outcome per candidate
 *   evals   [P][k] FP64 device or NULL; V [P][k][3][N] FP64 device or NULL
 *           (the lowest modes, e.g. to start the climb from);
 *   D       [P][P + n_archive] FP64 device or NULL: the l1 distances
 * The call synchronises with the stream (the eigen-solve's convergence
 * checks) and returns after queueing the summary.
 * Errors: MOTO_EINVAL for P (1..MOTO_MAX_POPULATION), k or n_archive
 * (0..MOTO_MAX_ARCHIVE) out of range, eig.warm != 0 or missing pointers;
 * MOTO_EWORKSPACE below moto_explorer_workspace(p, hvp, P, n_archive, opts). */
typedef struct {
    int32_t k;          /* modes solved per candidate, 2..16 - guard (default 2) */
    int32_t reserved;
    double Q_target;    /* feasibility target; NaN (default): Q(x0) */
    moto_eig_opts eig;  /* eigen-solve options (FP32 HVP default tolerance 1e-5) */
} moto_explorer_opts;

typedef struct {
    double E;           /* energy */
    double lambda1, lambda2;
    double gap;         /* lambda2 - lambda1 */
    double Q;           /* topological charge */
    double violation;   /* |Q - Q_target| */
    double l1_sum;      /* sum of l1 distances to the other candidates */
    double l1_min;      /* smallest l1 distance to another candidate or an archive member (inf if none) */
    int32_t status;     /* eigen-solve outcome (MOTO_CONVERGED, ...) */
    int32_t iters;
    int64_t n_hvp;
} moto_explorer_result;

#define MOTO_MAX_ARCHIVE 4096
void moto_default_explorer_opts(moto_dtype hvp, moto_explorer_opts *o);
size_t moto_explorer_workspace(moto_plan p, moto_dtype hvp, int32_t P, int32_t n_archive,
                               const moto_explorer_opts *o);
moto_status moto_explorer_objectives(moto_plan p, moto_dtype hvp, int32_t P, const double *x0,
                                     const uint8_t *mask, const double *delta, int32_t n_archive,
                                     const double *archive, const moto_explorer_opts *opts /* host */,
                                     double *x_out, moto_explorer_result *res, double *evals,
                                     double *V, double *D, void *ws, size_t ws_bytes,
                                     moto_stream stream);

/* Defaults for the option structs. */
void moto_default_eig_opts(moto_dtype hvp, moto_eig_opts *o);
void moto_default_step_opts(moto_step_opts *o);
void moto_default_descend_opts(moto_dtype hvp, moto_descend_opts *o);
void moto_default_search_opts(moto_dtype hvp, moto_search_opts *o);

/* Berg-Luescher topological charge of each lattice in a batch, FP64 out
 * (the Q of the Results; a check of starts and descent end points).
 * Workspace: moto_energy_grad_workspace(p, batch). */
moto_status moto_topological_charge(moto_plan p, int32_t batch, const double *m, double *Q,
                                    void *ws, size_t ws_bytes, moto_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* MOTO_H */
