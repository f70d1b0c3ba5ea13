/*
 * fagbi.h - C ABI of the MI355X Galerkin boundary-integral Poisson-Boltzmann
 * operator and solver (Cartesian Taylor FMM + stored Galerkin near field).
 *
 * Problem (paper Sec. 2.1-2.3): a closed, conforming, outward-oriented surface
 * of N flat triangles separates a solute (dielectric eps_in, point charges
 * q_k at x_k) from a solvent (eps_out, inverse Debye length kappa).  The
 * unknowns are the piecewise-constant surface potential phi and its normal
 * derivative dphi (box-function Galerkin discretisation of the derivative
 * boundary integral equations), stacked as x = [phi_1..phi_N, dphi_1..dphi_N]
 * in the caller's panel order.  A x = b is the Galerkin system of Sec. 2.3:
 *   A11 = (1+eps)/2 M - (eps I3 - I2),  A12 = -I1,
 *   A21 = -I6,                          A22 = (1+1/eps)/2 M - (I4 - I5/eps),
 * eps = eps_out/eps_in, M = diag(panel areas), I1..I6 the panel-pair integrals
 * of G0 - Gk, dG0/dn_y, dGk/dn_y, dG0/dn_x, dGk/dn_x, d2(Gk - G0)/dn_x dn_y
 * (G0 = 1/(4 pi r), Gk = exp(-kappa r)/(4 pi r)).
 *
 * Conventions for every call:
 *   - return value: 0 = ok, < 0 = error (message in fagbi_last_error(), which
 *     is per calling thread), > 0 = warning (e.g. FAGBI_W_NOT_CONVERGED);
 *   - mesh and charge arrays are HOST pointers, read during the call and not
 *     retained; solution/vector arrays are DEVICE pointers of the current HIP
 *     device, owned by the caller, of 2n doubles unless stated otherwise, with
 *     n = N (panels, FAGBI_BASIS_S0: [phi_1..phi_N, dphi_1..dphi_N] in the
 *     caller's panel order) or n = V (vertices, FAGBI_BASIS_S1: the nodal
 *     values in the caller's vertex order);
 *   - `stream` is a hipStream_t (NULL = the default stream); asynchronous calls
 *     are ordered on it, calls documented as synchronising wait for it;
 *   - a handle owns all of its device memory, is bound to the device current
 *     at fagbi_create, and is not thread-safe; calls on one handle must not
 *     overlap.
 */
#ifndef FAGBI_H
#define FAGBI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  FAGBI_OK = 0,
  FAGBI_E_ARG = -1,      /* bad argument or parameter value */
  FAGBI_E_MESH = -2,     /* open/non-manifold/degenerate/inward mesh */
  FAGBI_E_STATE = -3,    /* call out of order (e.g. matvec before assembly) */
  FAGBI_E_OOM = -4,      /* device allocation failed */
  FAGBI_E_HIP = -5,      /* HIP runtime error */
  FAGBI_E_NUMERIC = -6,  /* NaN/Inf met, singular preconditioner block */
  FAGBI_W_NOT_CONVERGED = 1
};

enum { FAGBI_FP64 = 0, FAGBI_MIXED = 1 };
enum { FAGBI_PRECOND_NONE = 0, FAGBI_PRECOND_DIAG = 1, FAGBI_PRECOND_BLOCK = 2, FAGBI_PRECOND_GROUP = 3 };
enum { FAGBI_MLP_OFF = 0, FAGBI_MLP_PRECOND = 1, FAGBI_MLP_GATED = 2 };
/* cluster radii of the separation ratio (fagbi_params.radii) */
enum { FAGBI_RADII_LEVEL = 0, FAGBI_RADII_CLUSTER = 1 };
/* Galerkin space of phi and dphi (fagbi_params.basis), Sec. 2.3:
   FAGBI_BASIS_S0 the piecewise-constant box functions (unknowns per panel),
   FAGBI_BASIS_S1 the continuous piecewise-linear hat functions (unknowns per
   vertex; on a panel the hat function of its corner a is the barycentric
   coordinate lambda_a).  With S1 every entry of the system is the S0 entry's
   integral with lambda_a(x) lambda_b(y) inside, summed over the panels at the
   two vertices, the identity terms use the mass matrix int phi_i phi_j, and
   the sources and the energy interpolate the nodal values. */
enum { FAGBI_BASIS_S0 = 0, FAGBI_BASIS_S1 = 1 };
/* parts of the operator for fagbi_matvec_parts */
enum { FAGBI_PART_NEAR = 1, FAGBI_PART_FAR = 2, FAGBI_PART_ALL = 3 };

typedef struct fagbi_params {
  /* physics (Sec. 2.1): dielectric constants and inverse Debye length [1/A] */
  double eps_in, eps_out, kappa;
  /* cluster tree and FMM (Sec. 2.4): clusters c, c' of one level are
     neighbours iff (rho_c + rho_c') / |x_c - x_c'| > eta0, x_c the cube
     centre; with radii = FAGBI_RADII_LEVEL every cluster of level l has the
     radius rho_l (farthest 3-point-rule quadrature point of the level's
     panels from their cube centres), with FAGBI_RADII_CLUSTER each cluster
     its own rho_c (farthest vertex of its panels from its cube centre; the
     shrink scheme of Sec. 2.4 with the centre kept on the cube lattice);
     uniform depth with at most leaf_size panels per leaf cube; expansion
     order p_leaf at the leaves, p_l = min(p_leaf + L - l, p_max) per level
     when adaptive != 0 */
  double eta0;
  int32_t leaf_size, p_leaf, adaptive, p_max;
  /* near-field quadrature: Gauss points per dimension of the singular and
     close-pair rules; pairs closer than near_ratio*max(h_i, h_j) (centroid
     distance, h = sqrt(area)) use the close-pair rule */
  int32_t quad_duffy;
  double near_ratio;
  /* solve: FAGBI_FP64 (GMRES on the FP64 operator) or FAGBI_MIXED (flexible
     GMRES with the FP64 operator around inner GMRES on the FP32 operator) */
  int32_t precision;
  int32_t precond;             /* FAGBI_PRECOND_* */
  double tol;                  /* relative true residual ||b - Ax||/||b|| */
  int32_t max_iter;            /* Krylov basis size (no restart) */
  int32_t max_outer;           /* outer iterations in FAGBI_MIXED */
  double inner_tol;            /* inner relative tolerance in FAGBI_MIXED */
  int32_t mlp_mode;            /* FAGBI_MLP_* (needs fagbi_mlp_set_weights) */
  double mlp_gate_tol;         /* gated near field: max estimated rel. error */
  /* right-hand side of fagbi_solve: 0 = direct sum (fagbi_rhs), in (0, 1) =
     reverse treecode with this acceptance parameter (fagbi_rhs_treecode) */
  double rhs_theta;
  int32_t rhs_pmax;            /* its order cap: terms |a| <= min(p_l, rhs_pmax) */
  int32_t radii;               /* FAGBI_RADII_LEVEL (default) or FAGBI_RADII_CLUSTER */
  /* FAGBI_BASIS_S0 (default) or FAGBI_BASIS_S1.  S1 needs every vertex to
     belong to a triangle, mlp_mode FAGBI_MLP_OFF and precond
     FAGBI_PRECOND_NONE or FAGBI_PRECOND_DIAG; the allocation-free energy is
     not available with it (FAGBI_E_ARG). */
  int32_t basis;
} fagbi_params;

#define FAGBI_MAX_LEVELS 21        /* levels 0..20 (cube keys have 20 levels) */

typedef struct fagbi_tree_info {
  int64_t n_panels, n_leaves;
  int32_t levels;              /* leaf level L (levels are 0..L) */
  int32_t lmin;                /* coarsest level with interactions (L+1: none) */
  int64_t near_pairs;          /* stored near-field panel pairs */
  int64_t m2l_pairs;           /* cluster pairs over all interaction lists */
  int64_t m2l_flops_fp;        /* M2L multiply-adds per matvec, both channels */
  int64_t singular_pairs[4];   /* identical, edge, vertex, close */
  int32_t order_leaf, order_root;
  double rho_leaf, h_leaf;
  /* per level l = 0..levels (entries beyond are 0) */
  int32_t lev_clusters[FAGBI_MAX_LEVELS];   /* clusters (non-empty cubes) */
  int32_t lev_order[FAGBI_MAX_LEVELS];      /* expansion order p_l */
  int32_t lev_offsets[FAGBI_MAX_LEVELS];    /* distinct interaction offsets */
  int32_t lev_pad;
  int64_t lev_pairs[FAGBI_MAX_LEVELS];      /* interaction pairs (c, c' in I(c)) */
  int64_t device_bytes;        /* device memory the handle holds (tree, near field, far-field tables and
                                  expansions, preconditioner, Krylov and treecode workspaces) */
  /* FAGBI_BASIS_S1 (after assembly): the near field by vertex pairs, rows
     (per leaf, the distinct vertices of its panels) and entries (rows times
     the distinct vertices of the leaf's source panels); 0 otherwise */
  int64_t hat_rows, hat_entries;
} fagbi_tree_info;

typedef struct fagbi_solve_info {
  int32_t outer_iterations;    /* FGMRES steps (FAGBI_MIXED) or 1 */
  int32_t inner_iterations;    /* total Krylov iterations */
  int32_t matvecs_fp64, matvecs_fp32;
  double rel_residual;         /* true ||b - A64 x|| / ||b|| at exit */
  double t_rhs_ms, t_solve_ms;
} fagbi_solve_info;

/* Per-phase matvec timings from HIP events recorded on the caller's stream
   around each phase (index 0: FAGBI_FP64, 1: FAGBI_MIXED). */
typedef struct fagbi_profile {
  int64_t matvecs[2];
  double ms_total[2];          /* whole matvec (incl. the reorder of x into tree order) */
  double ms_near[2];           /* near-field block SpMV kernel (incl. identity terms; it runs on a
                                  second stream beside the far field, so the phases overlap) */
  double ms_up[2];             /* P2M + MtM */
  double ms_m2l[2];            /* MtL, all levels */
  double ms_down[2];           /* LtL + LtP */
  /* setup stages of the last build/assembly (host wall clock around
     stream-synchronised stages, recorded while profiling is on) */
  double ms_tree;              /* fagbi_build_tree */
  double ms_classify;          /* near-field pair classes, regular pairs */
  double ms_surrogate;         /* network features, inference, gated entries */
  double ms_singular;          /* singular / close cubature */
  double ms_fmm_setup;         /* far-field tables, panel moments */
  double ms_precond;           /* block-diagonal factors */
  double ms_m2l_leaf[2];       /* the leaf level's MtL kernel alone (events on its stream) */
} fagbi_profile;

typedef struct fagbi_handle fagbi_handle;

/* Fill *p with the defaults: eps 1/80, kappa 0.1257, eta0 0.8, leaf 32,
   p_leaf 4 fixed order, p_max 8, quad_duffy 7, near_ratio 2, FP64, block
   preconditioner, tol 1e-6, max_iter 200, max_outer 5, inner_tol 5e-7 (one
   inner solve normally reaches the outer tolerance). */
int fagbi_default_params(fagbi_params* p);

/* Create a handle on the current device.  *out receives the handle. */
int fagbi_create(const fagbi_params* p, fagbi_handle** out);

/* Geometry and cluster tree (Sec. 2.3 panels; Sec. 2.4 cluster tree,
   separation ratio, neighbour and interaction lists).  verts: host f64[nv*3],
   tris: host i32[nt*3] (0-based, counter-clockwise seen from the solvent).
   Rejects open, non-manifold, degenerate (zero-area) and inward meshes with
   FAGBI_E_MESH.  Synchronises. */
int fagbi_build_tree(fagbi_handle* h, const double* verts, int64_t nv,
                     const int32_t* tris, int64_t nt);

/* Near-field Galerkin blocks for every leaf pair (c, c') with c' in N(c)
   (Sec. 2.3 linear system entries; singular pairs by Sauter-Schwab-type
   relative-coordinate cubature, Sec. 2.3 last paragraph), their FP32 copy,
   the FMM translation tables and the block-diagonal preconditioner factors
   (Sec. 2.6).  With FAGBI_BASIS_S1 each stored panel pair holds the 3 x 3
   corner integrals (singular and close pairs by the same relative-coordinate
   and Duffy rules with the barycentric products inside, the identical and
   edge rules' analytic inner variable replaced by exact 3- and 2-point
   rules), and the preconditioner is the diagonal of A.  Requires
   fagbi_build_tree.  Synchronises. */
int fagbi_assemble_nearfield(fagbi_handle* h, void* stream);

/* y = A x (Sec. 2.4 six-step FMM: near field, moments, upward pass,
   interaction phase, downward pass, evaluation).  precision FAGBI_FP64: FP64
   throughout; FAGBI_MIXED: FP32 near-field entries and FP32 expansions with
   FP64 accumulation of y.  x, y: device f64[2n], caller order, must not
   alias.  Asynchronous on stream. */
int fagbi_matvec(fagbi_handle* h, const double* x, double* y, int32_t precision,
                 void* stream);

/* As fagbi_matvec but restricted to parts (FAGBI_PART_* bit mask). */
int fagbi_matvec_parts(fagbi_handle* h, const double* x, double* y,
                       int32_t precision, int32_t parts, void* stream);

/* y = M^{-1} z for the block-diagonal preconditioner of Sec. 2.6: blocks
   [phi_c; dphi_c] of one leaf (FAGBI_PRECOND_BLOCK) or of consecutive leaves
   holding at most 32 panels (FAGBI_PRECOND_GROUP); each block holds the
   stored near-field entries between its panels plus the identity terms.  The
   assembly stores each block's explicit inverse, computed by Gauss-Jordan
   elimination with partial pivoting in FP64 (FAGBI_E_NUMERIC for a singular
   block); the apply is one dense block product per block.  With
   precond = FAGBI_PRECOND_DIAG the diagonal of A is used instead.  z, y:
   device f64[2n] (may alias).  Asynchronous on stream. */
int fagbi_precond_apply(fagbi_handle* h, const double* z, double* y, void* stream);

/* Right-hand side b (Sec. 2.2 source terms S1, S2 tested with the box
   functions): xq host f64[nc*3] charge positions [A], q host f64[nc] charges
   [e]; b device f64[2n].  Asynchronous on stream (arguments copied before
   return). */
int fagbi_rhs(fagbi_handle* h, const double* xq, const double* q, int64_t nc,
              double* b, void* stream);

/* Solve A x = b(charges), the Galerkin system of Sec. 2.3 (its closing
   paragraph: GMRES with the FMM product of Sec. 2.4 and the block-diagonal
   preconditioner of Sec. 2.6), by right-preconditioned GMRES without restart
   (classical Gram-Schmidt applied twice, Givens rotations; FP64) or, with
   FAGBI_MIXED, by flexible GMRES on the FP64 operator whose preconditioner is
   an inner GMRES on the FP32 operator to inner_tol.  The tolerance applies to
   the true relative residual ||b - A64 x|| / ||b||.  b comes from the charges
   by fagbi_rhs (rhs_theta = 0) or fagbi_rhs_treecode.  x: device f64[2n], the
   initial guess on entry (zeros: pass zeros), the solution on exit.  info may
   be NULL.  Returns FAGBI_W_NOT_CONVERGED with the best x if the tolerance is
   not met.  Synchronises. */
int fagbi_solve(fagbi_handle* h, const double* xq, const double* q, int64_t nc,
                double* x, fagbi_solve_info* info, void* stream);

/* Solvation energy (Sec. 2.3 discrete E_sol times 4 pi 332.0716, Sec. 3) in
   kcal/mol from a solution x (device f64[2n]).  FP64 direct sum over charges
   and panel quadrature points.  Synchronises. */
int fagbi_solvation_energy(fagbi_handle* h, const double* x, const double* xq,
                           const double* q, int64_t nc, double* E_kcal,
                           void* stream);

/* For callers that cannot allocate device memory during a call (code under
   HIP graph capture, tight serving loops, harnesses that forbid it): the
   direct energy sum of fagbi_solvation_energy with the same kernels and
   summation order, making no device allocation.  Its per-block partial sums
   live in a static device array of the library (65,536 doubles per GPU, held
   until the process ends), so N <= 2^24 panels (FAGBI_E_ARG beyond).
   chg: device f64[nc][4] {x, y, z [A], q [e]}, 32-byte aligned; x: device
   f64[2N] (caller order); E_kcal: device f64[1], receives the energy in
   kcal/mol.  Asynchronous on stream; no finite-value check (the caller reads
   E_kcal).  Every call on one GPU shares that GPU's array (nothing in it needs
   clearing: each call writes every partial sum it reads), so calls that
   overlap on one GPU, from any handles, race. */
int fagbi_solvation_energy_noalloc(fagbi_handle* h, const double* x, const double* chg,
                                   int64_t nc, double* E_kcal, void* stream);

/* Right-hand side as fagbi_rhs by the Cartesian treecode of Sec. 2.5 run in
   reverse: every charge visits the clusters as in
   fagbi_solvation_energy_treecode; an accepted cluster receives the charge's
   particle-to-local Taylor expansion (order min(p_l, p_max), Coulomb kernel;
   p_max >= 8 evaluates the full orders), a leaf that
   fails receives the direct 3-point sums; the far field's LtL then takes the
   local expansions to the leaves and LtP tests them with each panel's single-
   and double-layer moments (FAGBI_BASIS_S1: the leaf sums and LtP per panel
   corner with lambda_a, summed into the vertices).  theta in [0, 1) (theta =
   0: the direct sum).  xq: host f64[nc][3]; q:
   host f64[nc]; b: device f64[2n] (caller order), overwritten.  Requires
   fagbi_assemble_nearfield.  The expansions are accumulated with device
   atomics: results agree between runs to rounding, not bit for bit.  Uses
   the far field's local-expansion buffers (not concurrently with a matvec of
   the same handle).  FAGBI_E_ARG as for the treecode energy.  Synchronises. */
int fagbi_rhs_treecode(fagbi_handle* h, const double* xq, const double* q,
                       int64_t nc, double theta, int32_t p_max, double* b,
                       void* stream);

/* Solvation energy as above by the Cartesian treecode of Sec. 2.5: the
   moments of x (leaf moments and the MtM upward pass of the far field, FP64,
   orders p_l) give each charge a particle-cluster term of order
   min(p_l, p_max) (p_max >= 8: the full orders) from every cluster
   with rho_l / R <= theta (rho_l the level's cluster radius, R the distance
   of the charge from the cube centre); clusters failing the criterion pass
   it to their children, from level min(l_min, L) down; leaves failing it are
   summed directly as in fagbi_solvation_energy (FAGBI_BASIS_S1: the moments
   from the corner moments, the leaf sums with the nodal values interpolated).
   All charges advance level by level together (one list of (charge, cluster)
   pairs per level).  theta in [0, 1); theta = 0 gives the direct sum.
   x: device f64[2n] (caller order); xq: host f64[nc][3]; q: host f64[nc].
   Requires fagbi_assemble_nearfield (the far-field tables); orders above 8
   are rejected.  FAGBI_E_ARG when a level would hold more than 2^26
   (charge, cluster) pairs (theta too small for the tree and the charges).
   Contributions are accumulated with device atomics: results agree between
   runs to rounding, not bit for bit.  Uses the far field's moment buffers
   (not concurrently with a matvec of the same handle).  Synchronises. */
int fagbi_solvation_energy_treecode(fagbi_handle* h, const double* x,
                                    const double* xq, const double* q,
                                    int64_t nc, double theta, int32_t p_max,
                                    double* E_kcal, void* stream);

/* Turn per-phase matvec timing on (1) or off (0); turning it on resets the
   counters.  While on, every matvec waits for its last phase to finish
   (one host synchronisation per matvec). */
int fagbi_set_profiling(fagbi_handle* h, int32_t on);

/* Accumulated per-phase timings since profiling was turned on. */
int fagbi_get_profile(fagbi_handle* h, fagbi_profile* out);

/* Tree statistics (after fagbi_build_tree; near-field counts after assembly). */
int fagbi_get_tree_info(fagbi_handle* h, fagbi_tree_info* info);

/* Tree order: perm[k] = caller panel index of the k-th panel in tree (Morton)
   order; perm host i32[N]. */
int fagbi_get_permutation(fagbi_handle* h, int32_t* perm);

/* ---- learned near-field surrogate (an addition to the paper's method) ----
   A 16 -> 128 -> 128 -> 128 -> 6 tanh network predicts, from the geometry of
   a near-singular panel pair (edge- or vertex-adjacent, or closer than
   near_ratio), the correction of its six integrals I1..I6 over the 3x3
   regular rule, in units of h^3, h^2 (x4), h with h = sqrt(target area).
   Features: target corners (3) and source corners (9) in the target frame
   over h, kappa*h, class one-hot (3).  The blob exchanged by get/set holds
   the parameters (W1 b1 W2 b2 W3 b3 W4 b4, W row-major [in][out]), the
   input/output standardisation (input mean[16] sd[16], per class output
   mean[3][6] sd[3][6]) and the
   gate calibration (per class: 9 distance-ratio bin edges, then per class 8
   calibrated error values). */
enum { FAGBI_MLP_NIN = 16, FAGBI_MLP_NOUT = 6, FAGBI_MLP_NAUX = 8,
       FAGBI_MLP_NPARAM = 35974, FAGBI_MLP_NBLOB = 36093 };

/* Training data from the current mesh (after fagbi_assemble_nearfield):
   up to max_pairs near-singular pairs (every k-th of each class), labelled by
   the library's singular cubature.  X: device f32[max_pairs*16] features,
   T: device f32[max_pairs*6] targets, aux: device f32[max_pairs*8]
   {class 0/1/2 = edge/vertex/close, centroid distance / sqrt(h_i h_j),
   the six full integrals in target units}.  *n_out = rows written.
   Synchronises. */
int fagbi_mlp_dataset(fagbi_handle* h, int64_t max_pairs, float* X, float* T,
                      float* aux, int64_t* n_out, void* stream);

/* Train the handle's network on n >= 100 rows (device arrays as produced by
   fagbi_mlp_dataset; every tenth row is held out for the gate
   calibration): Adam, cosine-decayed learning rate, minibatches of `batch`
   rows, standardised inputs/targets, mean squared error; Xavier initial
   weights from the counter-based generator splitmix64(seed).
   loss_hist: host f32[epochs] mean training loss per epoch (may be NULL).
   Synchronises. */
int fagbi_mlp_train(fagbi_handle* h, const float* X, const float* T, const float* aux,
                    int64_t n, int32_t epochs, int32_t batch, float lr, uint64_t seed,
                    float* loss_hist, void* stream);

/* Inference: Y (device f32[n*6]) = network(X) in target units. */
int fagbi_mlp_forward(fagbi_handle* h, const float* X, float* Y, int64_t n, void* stream);

/* Loss and gradient of the raw network (no standardisation) with host
   parameters theta (f32[FAGBI_MLP_NPARAM]) on device X (f32[n*16]) and
   T (f32[n*6]), 1 <= n <= 65536: loss = mean over rows and outputs of
   (y - t)^2; grad host f32[FAGBI_MLP_NPARAM].  For checking the training
   kernels.  Synchronises. */
int fagbi_mlp_grad(fagbi_handle* h, const float* theta, const float* X, const float* T,
                   int32_t n, float* loss, float* grad, void* stream);

/* Copy the trained network out / in (host f32[FAGBI_MLP_NBLOB]). */
int fagbi_mlp_get_weights(fagbi_handle* h, float* blob, int64_t n);
int fagbi_mlp_set_weights(fagbi_handle* h, const float* blob, int64_t n);

/* After an assembly with mlp_mode != OFF: pairs whose entries came from the
   network (gated) out of the near-singular candidates. */
int fagbi_get_mlp_stats(fagbi_handle* h, int64_t* gated_pairs, int64_t* candidate_pairs);

void fagbi_destroy(fagbi_handle* h);
const char* fagbi_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FAGBI_H */
