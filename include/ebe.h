/*
 * ebe.h -- C ABI of the MI355X element-by-element (EBE) multi-case solver.
 *
 * The library computes, on one gfx950 GPU, the hot path of the implicit
 * low-order unstructured finite-element crust-deformation solver of
 * Yamaguchi et al. (WACCPD 2017): the EBE product f = sum_i Q_i K_i Q_i^T u
 * (Section 2, Eq. (3)) on 10-node tetrahedra with isotropic linear
 * elasticity (Eq. (1a-c)) and per-element moduli, applied to n load cases
 * at once (Section 3.1), inside the adaptive conjugate-gradient solver of
 * Algorithm 1 (FP64 outer loop, FP32 multigrid inner loops on the quadratic
 * mesh, its corner-only linear mesh and an algebraic coarsening of the
 * latter).
 * Element matrices are never stored: they are rebuilt from vertex
 * coordinates and material at every product (Section 2, EBE method).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Pointers named *_dev are device pointers (hipMalloc / torch CUDA tensors);
 *   all others are host pointers.  The caller owns every vector buffer; the
 *   library only reads inputs and writes outputs during the call's stream work.
 * - Multi-case vectors use the layout [node][component][rhs], rhs fastest
 *   (Section 3.1: the case index is the innermost, contiguous loop), so a
 *   vector of n cases on N nodes holds 3*N*n values.  Quadratic-level vectors
 *   have N = n_nodes; linear-level (corner-only) vectors have N = n_vertices;
 *   level-2 vectors have N = the number of aggregates (ebe_level2_info).
 * - Buffers must not overlap unless stated.  Device buffers must be 16-byte
 *   aligned (every hipMalloc / torch allocation is); a misaligned one is
 *   rejected with EBE_ERR_ARG.
 * - `stream` is a hipStream_t (NULL = the default stream).  Calls marked
 *   "asynchronous" only enqueue work on it; the others synchronise it.
 * - A mesh handle must be used by one stream at a time.
 * - No C++ exception crosses this interface.  Every call returns an
 *   ebe_status; on failure a thread-local message is kept for ebe_last_error().
 * - nrhs is 1..EBE_MAX_RHS.  Larger case sets are solved as several sets of at
 *   most 16 cases, as the paper does (Section 5: 368 cases as 23 sets of 16).
 */
#ifndef EBE_H
#define EBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EBE_MAX_RHS 16

typedef int32_t ebe_status;
#define EBE_OK 0
#define EBE_NOT_CONVERGED 1      /* result valid but tolerance not reached; see stats */
#define EBE_ERR_ARG (-1)         /* null pointer, size or enum out of range */
#define EBE_ERR_INDEX (-2)       /* connectivity index out of range or inconsistent */
#define EBE_ERR_INVERTED (-3)    /* element with det[x1-x0, x2-x0, x3-x0] <= 0 */
#define EBE_ERR_CURVED (-4)      /* edge node not at its edge midpoint */
#define EBE_ERR_MATERIAL (-5)    /* E <= 0, nu outside (-1, 0.5), or non-finite */
#define EBE_ERR_OOM (-6)         /* device allocation failed */
#define EBE_ERR_HIP (-7)         /* a HIP runtime call failed */
#define EBE_ERR_BREAKDOWN (-8)   /* (p, Kp) <= 0 in the outer loop: K not SPD on the free DOFs */
#define EBE_ERR_NONFINITE (-9)   /* NaN or Inf in an input or in the iteration */
#define EBE_ERR_NUMBERING (-10)  /* numbering is not vertex-first */

typedef int32_t ebe_dtype;
#define EBE_F64 0
#define EBE_F32 1

/* Preconditioner of the outer loop (Algorithm 1(a)). */
#define EBE_PREC_PCGE 0  /* plain CG with 3x3 block Jacobi ("PCGE", Section 4) */
#define EBE_PREC_MG2 1   /* adaptive CG: inner CG on the linear mesh, then on the quadratic mesh */
#define EBE_PREC_MG3 2   /* adaptive CG: inner CG on the level-2 aggregates, the linear mesh, the
                            quadratic mesh (the paper's three inner loops) */

/* Arithmetic of the preconditioner; the outer loop is always FP64. */
#define EBE_MODE_FP64 0
#define EBE_MODE_MIXED 1 /* preconditioner (inner loops, EBE products) in FP32 */

/* Forms of the product kernel (same result up to rounding, different
 * speed): GATHER reads each element's nodal values straight from x; STAGED
 * copies a patch's node rows into LDS first, a few cases at a time;
 * PIPELINED is GATHER in persistent workgroups that fetch the next patch's
 * metadata while computing the current one; ASSEMBLED (linear level only)
 * applies K1 assembled once (per material) into 3x3 blocks over the corner
 * graph instead of forming element products, so a product reads each block
 * once for all cases: a departure from the paper's element-by-element
 * coarse level, chosen only where it measures faster.  COLOURED (quadratic
 * level only) colours the element patches so that no two patches of a
 * colour share a node and runs the colours one after another, each patch
 * adding its sums straight into y (the multi-colouring Section 2 uses on
 * CPUs, where Section 3.2 takes atomics on GPUs; here over patches): no
 * staging buffer and no second pass; the patches' sums reach a node in a
 * fixed (colour) order, while inside a patch the sums are LDS atomics, as
 * in the other forms, so results agree to rounding, not bit for bit.
 * DETERMINISTIC (quadratic level only) is GATHER without atomics: each
 * element-case stores its nodal forces in slots of its own in LDS, and each
 * patch node adds the slots of the elements that touch it in a fixed order
 * (in FP64), so y = K x is the same bit for bit on every run (the (x, K x)
 * sums the solver takes from its products are not); its variant 1 runs the
 * patches colour by colour, as COLOURED does.  It needs the geometry
 * cache (filled by the entry points) and takes the cases in passes of at
 * most 8 (FP32) or 4 (FP64).
 * PIPELINED and COLOURED need a mesh below 2^25 nodes whose vectors at this
 * (dtype, nrhs) are below 4 GiB; elsewhere GATHER runs in their place.
 * AUTO: the mesh's tuned choice, else a fixed default. */
typedef enum {
  EBE_FORM_AUTO = -1,
  EBE_FORM_GATHER = 0,
  EBE_FORM_STAGED = 1,
  EBE_FORM_PIPELINED = 2,
  EBE_FORM_ASSEMBLED = 3,
  EBE_FORM_COLOURED = 4,
  EBE_FORM_DETERMINISTIC = 5,
  EBE_NUM_FORMS = 6
} ebe_form;

typedef struct ebe_mesh ebe_mesh;   /* opaque; owns device copies of the mesh and workspace */
typedef struct ebe_batch ebe_batch; /* opaque; a set of meshes solved together */

/* Solver options.  ebe_pcg_default_opts() fills the paper's settings:
 * MG3 (three inner levels), MIXED, tol 1e-8, inner tolerances
 * {0.1, 0.05, 0.025} and maxima {30, 300, 3000} (Section 4, Table 2).
 * MG3 needs every row of the level-2 operator to couple at most 800
 * aggregates (the set-up sums a row in 64 KB of LDS); on a mesh past that
 * limit a solve asked for MG3 runs MG2 instead and says so in
 * ebe_pcg_stats.precond_used. */
typedef struct {
  int32_t precond;      /* EBE_PREC_* */
  int32_t mode;         /* EBE_MODE_* */
  double tol;           /* stop when max_j ||f_j - K u_j|| / ||f_j|| <= tol (unsquared) */
  int32_t max_outer;    /* outer iteration cap */
  int32_t check_every;  /* host reads the device convergence flag every k outer iterations */
  double inner_eps[3];  /* squared relative-residual tolerance of inner levels 0, 1, 2 (Table 2) */
  int32_t inner_max[3]; /* inner loops run while i < N, i from 1: at most N-1 steps */
  int32_t use_x0;       /* 1: u_dev holds the initial guess on entry; 0: start from zero */
  int32_t coarse_guess; /* 0: u1 = P1^T u as printed; 1: u1 = corner values of u */
  int32_t graphs;       /* 1 (default): replay captured HIP graphs of the fixed runs of
                           inner steps (and of PCGE outer steps) enqueued between two
                           convergence checks; needs a stream other than NULL (the legacy
                           default stream cannot be captured), else ignored */
  int32_t coarse_half;  /* 1: (MIXED with MG2 / MG3) the linear level applies K1 assembled and
                           stored in FP16, and level 2 its A2 in FP16 (values scaled by the largest
                           magnitude over 2^14; FP32 arithmetic): a low-precision preconditioner
                           experiment that halves the coarse operators' traffic; 0 (default): off */
  int32_t deterministic; /* 1: a bit-reproducible solve: the same u and statistics on every run.
                            The quadratic-level products use EBE_FORM_DETERMINISTIC (with the
                            mesh's variant for it), the linear level the assembled K1, and every
                            (p, K p) is summed by a separate pass in a fixed order (the products'
                            own folds use atomics); about 1.2-1.5x the time of a tuned solve.
                            Straight-sided meshes only (else EBE_ERR_ARG); ebe_batch_solve then
                            solves every mesh on its own.  0 (default): off */
} ebe_pcg_opts;

typedef struct {
  int32_t outer_iters;
  int32_t status;          /* same as the return value of the solve */
  int64_t inner_iters[3];  /* total inner steps on levels 0, 1 and 2 */
  double max_rel_res;      /* max_j ||r_j|| / ||f_j|| of the recursive residual at exit */
  double seconds;          /* wall time of the solve, host clock */
  int32_t precond_used;    /* the preconditioner that ran: opts.precond, except that EBE_PREC_MG3
                              falls back to EBE_PREC_MG2 on a mesh whose level-2 rows are too long
                              for the level-2 set-up (more than 800 coupled aggregates) */
  int32_t graphs_captured; /* HIP graphs captured (not replayed) during this solve */
  int32_t merged;          /* ebe_batch_solve: number of meshes solved together in the merged
                              system that produced this result (0: solved on its own) */
  int32_t reserved;        /* 0 */
} ebe_pcg_stats;

/* ---- mesh ------------------------------------------------------------- */

/* Create a mesh handle from host arrays (copied; synchronous).
 * Defines Q_i (connectivity), the coordinates and the per-element material
 * from which every K_i is rebuilt (Section 2, Eq. (3) and the EBE method).
 *   xyz       [n_nodes][3] coordinates.
 *   conn10    [n_elem][10] node ids: corners 0..3, then edge nodes of
 *             edges (0,1),(1,2),(0,2),(0,3),(1,3),(2,3).
 *   n_vertices  nodes 0..n_vertices-1 must be exactly the corners
 *             (vertex-first numbering; checked, never reordered).
 *   young, poisson  [n_elem] isotropic moduli E_e, nu_e.
 *   dof_fixed [n_nodes][3] 1 = homogeneous Dirichlet DOF, or NULL (none).
 * Checks: index range and numbering, det > 0, edge nodes at midpoints
 * (|x_edge - midpoint| <= 1e-10 * longest edge), material range, finiteness.
 * n_nodes must be below 2^28.  On error *out is set to NULL. */
ebe_status ebe_mesh_create(const double* xyz, int64_t n_nodes, int64_t n_vertices,
                           const int32_t* conn10, int64_t n_elem,
                           const double* young, const double* poisson,
                           const uint8_t* dof_fixed, void* stream, ebe_mesh** out);

/* Create a mesh of curved (isoparametric) 10-node tetrahedra: the same
 * arguments and checks as ebe_mesh_create, except that edge nodes may lie
 * anywhere; instead the Jacobian of each element's quadratic map
 * x(L) = sum_a N_a(L) x_a must be positive (det J > 1e-14 * longest corner
 * edge^3) at the four quadrature points and at the ten nodes, else
 * EBE_ERR_INVERTED.  K_e = sum_q w_q B_q^T D B_q det J_q with the symmetric
 * 4-point rule (Section 2, Eq. (2): the isoparametric element with its
 * Jacobian evaluated per point; for straight elements this equals the
 * straight-sided operator to rounding).  Products on the quadratic level use
 * the gather form of the patch kernel with the element geometry formed at
 * every product from the ten node coordinates; the linear level (corners)
 * and level 2 are as for straight meshes.  Not supported on such a mesh
 * (EBE_ERR_ARG): ebe_adjoint_grad, ebe_fault_create; batches solve it on its
 * own (never merged). */
ebe_status ebe_mesh_create_curved(const double* xyz, int64_t n_nodes, int64_t n_vertices,
                                  const int32_t* conn10, int64_t n_elem,
                                  const double* young, const double* poisson,
                                  const uint8_t* dof_fixed, void* stream, ebe_mesh** out);

/* Replace the per-element moduli from device arrays [n_elem] (asynchronous
 * apart from a range check that synchronises the stream). */
ebe_status ebe_mesh_set_material(ebe_mesh* mesh, const double* young_dev,
                                 const double* poisson_dev, void* stream);

/* Sizes of a mesh; any out pointer may be NULL. */
ebe_status ebe_mesh_info(const ebe_mesh* mesh, int64_t* n_nodes, int64_t* n_vertices,
                         int64_t* n_elem);

void ebe_mesh_destroy(ebe_mesh* mesh);

/* Work decomposition of the EBE products on level 0 (quadratic mesh) or 1
 * (corners): element patches (consecutive elements whose nodal sums fit a
 * workgroup's LDS), nodes shared by several patches, staged partial-sum rows
 * (one per (patch, shared node) pair: what the staging forms write and the
 * node-centric pass reads back), and colours of the COLOURED form (0 at
 * level 1).  Any out pointer may be NULL. */
ebe_status ebe_patch_info(const ebe_mesh* mesh, int32_t level, int64_t* n_patches, int64_t* n_shared,
                          int64_t* n_staged, int32_t* n_colours);

/* ---- operators (asynchronous) ---------------------------------------- */

/* y = K x for nrhs cases (Section 2, Eq. (3)), K rebuilt element by element.
 * x_dev, y_dev: [n_nodes][3][nrhs] of dtype (double or float).  y is
 * overwritten.  apply_bc = 1 computes y = P K P x, P zeroing fixed DOFs.
 * FP32 sums in FP32 (element geometry is formed from FP64 coordinates). */
ebe_status ebe_matvec(ebe_mesh* mesh, ebe_dtype dtype, int32_t nrhs, const void* x_dev,
                      void* y_dev, int32_t apply_bc, void* stream);

/* y += K x: the same product accumulated into y (no clearing pass), e.g. for
 * residuals r = K u - f with y holding -f on entry.  Same arguments. */
ebe_status ebe_matvec_add(ebe_mesh* mesh, ebe_dtype dtype, int32_t nrhs, const void* x_dev,
                          void* y_dev, int32_t apply_bc, void* stream);

/* y = K x (or P K P x) like ebe_matvec, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): this call allocates nothing.  The
 * shared-node partial sums are staged in a fixed device array of the library
 * (64 MiB per GPU, held until the process ends); the call is refused with
 * EBE_ERR_ARG when the mesh needs more than that at this nrhs and dtype
 * (one staged row per (patch, shared node) pair, 3 x nrhs values of 8 or 4
 * bytes each: at FP32 with 16 cases at most 349,525 rows, which a 24^3-hex
 * cube of 82,944 tetrahedra, about 180k rows, fits).  Always the gather
 * form; element geometry from the mesh's geometry cache when an earlier call
 * filled it, else from the corner coordinates.  Every call on a GPU shares
 * that GPU's array: calls that overlap in time on one GPU (other streams,
 * other threads) race and give wrong results; calls in one stream order are
 * safe.  Asynchronous; same arguments and result as ebe_matvec up to
 * rounding. */
ebe_status ebe_matvec_noalloc(ebe_mesh* mesh, ebe_dtype dtype, int32_t nrhs, const void* x_dev,
                              void* y_dev, int32_t apply_bc, void* stream);

/* y = K1 x on the linear (4-node) mesh made of the corners, the coarse
 * operator of inner loop level 1 (Section 2, multigrid; Table 4 "1st order EBE").
 * x_dev, y_dev: [n_vertices][3][nrhs]. */
ebe_status ebe_matvec_p1(ebe_mesh* mesh, ebe_dtype dtype, int32_t nrhs, const void* x_dev,
                         void* y_dev, int32_t apply_bc, void* stream);

/* Grid transfers between the quadratic mesh and the corner-only linear mesh
 * (Algorithm 1(a), P1 and its transpose).  prolong: y[n_nodes] = P1 x[n_vertices]
 * (corner copied, edge node = mean of its two corners); restrict:
 * y[n_vertices] = P1^T x[n_nodes].  Fixed DOFs of y are zeroed when apply_bc = 1. */
ebe_status ebe_prolong_p1(ebe_mesh* mesh, ebe_dtype dtype, int32_t nrhs, const void* x_dev,
                          void* y_dev, int32_t apply_bc, void* stream);
ebe_status ebe_restrict_p1(ebe_mesh* mesh, ebe_dtype dtype, int32_t nrhs, const void* x_dev,
                           void* y_dev, int32_t apply_bc, void* stream);

/* 3x3 block Jacobi of Algorithm 1 ("diag[ ]"): level 0 = quadratic K, level 1
 * = linear K1, level 2 = A2.  Blocks are the nodal 3x3 diagonal blocks of
 * P K P with fixed rows/columns set to identity, formed and inverted in FP64.
 *   ebe_diag_blocks: writes the (uninverted) blocks, row-major [N][9] double.
 *   ebe_block_jacobi: y = M^-1 x, x/y [N][3][nrhs] of dtype. */
ebe_status ebe_diag_blocks(ebe_mesh* mesh, int32_t level, double* blocks_dev, void* stream);
ebe_status ebe_block_jacobi(ebe_mesh* mesh, int32_t level, ebe_dtype dtype, int32_t nrhs,
                            const void* x_dev, void* y_dev, void* stream);

/* ---- level 2: algebraic coarsening of the linear mesh ------------------- */

/* Inner loop level 2 of Algorithm 1(a) runs on a smoothed-aggregation
 * coarsening of the corner mesh: corners grouped into aggregates (three
 * greedy passes over the corner graph in increasing id: a corner whose
 * neighbours are all free roots an aggregate of itself and its neighbours; a
 * corner left joins the lowest neighbouring aggregate; leftovers root their
 * own), one 3-DOF node per aggregate.  The tentative map T copies an
 * aggregate's value to its members' free DOFs; P2 = (I - 2/3 D1^-1 K1p) T
 * (one damped block-Jacobi step, K1p = P K1 P, D1 the level-1 blocks);
 * A2 = P2^T K1p P2, kept as 3x3 blocks (Section 2: "3 x 3 block compressed
 * row storage"); a coarse DOF whose members are all fixed in that component
 * is fixed.  Built with the mesh (structure) and on first use (values, per
 * material).
 *   ebe_level2_info: number of aggregates, and (agg_host [n_vertices] or
 *     NULL) each corner's aggregate; synchronous.
 *   ebe_matvec_l2: y = A2 x, x/y [n_agg][3][nrhs] of dtype (apply_bc: P A2 P).
 *   ebe_prolong_l2: y[n_vertices] = P2 x[n_agg] (zero at fixed DOFs).
 *   ebe_restrict_l2: y[n_agg] = P2^T x[n_vertices] (zero at fixed coarse
 *     DOFs).
 * The vector entry points are asynchronous except the first call after a
 * material change, which forms A2 and synchronises the stream. */
ebe_status ebe_level2_info(const ebe_mesh* mesh, int64_t* n_agg, int32_t* agg_host);
ebe_status ebe_matvec_l2(ebe_mesh* mesh, ebe_dtype dtype, int32_t nrhs, const void* x_dev, void* y_dev,
                         int32_t apply_bc, void* stream);
ebe_status ebe_prolong_l2(ebe_mesh* mesh, ebe_dtype dtype, int32_t nrhs, const void* x_dev, void* y_dev,
                          void* stream);
ebe_status ebe_restrict_l2(ebe_mesh* mesh, ebe_dtype dtype, int32_t nrhs, const void* x_dev, void* y_dev,
                           void* stream);

/* ---- solver ----------------------------------------------------------- */

void ebe_pcg_default_opts(ebe_pcg_opts* opts);

/* Solve P K P u_j = P f_j for nrhs cases (Eq. (2)) with the adaptive CG of
 * Algorithm 1 (or PCGE).  f_dev, u_dev: [n_nodes][3][nrhs] double; u is
 * written (fixed DOFs set to 0).  opts NULL = defaults; stats may be NULL.
 * Synchronises the stream at every convergence check and at exit.
 * Returns EBE_OK, EBE_NOT_CONVERGED (u holds the last iterate),
 * EBE_ERR_BREAKDOWN or EBE_ERR_NONFINITE. */
ebe_status ebe_pcg_solve(ebe_mesh* mesh, int32_t nrhs, const double* f_dev, double* u_dev,
                         const ebe_pcg_opts* opts, ebe_pcg_stats* stats, void* stream);

/* ---- adjoint (extension: inverse analysis, Section 5) ------------------ */

/* Per-element gradient of a misfit with respect to E_e, given the forward
 * states u_c and adjoint states lambda_c (K lambda_c = dL/du_c):
 *   g_e = - sum_c lambda_{c,e}^T (K_e / E_e) u_{c,e}      (K_e is linear in E_e).
 * u_dev, lam_dev: [n_nodes][3][nrhs] of dtype; g_dev: [n_elem] of dtype,
 * overwritten.  No scatter: each element writes its own entry (asynchronous). */
ebe_status ebe_adjoint_grad(ebe_mesh* mesh, ebe_dtype dtype, int32_t nrhs, const void* u_dev,
                            const void* lam_dev, void* g_dev, void* stream);

/* ---- Green's functions of fault slip and their inversion (Section 5) ---- */

typedef struct ebe_fault ebe_fault; /* opaque; a fault and its unit-slip basis on one mesh */

/* A fault for split-node loading (Section 2 cites the split-node technique
 * for the fault) with the unit-slip basis functions of Eq. (4).  Host
 * inputs, copied (synchronous):
 *   sides [n_elem]: +1 / -1 for elements touching a fault node, on the two
 *     sides of the fault; 0 for every other element;
 *   fault_nodes [n_fault_nodes]: the fault's node ids (distinct);
 *   basis [n_fault_nodes][n_basis]: value of basis function i at fault node k;
 *   dirs [n_basis][3]: slip direction (a vector) of basis function i.
 * Slip of basis function i at fault node k: basis[k][i] * dirs[i]; zero at
 * every other node.  The mesh must outlive the fault.  Errors: EBE_ERR_INDEX
 * (node out of range or repeated), EBE_ERR_ARG (a side other than -1/0/1, or
 * an element touching a fault node with side 0), EBE_ERR_NONFINITE. */
ebe_status ebe_fault_create(ebe_mesh* mesh, const int8_t* sides, int64_t n_fault_nodes, const int32_t* fault_nodes,
                            int32_t n_basis, const double* basis, const double* dirs, ebe_fault** out);
void ebe_fault_destroy(ebe_fault* fault);

/* Split-node forces of basis functions col0 .. col0 + nrhs - 1 (nrhs 1..16):
 * a fault node carries two displacements, u+ on the +1 side and u- on the
 * -1 side, with u+ - u- = s; for the mean v = (u+ + u-) / 2 equilibrium
 * gives K v = f on the unsplit mesh with
 *     f = sum_{e, side_e != 0} -(side_e / 2) K_e s_e
 * (s_e: the slip at element e's nodes).  f_dev [n_nodes][3][nrhs] FP64,
 * overwritten (asynchronous).  Away from the fault v is the displacement. */
ebe_status ebe_split_node_forces(ebe_fault* fault, int32_t col0, int32_t nrhs, double* f_dev, void* stream);

/* Green's functions (Eq. (4)): for every basis function i, the displacement
 * at the observation points due to its unit slip:
 *   G_dev[3 s + c][i] = v_i(stations_host[s], component c),
 * G_dev [3 n_stations][n_basis] FP64 row-major, stations_host [n_stations]
 * node ids (host, checked: EBE_ERR_INDEX).  Basis functions are taken in sets of 16 (the
 * paper's case sets): per set the split-node forces, one ebe_pcg_solve with
 * opts (NULL: defaults), and the gather of the station components.  stats:
 * [ceil(n_basis / 16)] per-set solve statistics, or NULL.  Synchronous (the
 * solves are); allocates two [n_nodes][3][16] FP64 vectors with the fault.
 * Returns the worst status of the solves (EBE_NOT_CONVERGED when any set
 * missed tol). */
ebe_status ebe_greens_functions(ebe_fault* fault, int32_t n_stations, const int32_t* stations_host, double* G_dev,
                                const ebe_pcg_opts* opts, ebe_pcg_stats* stats, void* stream);

/* Regularised least squares of Eq. (5) over a list of weights, and the
 * L-curve corner: for each alpha_k (alphas_host[n_alpha], positive,
 * increasing)
 *     a_k = argmin ||G a - d||^2 + alpha_k^2 ||L a||^2,
 * the least-squares solution of the stacked system [G; alpha_k L] a = [d; 0]
 * by Householder QR in FP64; rho_k = ||G a_k - d||, eta_k = ||L a_k||.  With
 * three or more weights: the curvature of the curve (log rho, log eta) as a
 * function of log alpha (derivatives by second-order central differences on
 * the nonuniform grid, first-order one-sided at its two ends) and the index
 * of its largest value (Hansen's L-curve corner; the first one if tied).
 *   G_dev [n_obs][n_basis], d_dev [n_obs], L_dev [n_reg][n_basis] (row-major,
 *   device); a_dev [n_alpha][n_basis]; rho_dev, eta_dev, curvature_dev
 *   [n_alpha]; corner_dev [1] int32 (curvature and corner may be NULL with
 *   fewer than three weights).  n_basis <= 512, n_alpha <= 1024; [G; L]
 *   must have full column rank.  Synchronous; allocates a workspace of
 *   n_alpha (n_obs + n_reg)(n_basis + 1) doubles. */
ebe_status ebe_invert_lcurve(int32_t n_obs, int32_t n_basis, const double* G_dev, const double* d_dev, int32_t n_reg,
                             const double* L_dev, int32_t n_alpha, const double* alphas_host, double* a_dev,
                             double* rho_dev, double* eta_dev, double* curvature_dev, int32_t* corner_dev,
                             void* stream);

/* ---- product forms and the autotuner ------------------------------------ */

/* Time every product form of y = K x (level 0: quadratic mesh, level 1:
 * linear mesh) for (dtype, nrhs) on this mesh, and for GATHER, STAGED,
 * PIPELINED, COLOURED, DETERMINISTIC and ASSEMBLED every kernel variant
 * (ebe_set_product_variant), and keep the
 * fastest for every later product with these
 * parameters (Section 4 tunes its kernels' parameters by hand; here the
 * search is measured on the mesh); ms_out[EBE_NUM_FORMS] (or NULL) receives
 * the times in milliseconds, indexed by form (the faster variant), -1 for a
 * form that does not exist at this level or cannot run on this mesh.
 * Synchronous;
 * allocates temporary vectors.  ebe_pcg_solve tunes the products it uses by
 * itself. */
ebe_status ebe_autotune(ebe_mesh* mesh, int32_t level, ebe_dtype dtype, int32_t nrhs, void* stream,
                        double* ms_out);

/* Force (EBE_FORM_GATHER / _STAGED / _PIPELINED, _COLOURED and
 * _DETERMINISTIC for level 0, _ASSEMBLED for level 1) or reset
 * (EBE_FORM_AUTO) the form used
 * for (level, dtype, nrhs), and read the form that would be used. */
ebe_status ebe_set_product_form(ebe_mesh* mesh, int32_t level, ebe_dtype dtype, int32_t nrhs, int32_t form);
ebe_status ebe_get_product_form(const ebe_mesh* mesh, int32_t level, ebe_dtype dtype, int32_t nrhs,
                                int32_t* form);

/* Kernel variant of a form for (level, dtype, nrhs).  PIPELINED and
 * COLOURED: 0 = element geometry prefetched with the patch metadata and kept
 * in LDS (the default), 1 = read from the geometry cache by each work-item
 * of the element phase.  GATHER and STAGED: 0 = element geometry read from
 * the mesh's geometry cache (the default), 1 = formed at every product from
 * the four corner coordinates (fewer bytes where few cases share an
 * element).  DETERMINISTIC: 0 = shared nodes' partial sums staged and
 * added by a second pass, 1 = patches colour by colour with their sums added
 * straight into y (the colour order is fixed, so still bit-reproducible).
 * ASSEMBLED: the tile, cases per work-item and block slots per trip: FP32
 * 0 = 4 / 4, 1 = 2 / 4, 2 = 8 / 2; FP64 0 = 4 / 1, 1 = 2 / 2, 2 = 1 / 4
 * (cases per work-item reduced to a divisor of nrhs).  Variant 2 exists for
 * ASSEMBLED only; the other forms take it as 0.
 * Same result up to rounding; ebe_autotune sets it,
 * ebe_set_product_form resets it to 0; other forms ignore it. */
ebe_status ebe_set_product_variant(ebe_mesh* mesh, int32_t level, ebe_dtype dtype, int32_t nrhs, int32_t variant);
ebe_status ebe_get_product_variant(const ebe_mesh* mesh, int32_t level, ebe_dtype dtype, int32_t nrhs,
                                   int32_t* variant);

/* ---- batches: many meshes / case sets solved together ------------------ */

/* A batch runs the solves of several meshes, each with its own nrhs (1..16),
 * so that meshes too small to fill the GPU share it (Section 5 solves its
 * case sets one after another).  With ebe_batch_set_merge(batch, max_elems)
 * (default 0: off), meshes of at most max_elems elements are grouped by case count (bands
 * 9-16, 5-8, 3-4, 1-2) into merged block-diagonal meshes of at most 1M
 * elements, built on the first solve from the members' device copies: one
 * solve of a merged mesh runs every product and vector pass as one launch
 * over all its members' element patches (and replays its inner loops as
 * captured HIP graphs).  A member's cases are scaled to unit norm in the
 * merged system, which is solved to tol / sqrt(members), so each member's own
 * relative residual is at most tol; after the solve each member's residual
 * ||P(f - K u)|| / ||P f|| is recomputed with its own operator and reported in
 * its stats (max_rel_res; merged = number of members).  Merged groups and the
 * other meshes are solved several at a time on worker streams, largest
 * first.
 * ebe_batch_create: meshes[n_mesh] distinct handles on one device, nrhs[n_mesh];
 *   the batch keeps the pointers (the meshes must outlive it) and creates its
 *   own worker streams (default priority).
 * ebe_batch_solve: f_dev[i], u_dev[i] are mesh i's [N_i][3][nrhs_i] FP64
 *   vectors; opts as ebe_pcg_solve (NULL: defaults) for every mesh;
 *   stats[n_mesh] or NULL.  Work starts after what is already enqueued on
 *   `stream`; the call returns when every solve has finished (synchronous).
 *   Returns the first error met (the message names the mesh), else
 *   EBE_NOT_CONVERGED if any mesh did not converge, else EBE_OK.  A batch is
 *   used by one thread at a time. */
ebe_status ebe_batch_create(ebe_mesh* const* meshes, int32_t n_mesh, const int32_t* nrhs,
                            ebe_batch** out);
ebe_status ebe_batch_solve(ebe_batch* batch, const double* const* f_dev, double* const* u_dev,
                           const ebe_pcg_opts* opts, ebe_pcg_stats* stats, void* stream);
void ebe_batch_destroy(ebe_batch* batch);
/* Merge meshes of at most max_elems elements (0, the default: merge none);
 * takes effect at the next solve (the merged meshes are rebuilt).  On the
 * serving set of 32 meshes of 5e4..2e6 elements plus one of 6.3M, merged
 * solves measured slower than concurrent separate ones (3.0 s at 150,000
 * against 2.8 s), so merging is an option, not the default. */
ebe_status ebe_batch_set_merge(ebe_batch* batch, int64_t max_elems);
/* Number of merged groups and (group_of [n_mesh] or NULL) each mesh's group,
 * -1 for a mesh solved on its own; plans the groups if no solve has yet
 * (synchronous). */
ebe_status ebe_batch_info(ebe_batch* batch, int32_t* n_groups, int32_t* group_of);

/* ---- diagnostics ------------------------------------------------------- */

const char* ebe_status_string(ebe_status status);
const char* ebe_last_error(void);   /* thread-local detail of the last failure */
const char* ebe_build_info(void);   /* target architecture and build flags */

#ifdef __cplusplus
}
#endif

#endif /* EBE_H */
