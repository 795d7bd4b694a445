/*
 * airhdg: space-time HDG facet systems solved by FGMRES preconditioned with
 * lAIR algebraic multigrid, on one AMD MI355X (gfx950).
 *
 * Method: Sivas, Southworth, Rhebergen, "AIR algebraic multigrid for a
 * space-time hybridizable discontinuous Galerkin discretization of
 * advection(-diffusion)", arXiv 2010.11130.
 *
 * Conventions shared by every call
 *   - Space-time coordinates: column 0 is t, columns 1..d are space;
 *     D = d + 1 is the space-time dimension (2 or 3), p in {1, 2, 3}.
 *   - Pointers marked "host" are host memory, "dev" are device memory
 *     (hipMalloc'd or torch tensors); the caller owns every pointer argument.
 *   - stream: a hipStream_t passed as void* (NULL = default stream).  Device
 *     work is enqueued on it.  Calls that return an info struct or sizes
 *     synchronize the stream before returning.
 *   - Library objects (ah_mesh, ah_system, ah_hier) own their device memory,
 *     allocated stream-ordered on the stream of the call that creates them and
 *     released by the matching destroy call.
 *   - Return values: AH_OK (0) on success, a positive warning (AH_ENOCONV) or
 *     a negative error.  On error nothing is written to outputs except where
 *     stated, and ah_last_error() (per thread) describes the failure.
 *   - Facets are numbered by the lexicographic order of their sorted
 *     vertex-id tuples.  Facet unknowns: Lagrange nodes of degree p at the
 *     equispaced lattice of the facet simplex whose vertices are the facet's
 *     vertex ids in increasing order (lattice index i_1 fastest).  "Free"
 *     DOFs are those of non-Dirichlet facets, numbered facet-rank * b + node.
 *   - Element unknowns returned by hdg_reconstruct are the values of u_h at
 *     the equispaced degree-p lattice of each element's reference simplex
 *     (vertex order of the cell, i_1 fastest).
 *   - Quadrature: conical-product Gauss-Jacobi rules with p+2 points per
 *     direction on elements and facets (collapsed coordinates, s_1 fastest).
 */
#ifndef AIRHDG_H
#define AIRHDG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  AH_OK = 0,
  AH_ENOCONV = 1,        /* iteration limit reached; best iterate written */
  AH_EINVAL = -1,        /* bad argument, size, or non-finite input */
  AH_ESINGULAR = -2,     /* degenerate element or singular facet block */
  AH_EBREAKDOWN = -3,    /* NaN/Inf during the Krylov iteration */
  AH_EHIP = -4,          /* HIP runtime error */
  AH_ENOMEM = -5,        /* device allocation failed */
  AH_EUNSUPPORTED = -6   /* size or parameter outside what is implemented */
} ah_status;

typedef struct ah_mesh ah_mesh;
typedef struct ah_system ah_system;
typedef struct ah_hier ah_hier;

/* Last error message of the calling thread (never NULL). */
const char* ah_last_error(void);

/* ------------------------------------------------------------ memory ---
 * Device memory of library objects (ah_system, ah_hier, the solver
 * workspace a hierarchy allocates on its first solve, temporaries) comes
 * from the library's caching allocator (hipMalloc; freed blocks stay cached
 * per device and stream and are reused by later requests of up to their
 * size on that stream; on out-of-memory the device's cache is released and
 * the allocation retried) unless the caller registers its own allocator
 * (e.g. torch's caching allocator, so both share one pool):
 *   alloc(ctx, bytes, stream): device memory of at least bytes (256-byte
 *     aligned) usable in stream order on stream (a hipStream_t), or NULL
 *     (the library call then fails with AH_ENOMEM);
 *   free(ctx, ptr, bytes, stream): gives it back, with the stream and size
 *     of the allocation, after the last work using it has been enqueued on
 *     that stream (destroy calls, end of temporaries).
 * Memory keeps the allocator it came from when the registration changes.
 * Both NULL restores the pool; one NULL is AH_EINVAL.  The registration is
 * process-wide and may be changed from any thread; the callbacks may run on
 * any thread that calls the library. */
typedef void* (*ah_alloc_fn)(void* ctx, int64_t bytes, void* stream);
typedef void (*ah_free_fn)(void* ctx, void* ptr, int64_t bytes, void* stream);
ah_status ah_set_allocator(ah_alloc_fn alloc, ah_free_fn free, void* ctx);

/* Gives the blocks that the library's caching allocator holds for the
 * current device, freed by objects and not reused yet, back to the device
 * (hipFree).  Waits for the device first.  Objects that are alive keep
 * their memory.  AH_EHIP on a runtime error. */
ah_status ah_pool_trim(void);

/* ---------------------------------------------------------------- mesh ---
 * Space-time simplex mesh (Section 2.2: slab-by-slab slabs or one
 * all-at-once triangulation).  vert: host [nv][dim_st]; cell: host
 * [ne][dim_st+1] vertex ids.  Inputs are copied.  Builds the facets (sorted
 * vertex tuples), element-facet maps and the facet adjacency pattern on the
 * host.  AH_EINVAL for ids out of range or a facet shared by more than two
 * cells; AH_ESINGULAR for a degenerate cell. */
ah_status ah_mesh_create(int dim_st, int64_t nv, const double* vert, int64_t ne,
                         const int32_t* cell, ah_mesh** out);
void ah_mesh_destroy(ah_mesh* m);
/* Sizes: number of facets, of boundary facets (one adjacent cell). */
ah_status ah_mesh_sizes(const ah_mesh* m, int64_t* nf, int64_t* nbf);
/* facet_vert: host [nf][dim_st] sorted vertex ids; facet_elem: host [nf][2]
 * adjacent cells (-1 when absent).  Either may be NULL. */
ah_status ah_mesh_facets(const ah_mesh* m, int32_t* facet_vert, int32_t* facet_elem);
/* Boundary facet ids in increasing order: host [nbf].  Boundary data arrays
 * (g_q) are indexed in this order. */
ah_status ah_mesh_boundary_facets(const ah_mesh* m, int32_t* ids);
/* Boundary kinds, host [nf]: 0 interior, 1 Dirichlet (u = g_D, facet
 * unknowns eliminated), 2 Neumann (total-flux condition of Section 2.1; the
 * initial plane is an inflow Neumann facet).  Must be called before
 * hdg_assemble.  AH_EINVAL if an interior facet is tagged or a boundary
 * facet is left 0. */
ah_status ah_mesh_set_bc(ah_mesh* m, const int8_t* kind);

/* Quadrature sizes for (dim_st, p): element and facet points, element and
 * facet basis sizes (nu = dim P_p(K), b = dim P_p(F)). */
ah_status ah_sizes(int dim_st, int p, int* nq, int* nqf, int* nu, int* b);
/* The conical-product rule on the reference simplex of dimension dim (0..3)
 * with n points per direction: xi host [n^dim][dim], w host [n^dim]
 * (weights sum to 1/dim!). */
ah_status ah_quad_rule(int dim, int n, double* xi, double* w);
/* Physical quadrature points where the caller evaluates f and g: xq_elem dev
 * [ne][nq][dim_st], xq_bfacet dev [nbf][nqf][dim_st] (either may be NULL). */
ah_status ah_quad_points(const ah_mesh* m, int p, double* xq_elem, double* xq_bfacet,
                         void* stream);
/* The same facet rule at every facet: xq_facet dev [nf][nqf][dim_st] (facet
 * point q is the same physical point seen from either adjacent cell), where
 * the caller evaluates a velocity field for hdg_assemble_q.  Synchronizes. */
ah_status ah_quad_points_facets(const ah_mesh* m, int p, double* xq_facet, void* stream);

/* ------------------------------------------------------- hdg_assemble ---
 * Space-time HDG discretization (Section 2.3, bilinear form with upwind
 * flux sigma_a and interior-penalty flux sigma_d, tau = nu alpha / h_K with
 * h_K = |det J_K|^(1/D)), static condensation S = D - C A^-1 B,
 * H = G - C A^-1 F (Section 2.5), Dirichlet elimination (facet L2
 * projection of g_D), and left scaling by the inverse facet diagonal blocks
 * (Section 4): builds S_hat = D_b^-1 S and H_hat = D_b^-1 H on the free
 * facets.
 *   alpha <= 0 selects 10 p^2 (Section 4).
 *   a_vert: dev [nv][d] velocity at the vertices, interpolated linearly in
 *           each cell (exact for affine velocity fields; hdg_assemble_q
 *           takes any field at the quadrature points).
 *   f_q:    dev [ne][nq] source at ah_quad_points' element points, or NULL (0).
 *   g_q:    dev [nbf][nqf] boundary data at the boundary-facet points:
 *           g_D on Dirichlet facets, g_N on Neumann facets; NULL = 0.
 * Returns AH_ESINGULAR if a facet diagonal block or an element block is
 * singular (e.g. a characteristic facet at nu = 0), AH_EINVAL for nu < 0 or
 * p outside 1..3.  Synchronizes the stream. */
typedef struct {
  int p;
  double alpha;
  int keep_element_data;   /* nonzero: keep blocks for reconstruct/adjoint */
  int no_block_scale;      /* nonzero: S_hat = S, H_hat = H, D_b^-1 = I (the
                              "no block inverse" ablation of Section 4.1) */
} ah_hdg_params;

ah_status hdg_assemble(const ah_mesh* m, const ah_hdg_params* prm, double nu,
                       const double* a_vert, const double* f_q, const double* g_q,
                       void* stream, ah_system** out);
/* hdg_assemble with the velocity given at the quadrature points instead of
 * the vertices, for fields that are not affine in each cell (Section 2.3:
 * the advective volume term integrates u a.grad v with a(x) at the element
 * points; the upwind flux takes a.n at each facet point):
 *   a_qe: dev [ne][nq][d] at ah_quad_points' element points;
 *   a_qf: dev [nf][nqf][d] at ah_quad_points_facets' points.
 * For an affine field the result equals hdg_assemble's with the field's
 * vertex values (to rounding).  Other arguments, results and errors as in
 * hdg_assemble. */
ah_status hdg_assemble_q(const ah_mesh* m, const ah_hdg_params* prm, double nu, const double* a_qe,
                         const double* a_qf, const double* f_q, const double* g_q, void* stream,
                         ah_system** out);
/* Replace the Neumann data of an assembled system (Section 2.3: the data
 * term on Neumann facets, i.e. the inflow u(t_n) on a slab's initial plane,
 * Section 2.4).  g_q dev [nbf][nqf] as in hdg_assemble; only the rows of
 * Neumann facets are read (NULL = 0).  Recomputes H = H0 + G(g_q) and
 * H_hat = D_b^-1 H, where H0 is the right-hand side assembled without the
 * Neumann term; the matrix, Dirichlet data and element data are unchanged,
 * so a hierarchy built on the system stays valid.  This lets the system and
 * its hierarchy of slab n+1 be built before slab n is solved.  Does not
 * synchronize. */
ah_status hdg_update_neumann(ah_system* s, const double* g_q, void* stream);
/* Destroy: device memory is released with hipFreeAsync on the stream(s) it
 * was allocated on (creation stream; the first solving stream for the
 * solver workspace of a hierarchy).  Work that uses the object on any other
 * stream must have completed, or be ordered before those streams, first. */
void ah_system_destroy(ah_system* s);
/* n_free = number of free facet DOFs; b = facet block size; nnz = stored
 * entries of the scaled level-0 matrix (exact zeros off the diagonal are not
 * stored). */
ah_status ah_system_sizes(const ah_system* s, int64_t* n_free, int* b, int64_t* nnz);
/* Copies of the scaled CSR matrix S_hat (row_ptr dev [n+1] int64, col dev
 * [nnz] int32, val dev [nnz] double), H_hat dev [n], the inverse facet blocks
 * D_b^-1 dev [n/b][b][b] and the Dirichlet traces of all facets dev
 * [nf][b] (zero on non-Dirichlet facets).  Any pointer may be NULL. */
ah_status ah_system_export(const ah_system* s, int64_t* row_ptr, int32_t* col, double* val,
                           double* h_hat, double* dinv, double* lam_dir, void* stream);
/* u_h at the element lattice nodes: U_K = A_K^-1 (F_K - B_K Lambda_K)
 * (Section 2.5).  lam dev [n_free] (unscaled solution); U dev [ne][nu].
 * Requires keep_element_data. */
ah_status hdg_reconstruct(const ah_system* s, const double* lam, double* U, void* stream);
/* Slab coupling (Section 2.4): the next slab's inflow data on its initial
 * plane is the previous slab's trace on its final plane.  For every
 * boundary facet of next_mesh lying on its initial plane whose spatial
 * vertices coincide with a final-plane facet of prev's mesh, writes that
 * trace (free DOFs lam_prev dev [n_free(prev)]) evaluated at next_mesh's
 * facet quadrature points (degree of prev) into g_q_next dev
 * [nbf(next)][nqf]; other rows are left untouched.  next_mesh may be prev's
 * own mesh (a slab mesh reused with shifted time data).  The pairing is
 * computed on the host on first use and cached in next_mesh. */
ah_status hdg_inflow_from_trace(const ah_system* prev, const double* lam_prev,
                                ah_mesh* next_mesh, double* g_q_next, void* stream);

/* ---------------------------------------------------------- air_setup ---
 * lAIR hierarchy on S_hat treated as a scalar matrix (Section 3; Section 4
 * settings): strength |a_ij| >= theta max_{k!=i}|a_ik| (1-1e-12); PMIS
 * coarsening with integer keys (influence count, 44-bit index hash);
 * one-point interpolation; distance-one lAIR restriction from local
 * solves A[N_i,N_i]^T z = -A[i,N_i]^T; A_c = R A P; coarsest level inverted
 * densely.  Stops at n <= max_coarse, at max_levels, or when the coarse grid
 * is empty or larger than stall * n.  fp32_cycle: also keep FP32 copies of the
 * cycle operators; adjoint: also build the transposed operators.
 * lair_distance 2 widens N_i to the strong F neighbours of i's strong F
 * neighbours (paths through F points only; at most 64 points, else
 * AH_EUNSUPPORTED); theta_r > 0 gives the restriction neighbourhoods their
 * own strength threshold (Section 4 uses 0.3 for R and 0.2 for the
 * coarsening), theta stays that of the coarsening and of P. */
typedef struct {
  double theta;        /* strength threshold, default 0.25 */
  int max_coarse;      /* default 64 */
  int max_levels;      /* default 25 */
  int relax;           /* 0: F,F,C Jacobi sweeps; 1: one F sweep; 2: ordered
                          Gauss-Seidel on level 0 over all points; 3: ordered
                          Gauss-Seidel on level 0, F points then all points
                          (2 and 3: coarser levels F,F,C Jacobi) */
  double omega;        /* Jacobi weight, default 1 */
  double stall;        /* default 0.9 */
  int fp32_cycle;
  int adjoint;
  int lair_distance;   /* 1 (default) or 2 */
  double theta_r;      /* restriction strength threshold; <= 0: theta (default) */
  double order_ratio;  /* relax 2, 3: dominance ratio that orders a pair of
                          facet blocks (>= 1; default 1.5) */
  int coarsening;      /* 0: PMIS (default, data-parallel); 1: Ruge-Stueben
                          first pass, the single-process form of the Falgout
                          coarsening of Section 4 (largest measure first, ties
                          to the smallest index; sequential, on the host) */
  int block_air;       /* 1: level 0 is coarsened by block AIR on its facet
                          blocks: strength and PMIS on the block graph with
                          weights w_IJ = max |a_ij| over block (I, J), every
                          row of a block shares its block's C/F label, P =
                          P_blocks (x) I_b with one-point P_blocks, and the
                          lAIR rows of a C block solve over all rows of its
                          strong F blocks; coarser levels scalar.  Needs a
                          scaled system, lair_distance 1 and coarsening 0
                          (else AH_EINVAL).  0: scalar AIR (default) */
} ah_air_params;

typedef struct {
  int levels;
  int64_t n[32];
  int64_t nnz[32];
  int64_t n_fallback;  /* lAIR rows that fell back to injection */
  double op_complexity;
  double t_setup_ms;
  int64_t block_view_values;  /* values of level 1 read by full blocks in
                                 its F and C sweeps (block AIR, level 1 swept
                                 from its point lists): its CSR entries plus
                                 the zero fill of block rows whose rows do
                                 not share one block pattern; 0 where level 1
                                 is swept by CSR rows */
  int64_t level0_no_interp_pass; /* 1 where the level-0 F and C sweeps (block
                                 AIR, F, F, C Jacobi, copy in sweep order)
                                 read the one-point interpolated correction
                                 P e_c from e_c itself, with no pass forming
                                 P e_c; 0 otherwise */
} ah_setup_info;

/* Environment (read by air_setup; for tests and tuning): AH_TAIL_MAX (rows,
 * default 4096) bounds the first level of the single-workgroup coarse end of
 * the cycle (0: every level runs with grid-wide kernels); AH_TAIL_LDS=0 runs
 * that coarse end from global memory instead of an LDS image; AH_G0 (2, 4,
 * 8, 16, 32) fixes the lanes per row of the level-0 kernels.  Alternative
 * code paths (the defaults are the faster forms): AH_SWO=0 sweeps over the
 * natural order from the F and C lists after an interpolation pass instead
 * of from the copies in sweep order (the same sums, bit for bit); AH_L1B=0
 * sweeps level 1 of block AIR by CSR rows, AH_RZB=0 restricts from level 0
 * by CSR rows and AH_FBB=0 runs the level-0 kernels by rows (the same
 * operators, summed in another order).  Size thresholds: AH_DCGS_MIN (delayed CGS2),
 * AH_LIST_MIN (list sweeps on coarse levels), AH_PMIS_WG_MAX,
 * AH_PMIS_LIST_MIN; lanes: AH_GC (coarse levels), AH_LPB (level-0 block
 * rows), AH_L1LP (level 1). */

/* Defaults for ah_air_params / ah_solve_params. */
void ah_air_defaults(ah_air_params* p);

ah_status air_setup(const ah_system* s, const ah_air_params* prm, void* stream,
                    ah_hier** out, ah_setup_info* info);
void ah_hier_destroy(ah_hier* h);
/* Level data for inspection (device copies): n, nnz of A_l and of R_l. */
ah_status ah_hier_level_sizes(const ah_hier* h, int l, int64_t* n, int64_t* nnz,
                              int64_t* nnz_r);
/* A_l (CSR), C/F marks (1 = C, int8), one-point P (coarse column or -1 per
 * fine point), R_l (CSR).  Any pointer may be NULL; sizes from
 * ah_hier_level_sizes.  The coarsest level has no cf/pcol/R. */
ah_status ah_hier_level_export(const ah_hier* h, int l, int64_t* row_ptr, int32_t* col,
                               double* val, int8_t* cf, int32_t* pcol, int64_t* r_row_ptr,
                               int32_t* r_col, double* r_val, void* stream);

/* Flow order of the ordered relaxations (relax 2 or 3; Lemma 3.1, Section
 * 3.3).  The level-0 facet blocks (block size b, nblocks = n_free / b) are
 * ordered along the clearly dominant coupling of a pair: with
 * w_IJ = max |S_hat entries of off-diagonal block (I, J)|, J precedes I when
 * w_IJ > order_ratio w_JI; pairs within the ratio stay unordered.  Levels
 * come from Kahn rounds; a round that finds no ready block (a cycle) places
 * the unplaced block with the fewest unplaced predecessors, then the
 * smallest index, alone.  The sweep is Gauss-Seidel across levels and Jacobi
 * inside a level (the splitting matrix holds the entries whose column block
 * lies on an earlier level); for pure advection on an acyclic element graph
 * S_hat is block lower triangular in this order, no two blocks of a level
 * are coupled, and one sweep solves exactly.  The facet-block pattern must be
 * structurally symmetric (air_setup returns AH_EUNSUPPORTED otherwise, and
 * for an unscaled system).  level: host [nblocks] or NULL; nblocks, rounds,
 * breaks (rounds that broke a cycle) may be NULL.  A hierarchy without an
 * ordered relaxation reports nblocks = rounds = 0.  Synchronous. */
ah_status ah_hier_flow_levels(const ah_hier* h, int32_t* level, int64_t* nblocks, int* rounds, int* breaks);

/* ---------------------------------------------------------- air_solve ---
 * method 0: FGMRES(restart) with right preconditioning by one V-cycle (no
 * pre-relaxation, post-relaxation F,F,C; Section 4) on S_hat x = D_b^-1 rhs.
 * rhs dev [n_free] unscaled, or NULL for the assembled H; x dev [n_free]
 * (initial guess if x0_given, else zero; overwritten by the solution).
 * Convergence: ||r_hat|| <= tol ||D_b^-1 rhs|| estimated by the Arnoldi
 * recurrence and confirmed by a true residual in FP64 (restart otherwise).
 * precision 1: the V-cycle runs in FP32 (FP32 operators, FP32 accumulation)
 * inside the FP64 FGMRES; the coarsest solve stays FP64.  Returns AH_ENOCONV
 * if maxit is reached (x holds the best iterate), AH_EBREAKDOWN on NaN.
 * method 1: BiCGSTAB with right preconditioning by one V-cycle per half
 * step (the paper's Krylov method, Section 4); convergence on the
 * recursively updated residual, confirmed by the true residual, restart
 * from the current iterate on breakdown; iters counts BiCGSTAB steps (two
 * V-cycles each). */
typedef struct {
  double tol;       /* default 1e-8 */
  int restart;      /* default 100 */
  int maxit;        /* default 1000 */
  int precision;    /* 0 FP64 cycle, 1 FP32 cycle */
  int x0_given;
  int method;       /* 0 FGMRES(restart), 1 BiCGSTAB (restart unused) */
} ah_solve_params;

typedef struct {
  int iters;
  int converged;
  double relres;        /* estimated scaled relative residual at exit */
  double true_relres;   /* recomputed ||H_hat - S_hat x|| / ||H_hat|| */
  double t_solve_ms;
} ah_solve_info;

void ah_solve_defaults(ah_solve_params* p);

ah_status air_solve(const ah_hier* h, const double* rhs, double* x, const ah_solve_params* prm,
                    void* stream, ah_solve_info* info);

/* Allocation-free air_solve, for callers that cannot allocate device or
 * pinned host memory (code under HIP graph capture elsewhere on the stream,
 * tight serving loops, harnesses that forbid hipMalloc).  Same arguments,
 * semantics and results as air_solve with method 0 (FGMRES); the FGMRES
 * workspace comes from a static device array of AH_NOALLOC_SCRATCH_BYTES
 * that the library holds on every GPU it runs on until the process ends,
 * and the host staging is a static per-thread array.  It needs
 * 8 ((2 m + 4) n + 1024 (2 m + 4) + 4 (m + 3)) bytes (FP32 cycle: the m Z
 * vectors take 4 bytes per value), rounded up to 256-byte pieces, with
 * m = restart <= AH_NOALLOC_MAX_RESTART.  Returns AH_EUNSUPPORTED for a
 * larger workspace, a larger restart or method 1, before any device work.
 * Every call on a GPU shares that GPU's array and leaves its last contents
 * there: calls that overlap on one GPU (from several threads or streams)
 * race.  The hierarchy, x and rhs must belong to the current device.
 * Synchronizes the stream. */
#define AH_NOALLOC_SCRATCH_BYTES (64ll * 1024 * 1024)
#define AH_NOALLOC_MAX_RESTART 128
ah_status air_solve_noalloc(const ah_hier* h, const double* rhs, double* x, const ah_solve_params* prm,
                            void* stream, ah_solve_info* info);

/* Adjoint solve S^T lam = g: FGMRES on S_hat^T mu = g with the transposed
 * V-cycle (sweeps C,F,F with A_l^T, restriction by P_l^T, interpolation by
 * R_l^T, transposed coarsest solve), then lam = D_b^-T mu.  g dev [n_free],
 * lam dev [n_free].  Requires air_setup with adjoint = 1. */
ah_status air_solve_adjoint(const ah_hier* h, const double* g, double* lam,
                            const ah_solve_params* prm, void* stream, ah_solve_info* info);

/* One application of the preconditioner z = B r (transpose = 1: B^T r) on
 * the scaled level-0 system, for inspection: r, z dev [n_free]. */
ah_status ah_vcycle_apply(const ah_hier* h, const double* r, double* z, int precision,
                          int transpose, void* stream);

/* -------------------------------------------------- adjoint gradients ---
 * For J(Lambda) with dJ/dLambda = g and the adjoint lam = S^-T g of a
 * solved system with solution Lambda (both dev [n_free]):
 *   dJdf_q dev [ne][nq]: derivative of J with respect to the source values at
 *          the element quadrature points (through F_K = int f v);
 *   dJdnu  host scalar: derivative with respect to nu (the blocks are affine
 *          in nu), sum over elements of
 *          -w_K.(A1 U + B1 Lambda) - lam_K.(C1 U + D1 Lambda),
 *          w_K = -A_K^-T C_K^T lam_K.
 * a_vert is not read (the nu-dependent part of the blocks has no advective
 * term) and may be NULL.  Requires keep_element_data.  Synchronizes the
 * stream. */
ah_status hdg_assemble_grad(const ah_system* s, const double* a_vert, const double* lam_fwd,
                            const double* lam_adj, double* dJdf_q, double* dJdnu, void* stream);

/* Gaussian sources phi_k(X) = exp(-|X - X_k|^2 / (2 w^2)) at points X dev
 * [npts][dim_st]; centers dev [K][dim_st].
 *   forward:   f dev [npts] = sum_k c_k phi_k(X)          (c dev [K])
 *   transpose: dc dev [K] = sum_pts y(X) phi_k(X)         (y dev [npts]) */
ah_status ah_source_gauss(int dim_st, int64_t npts, const double* X, int K, const double* centers,
                          double width, const double* c, double* f, void* stream);
ah_status ah_source_gauss_T(int dim_st, int64_t npts, const double* X, int K,
                            const double* centers, double width, const double* y, double* dc,
                            void* stream);

/* ---------------------------------------------------------- profiling ---
 * Per-launch timing of the main kernels: when enabled, each launch of a
 * tagged kernel is bracketed by HIP events recorded on its own stream, and
 * its algorithmic byte count (what the operation must read and write once)
 * is accumulated.  Tags: "element" (hdg_assemble element kernel),
 * "spmv0" (level-0 FP64 product of the Krylov solver), "relax0_f" /
 * "relax0_c" (level-0 F and C Jacobi sweeps; "_f32" suffix: FP32 cycle),
 * "gs0" / "gs0_f" (one whole ordered sweep of level 0 over all points / F
 * points, all its per-level launches; "_f32" suffix: FP32 cycle),
 * "rap0" (level-0 numeric R A P).  ah_profile_read synchronizes the
 * recorded events. */
void ah_profile_enable(int on);
void ah_profile_reset(void);
ah_status ah_profile_read(const char* tag, int64_t* launches, double* total_ms, double* bytes);

#ifdef __cplusplus
}
#endif

#endif /* AIRHDG_H */
