/*
 * pff.h - C ABI of the MI355X (gfx950) matrix-free phase-field Jacobian
 * library.
 *
 * Method: Kolditz & Wick, "Matrix-Free Geometric Multigrid Preconditioning of
 * Combined Newton-GMRES for Solving Phase-Field Fracture with Local Mesh
 * Refinement". The library applies the linearised, active-set-masked
 * Jacobian of the 2-D displacement / phase-field system (Sec. 3.1) matrix-free
 * on quadtree meshes with hanging nodes (Q1 or Q2, Sec. 3.3), preconditions it
 * with one local-smoothing geometric-multigrid V-cycle per diagonal block
 * (Chebyshev-Jacobi smoothing, Sec. 3.2), solves with left-preconditioned
 * GMRES (Sec. 3.2, Table 1) and performs primal-dual active set / line-search
 * Newton iterations (Alg. 2). It also offers the transposed operator, the
 * parameter derivatives of the residual and the crack-volume functional of
 * Sec. 4 for adjoint gradients.
 *
 * Conventions (all entry points):
 *  - Vectors are DEVICE pointers owned by the caller; the library never frees
 *    them. Nodal vectors hold 3 components blocked: [u_x(n) | u_y(n) | phi(n)],
 *    double precision unless an argument says fp32. Node order is the
 *    library's own; pff_node_coords exports the integer lattice position of
 *    every node so that callers can map values by position.
 *  - Host pointers are marked "host".
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream). Work is
 *    enqueued on it; entry points that need scalars on the host (set_state
 *    with multigrid setup, gmres_solve, newton_step, tcv, param_grad, dot
 *    products) synchronise that stream before returning.
 *  - Constrained unknowns: u on the domain boundary (Dirichlet, u in H^1_0,
 *    Sec. 2), hanging nodes (interpolated from the coarse face), and phase-field
 *    unknowns in the active set. The operators have identity rows and columns
 *    there (dst_i = src_i).
 *  - Return value: 0 on success; negative on error (PFF_E_*), with text from
 *    pff_last_error; positive PFF_W_* when an iteration did not converge
 *    (results are still written). Iterations check their norms and
 *    Gram-Schmidt coefficients: a NaN or infinity (e.g. from a non-finite
 *    input) stops them with PFF_E_NONFINITE.
 *  - Device memory of a context: its mesh, tile and transfer tables and a few
 *    KB of scalars are allocated by pff_create; its work buffers live in a
 *    caller-owned workspace (pff_bind_workspace) or, without one, are
 *    allocated on first use. pff_destroy frees what the library allocated.
 *  - A context is not thread-safe; calls on one context must not overlap.
 */
#ifndef PFF_H_
#define PFF_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PFF_OK 0
#define PFF_E_ARG (-1)      /* invalid argument or size */
#define PFF_E_STATE (-2)    /* call needs a state (pff_set_state) first */
#define PFF_E_HIP (-3)      /* HIP runtime error */
#define PFF_E_MESH (-4)     /* mesh construction failed */
#define PFF_E_NOMEM (-5)    /* device allocation failed */
#define PFF_E_NONFINITE (-6) /* a norm or reduction of an iteration came out NaN or infinite */
#define PFF_W_NOCONV 1      /* GMRES reached its iteration limit */
#define PFF_W_LINESEARCH 2  /* no line-search trial decreased the residual */

typedef struct pff_ctx pff_ctx;

/* Mesh of (-10,10)^2 (Sec. 4, Table 1): an n_base x n_base uniform mesh
 * reached from a coarse x coarse grid by global refinement, then n_local
 * passes refining every cell whose centre lies strictly inside
 * |x| < band_x, |y| < band_y, then 2:1 face balancing. degree = 1 (Q1) or
 * 2 (Q2). tile_x, tile_y: cells per tile along x and y, at most 256 cells
 * per tile (0 = default: 16 x 16 for Q1, 8 x 8 for Q2). mg_global != 0 also
 * builds the levels of global-coarsening multigrid (each level the quadtree
 * cut off at one depth, a complete mesh with its own hanging nodes; the
 * uniform levels up to the base mesh are shared with local smoothing, the
 * finest is the leaf mesh), which pff_params.mg_kind = 1 selects. */
typedef struct {
  int32_t n_base, n_local, degree, coarse;
  double band_x, band_y;
  int32_t tile_x, tile_y;
  int32_t mg_global;
} pff_mesh_spec;

/* Material and solver parameters.
 *  E, nu: Young's modulus and Poisson ratio (plane strain Lame parameters);
 *  Gc: critical energy release rate; pressure: p; kappa: regularisation;
 *  ell: phase-field length scale l (Sec. 2, Table 1).
 *  cheb_degree: Chebyshev updates per smoothing step; smooth_range (0.08) and
 *  upper_factor (1.2): smoothing interval [smooth_range, upper_factor] *
 *  lambda_max (Sec. 3.2); eig_cg_its: CG steps of the displacement block's
 *  eigenvalue estimate on levels > 0 (1..200, else PFF_E_ARG; default 20:
 *  with 10, the estimate of the finest level's displacement block stays up
 *  to 37 % below lambda_max once a crack of stiffness kappa ~ 1e-12 h is
 *  present, beyond the 1.2 safety factor, and the smoother amplifies the top
 *  of the spectrum); eig_cg_its_phi: the same for the phase-field block
 *  (1..200; default 10: within 3 % of lambda_max on every level of the
 *  paper's meshes, inside the safety factor);
 *  coarse_mode 0: Chebyshev over [lambda_min, upper_factor * lambda_max] on
 *  level 0 with coarse_its updates (Sec. 3.2); coarse_mode 1: coarse_its
 *  Jacobi-preconditioned CG steps from zero on level 0, each block with its
 *  own scalars (a fixed number of steps, so the cycle is reproducible; it is
 *  not a linear operator). Either runs in one kernel when level 0 fits one
 *  workgroup (at most 256 cells) and coarse_its <= 64, else step by step;
 *  the results agree to rounding. coarse_eig_its: CG steps for the level-0
 *  estimate (1..200).
 *  gmres_restart, gmres_max_its, gmres_rtol, gmres_atol: GMRES(m) stops when
 *  the preconditioned residual is below max(atol, rtol * |rhs|) (Table 1).
 *  ls_omega, ls_max: line-search damping omega and l_max (Alg. 2).
 *  vcycle_fp32: 1 = the V-cycle inside gmres_solve/newton_step runs in FP32.
 *  pdas_c: the active-set constant c of Sec. 2 (an unknown is active when
 *  lambda + c (phi - phi_old) > 0). 0 (default) takes the per-unknown choice
 *  c_i = 2 |lambda_i / (phi_i - phi_old_i)| (Sec. 2, with c_i * 0 := 0); a
 *  positive value is used as one constant for every unknown (the paper notes
 *  c may be chosen freely). Negative or non-finite: PFF_E_ARG.
 *  mg_kind: the multigrid of the block preconditioner. 0 (default): local
 *  smoothing (Sec. 3.2: level l holds the cells of refinement level l, the
 *  refinement edge fixed during smoothing). 1: global coarsening (every level
 *  a complete mesh, the quadtree cut at one depth, smoothed over all its
 *  unknowns with its own hanging-node constraints; transfers interpolate the
 *  coarse finite-element function; a coarse phase-field unknown is active if
 *  any finer unknown its interpolation reaches is). 1 needs a context created
 *  with pff_mesh_spec.mg_global != 0, else PFF_E_ARG.
 *  prec_kind: 0 (default): the block-diagonal preconditioner of Sec. 3.2 (one
 *  V-cycle per diagonal block; the coupling block G_phi,u dropped). 1: block
 *  triangular, keeping G_phi,u (the Jacobian is lower block triangular, since
 *  the u-equation uses phi~): forward substitution x_u = M_u^-1 b_u,
 *  x_phi = M_phi^-1 (b_phi - G_phi,u x_u), and for transposed solves the
 *  backward form; two V-cycles and one operator application per use. */
typedef struct {
  double E, nu, Gc, pressure, kappa, ell;
  int32_t cheb_degree;
  double smooth_range, upper_factor;
  int32_t eig_cg_its;
  int32_t coarse_mode;
  int32_t coarse_its;
  int32_t coarse_eig_its;
  int32_t gmres_restart, gmres_max_its;
  double gmres_rtol, gmres_atol;
  double ls_omega;
  int32_t ls_max;
  int32_t vcycle_fp32;
  double pdas_c;
  int32_t mg_kind;
  int32_t prec_kind;
  int32_t eig_cg_its_phi;
} pff_params;

typedef struct {
  int32_t iterations;     /* GMRES iterations (Arnoldi steps) */
  int32_t converged;      /* 1 if the tolerance was met */
  double initial_residual;   /* |P^{-1} b| */
  double final_residual;     /* preconditioned residual estimate at exit */
  double tolerance;
} pff_gmres_info;

typedef struct {
  double residual_before;  /* |R~(U)| with the new active set */
  double residual_after;   /* |R~| at the accepted trial */
  double rhs_norm;         /* |R~(U_c)|: right-hand side of the linear system */
  int32_t gmres_iterations;
  int32_t gmres_converged;
  int32_t ls_trials;
  int64_t n_active;
  int64_t active_changed;  /* entries that differ from the active set passed in */
  double setup_seconds, solve_seconds, linesearch_seconds;
} pff_newton_info;

/* Fill *p with the defaults listed above (Table 1 values for the Sneddon test,
 * ell = 0.1). Returns PFF_OK. */
int pff_default_params(pff_params* p);

/* Build the mesh, tile tables and multigrid levels on the host and upload
 * them to the current HIP device. The context owns those device tables; its
 * work vectors come from a bound workspace (pff_bind_workspace) or are
 * allocated on first use. Errors: PFF_E_ARG (invalid parameters: see
 * pff_params; also gmres_max_its < 1, ls_max < 1, ls_omega outside (0, 1]),
 * PFF_E_MESH, PFF_E_NOMEM, PFF_E_HIP; *out stays NULL, whatever was already
 * uploaded is freed, and pff_last_error(NULL) returns the reason (text of the
 * last failed pff_create on the calling thread). */
int pff_create(const pff_mesh_spec* spec, const pff_params* params, pff_ctx** out);
int pff_destroy(pff_ctx* ctx);
/* Replace material/solver parameters (takes effect at the next set_state). */
int pff_set_params(pff_ctx* ctx, const pff_params* params);

/* Device memory for the context's work buffers, to be owned by the caller
 * (e.g. a torch uint8 tensor): the leaf state copies and work vectors (10
 * vectors of 3n doubles and 2 of n), the partial sums of shared nodes, both
 * precisions of every level's vectors (7 of 3 n_level each) and the GMRES
 * basis for the current gmres_restart ((restart + 1) vectors of 3n doubles),
 * each rounded up to 256 bytes. The mesh, tile and transfer tables and a few
 * KB of scalars stay allocated by the library (pff_create). */
int pff_workspace_bytes(const pff_ctx* ctx, size_t* bytes);
/* Bind a caller-owned device buffer of at least pff_workspace_bytes bytes,
 * 256-byte aligned, as the home of every work buffer: after this call the
 * library allocates no device memory for them (without it they are allocated
 * on first use). Must precede every call that uses work vectors (set_state,
 * newton_step, tcv); the buffer must stay valid until pff_destroy, which does
 * not free it. While bound, pff_set_params refuses a gmres_restart above the
 * one the workspace was sized for. Errors: PFF_E_ARG (null, misaligned or too
 * small), PFF_E_STATE (work vectors already exist or a workspace is bound). */
int pff_bind_workspace(pff_ctx* ctx, void* dev_ptr, size_t bytes);

/* Sizes: leaf nodes n (vectors have 3n entries), number of multigrid levels,
 * and (if level_nodes != NULL, host, n_levels entries) nodes per level.
 * Every call that takes a level index (sizes, coords, flags, tile stats,
 * inverse diagonal, eigenvalues) addresses the hierarchy that the current
 * pff_params.mg_kind selects; for global coarsening the last level is the
 * leaf mesh. */
int pff_sizes(const pff_ctx* ctx, int64_t* n_nodes, int32_t* n_levels, int64_t* level_nodes);
/* Lattice size M: a node at integer (X, Y) sits at x = -10 + 20 X / M. */
int pff_lattice(const pff_ctx* ctx, int64_t* M);
/* Host copies of node positions (xy: 2n int32, X then Y per node) and flags
 * (n bytes: 1 Dirichlet, 2 hanging, 4 active, 8 refinement edge, 16 node of a
 * leaf cell, 32 leaf-to-level copy target) for the leaf (level = -1) or a
 * level. */
int pff_node_coords(const pff_ctx* ctx, int32_t level, int32_t* xy);
int pff_node_flags(const pff_ctx* ctx, int32_t level, uint8_t* flags);
/* Number of tiles, cell records (own + halo) and largest tile of the leaf
 * operator or a level (host out-pointers, each nullable). */
int pff_tile_stats(const pff_ctx* ctx, int32_t level, int64_t* n_tiles, int64_t* n_records,
                   int64_t* max_cells);

/* Load the linearisation state (Sec. 3.1): U (3n, the Newton iterate),
 * phi_old (n, phase field of the previous load step), phi_tilde (n, the
 * phase field of the linearised degradation, Sec. 2). The library copies them
 * and sets hanging entries of its copies from their masters. active: device
 * n bytes (nonzero = active) or NULL to evaluate the active-set rule of
 * Alg. 2 (constant c as selected by pdas_c) at this state. setup_mg != 0 also prepares the V-cycle: level states
 * and active sets (Sec. 3.2), inverse diagonals and eigenvalue estimates.
 * Synchronises the stream when setup_mg != 0. */
int pff_set_state(pff_ctx* ctx, const double* U, const double* phi_old, const double* phi_tilde,
                  const uint8_t* active, int32_t setup_mg, void* stream);
/* Linearisation phase field for the next load step (Sec. 2: phi~ is the
 * previous step's phase field or an extrapolation from earlier steps):
 * out = min(1, max(0, phi_prev + theta (phi_prev - phi_prev2))) over the n
 * leaf nodes; device pointers, n doubles each, owned by the caller; out may
 * alias either input. theta = (t_n - t_{n-1}) / (t_{n-1} - t_{n-2}) for load
 * parameters t (1 for equal increments); theta = 0 gives phi_prev. The clip
 * keeps phi~ in the range of the phase field. Hanging entries follow the
 * formula; set_state replaces them by the interpolation of their masters.
 * Needs no state. Errors: PFF_E_ARG (null pointer, theta negative or not
 * finite). */
int pff_extrapolate_phi(pff_ctx* ctx, const double* phi_prev, const double* phi_prev2, double theta,
                        double* out, void* stream);
/* The same extrapolation from the load parameters of the two solved steps
 * and the next one (t_prev2 < t_prev <= t_next, e.g. pressures): theta =
 * (t_next - t_prev) / (t_prev - t_prev2). Errors: PFF_E_ARG if the
 * parameters do not increase. */
int pff_extrapolate_phi_load(pff_ctx* ctx, const double* phi_prev, const double* phi_prev2, double t_prev2,
                             double t_prev, double t_next, double* out, void* stream);
/* Copy the current active set (device n bytes, 1 = active). */
int pff_get_active(pff_ctx* ctx, uint8_t* active, void* stream);

/* dst = J~ src: the Jacobian of Sec. 3.1 at the loaded state with hanging-node
 * condensation, constrained columns removed and identity on constrained rows
 * (3n doubles each; dst and src must not overlap). */
int pff_vmult(pff_ctx* ctx, double* dst, const double* src, void* stream);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * dst = J~ src as pff_vmult, with the same kernels and bitwise the same
 * result, but the partial sums of shared nodes go to a static device array
 * of PFF_NOALLOC_SCRATCH_BYTES bytes (one per GPU, held until the process
 * ends) instead of the context's work buffers. The call itself allocates
 * nothing (no hipMalloc, hipFree or allocating library routine); the
 * context, its state (pff_set_state) and the caller's dst and src must exist
 * beforehand. Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (two streams, two contexts or two threads at once) race
 * and must be serialised by the caller; the array keeps the last call's
 * contents, and nothing in it needs to start at zero (every slot is written
 * before it is read within a call). Errors: PFF_E_ARG (null or overlapping
 * vectors, or a mesh whose 3 x n_slots partial sums exceed the array, with
 * the sizes in pff_last_error), PFF_E_STATE (no state). */
#define PFF_NOALLOC_SCRATCH_BYTES (16u * 1024u * 1024u)
int pff_vmult_noalloc(pff_ctx* ctx, double* dst, const double* src, void* stream);
/* dst = J~^T src for `batch` vectors stored one after another (3n each):
 * the transpose of the operator of pff_vmult (the Jacobian of Sec. 3.1 with
 * its coupling block moved to the displacement rows), used by the adjoint
 * of the crack-volume functional (Sec. 4). Identity on constrained rows. */
int pff_vmult_T(pff_ctx* ctx, double* dst, const double* src, int32_t batch, void* stream);

/* Inverse diagonal of the leaf operator (level = -1: 1/diag on free rows, 1 on
 * constrained rows) or of a level block operator (1/diag on free rows, 0 on
 * fixed rows: Dirichlet, level-active, refinement edge, hanging; the level
 * operators of global coarsening carry the hanging-node constraints of their
 * mesh, C^T A C), as used by the
 * Chebyshev-Jacobi smoother (Sec. 1, Sec. 3.2). fp32 selects float output for
 * levels. Needs set_state (and setup_mg for levels). */
int pff_inverse_diagonal(pff_ctx* ctx, int32_t level, void* dst, int32_t fp32, void* stream);

/* dst = P^{-1} src: one V-cycle per diagonal block (Sec. 3.2) with local
 * smoothing (mg_kind 0) or global coarsening (mg_kind 1: smoothing on every
 * level over all its free unknowns, restriction the transpose of the
 * interpolation, leaf rows enter and leave on the finest level); with
 * prec_kind = 1 the block-triangular form (forward substitution, see
 * pff_params). src, dst: 3n doubles (the V-cycle runs in FP32 inside when
 * fp32 != 0). Identity on constrained leaf rows. */
int pff_vcycle(pff_ctx* ctx, double* dst, const double* src, int32_t fp32, void* stream);
/* Eigenvalue estimates per level and block (host arrays): lam_max[2 * l + b]
 * for level l and block b (0 = u, 1 = phi), lam_min0[b] on level 0. get
 * reads the current values; set overrides them (for reproducible tests). */
int pff_get_eigen(const pff_ctx* ctx, double* lam_max, double* lam_min0);
int pff_set_eigen(pff_ctx* ctx, const double* lam_max, const double* lam_min0);

/* Solve J~ x = b (or J~^T x = b when transpose != 0) by GMRES with the block
 * V-cycle as left preconditioner, x0 = 0 (Sec. 3.2). x, b: 3n doubles.
 * tol_override > 0 replaces the absolute tolerance. Synchronises. Returns
 * PFF_W_NOCONV if the iteration limit was reached. */
int pff_gmres_solve(pff_ctx* ctx, double* x, const double* b, int32_t transpose, double tol_override,
                    pff_gmres_info* info, void* stream);

/* One combined Newton / primal-dual active set iteration (Alg. 2) in place on
 * U (3n): residual, active set (active_inout: device n bytes, in = previous
 * set for the change count, out = new set; may be NULL), constraint
 * dphi = phi_old - phi on the active set, multigrid setup, GMRES, line search.
 * phi_old, phi_tilde: n doubles. info: host, nullable. Synchronises. */
int pff_newton_step(pff_ctx* ctx, double* U, const double* phi_old, const double* phi_tilde,
                    uint8_t* active_inout, pff_newton_info* info, void* stream);

/* R = -F(U) condensed (Problem 2 with the linearised degradation) at U with
 * the loaded phi_tilde; masked != 0 zeroes constrained rows with the current
 * active set (the R~ of Alg. 2). */
int pff_residual(pff_ctx* ctx, double* R, const double* U, int32_t masked, void* stream);
/* Total crack volume TCV = int u . grad phi (Sec. 4) of U (host *tcv) and,
 * if dTCVdU != NULL, its derivative with respect to the unknowns (3n,
 * condensed). Synchronises. */
int pff_tcv(pff_ctx* ctx, const double* U, double* tcv, double* dTCVdU, void* stream);
/* Crack opening displacement COD(x) = int u . grad phi dy along the vertical
 * line at x (Sec. 4), for nx positions x (host array, physical coordinates
 * in (-10, 10)); cod: host array of nx results. U: device, 3n; hanging
 * entries are not read (cells with hanging faces take the coarse face's
 * values). A line on a cell edge belongs to the cell on its right; a
 * position outside [-10, 10) gives 0. Each cell integrates with p + 1 Gauss
 * points in y (exact for the degree-2p integrand). Lines are processed in
 * launches of up to 64; no device allocation. Synchronises. Errors: PFF_E_ARG
 * (null pointers with nx > 0, nx < 0, a non-finite position). */
int pff_cod(pff_ctx* ctx, const double* U, const double* x, int32_t nx, double* cod, void* stream);
/* out[0..2] = z^T dF~/d(Gc, E, p) at the loaded state, constrained rows of z
 * ignored (host out): the residual of Problem 2 differentiated in the
 * material parameters of Table 1 (sigma is linear in E at fixed nu; Gc and
 * p enter linearly), with l, kappa and the active set held fixed.
 * Synchronises. */
int pff_param_grad(pff_ctx* ctx, const double* z, double* out, void* stream);
/* Adjoint gradient of the crack volume TCV = int u . grad phi (Sec. 4) with
 * respect to theta = (Gc, E, p) at the loaded state U (3n; pass the U of
 * pff_set_state, which must have run with setup_mg) with the active set held
 * fixed: solves J~^T z = dTCV/dU (constrained rows zero) by transposed GMRES
 * (tolerance: tol_override if > 0, else max(gmres_atol, gmres_rtol |rhs|))
 * and returns grad[0..2] = dTCV/dtheta = -z^T dF~/dtheta (host), *tcv
 * (host, nullable) and z (device 3n, nullable). info: host, nullable.
 * Synchronises. Returns PFF_W_NOCONV if GMRES stopped at its limit. */
int pff_adjoint_tcv(pff_ctx* ctx, const double* U, double* tcv, double* grad, double* z, double tol_override,
                    pff_gmres_info* info, void* stream);
/* Set hanging entries of a nodal vector with ncomp blocked components from
 * their masters. */
int pff_distribute(pff_ctx* ctx, double* v, int32_t ncomp, void* stream);
/* Zero the constrained rows (Dirichlet u, hanging, active phi with the
 * loaded active set) of a 3n vector in place. */
int pff_mask_constrained(pff_ctx* ctx, double* v, void* stream);
/* Deterministic dot product of two device vectors of length len (host out). */
int pff_dot(pff_ctx* ctx, const double* a, const double* b, int64_t len, double* out, void* stream);

const char* pff_last_error(const pff_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* PFF_H_ */
