/*
 * fftc -- constrained DTT/FFT elasticity solver for AMD Instinct MI355X (gfx950).
 *
 * C ABI of libfftc.so.  The library solves the displacement-based fixed point of
 * Gelebart & Amouzou-Adoun ("Constrained minimization problems and FFT-based
 * solvers", Section 3.1.2, eq 3) on a regular voxel grid with the TETRA2 scheme,
 * boundary conditions per face and per component applied through discrete
 * trigonometric transforms (Section 3.2, Tables 1-3, eq 7), local kinematic
 * constraints through Lagrange-multiplier projections (Section 4, Algorithm 1,
 * eq 9-14), unilateral contact with a rigid sphere through an active set
 * (Section 5.1, Algorithm 2, eq 24-28) and depth-4 Anderson acceleration.
 *
 * Conventions
 *  - Every call returns an int status (FFTC_OK = 0, errors negative); nothing
 *    aborts or throws across the ABI; fftc_last_error() returns a message.
 *  - Grid: n[3] = voxels (nx, ny, nz) of edge h.  Nodes per axis N_J = n_J + 1, or
 *    n_J on a periodic axis.  Node (i, j, k) has flat index i + N_x (j + N_y k).
 *    Vector node fields are component-planar [3][N_z][N_y][N_x], x fastest;
 *    voxel fields are [n_z][n_y][n_x].
 *  - Pointers named *_dev are device pointers, borrowed for the duration of the
 *    call.  Pointers named *_host are host pointers.  Set-up calls copy what
 *    they need.
 *  - Device memory: the caller owns the workspace (size from
 *    fftc_workspace_bytes) and binds it with a HIP stream; all device work of a
 *    handle is enqueued on that stream.  The library allocates no device memory.
 *  - Values at the ABI are FP64.  precision selects the arithmetic of the
 *    iteration: FFTC_FP64, or FFTC_FP32 (FP32 fields, stresses, transforms and
 *    Green solve; FP64 norms, convergence test, Anderson Gram matrix and least
 *    squares, reactions and contact forces).
 *  - A handle is not thread safe; distinct handles are independent.
 */
#ifndef FFTC_H
#define FFTC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define FFTC_OK 0
#define FFTC_E_ARG (-1)         /* invalid argument (sizes, indices, duplicates)   */
#define FFTC_E_BC (-2)          /* inconsistent boundary table or constraint on an
                                   eliminated (antisymmetric) DOF with value != 0  */
#define FFTC_E_OVERLAP (-3)     /* overlapping average supports on one component   */
#define FFTC_E_WORKSPACE (-4)   /* workspace missing or too small                   */
#define FFTC_E_NOCONV (-5)      /* max_iter reached; the last iterate is returned   */
#define FFTC_E_NAN (-6)         /* non-finite input or iterate                      */
#define FFTC_E_UNSUPPORTED (-7) /* feature or axis length not supported             */
#define FFTC_E_STATE (-8)       /* call out of order (e.g. solve before stiffness)  */
#define FFTC_E_HIP (-9)         /* HIP runtime error                                */

/* precision */
#define FFTC_FP64 0
#define FFTC_FP32 1

/* boundary codes, bc[comp][axis][face] (Section 3.2.1, Table 1) */
#define FFTC_BC_NEUMANN 0
#define FFTC_BC_DIRICHLET 1
#define FFTC_BC_PERIODIC 2

/* convergence acceleration (Algorithm 1: ACV_U, ACV_P) */
#define FFTC_ACV_NONE 0
#define FFTC_ACV_U 1
#define FFTC_ACV_P 2

typedef struct fftc_problem* fftc_h;

typedef struct {
  double tol;          /* equilibrium tolerance of eq (5); 0 disables the exit test  */
  int32_t max_iter;    /* iterations before FFTC_E_NOCONV                           */
  int32_t acv;         /* FFTC_ACV_*                                                 */
  int32_t depth;       /* Anderson depth; must be 4                                  */
  int32_t period;      /* acceleration period mod_ACV (>= 1)                         */
  double update_gate;  /* contact: residual below which the active set may change   */
  double refine_below; /* FP32 form: once the residual falls below this value, or once
                        * it is below 1e-2 and has not halved in 100 iterations, the
                        * residual pass forms the stresses in FP64 (their rounding in
                        * FP32 is a noise floor of about 3e-7 of ||sigma|| on p, higher
                        * on high-contrast cells); all fields stay FP32.  0 keeps FP32
                        * stresses to the end.                                      */
  int32_t anchor_every; /* FP32 form on small-strain problems without obstacle,
                        * singular modes or relations: the residual pass forms
                        * p_i = p_{i-1} + the divergence term of the stresses of
                        * delta_i = u_i - u_{i-1} (eq 3 is linear in u there), so that
                        * the Anderson differences carry no cancellation against |p|;
                        * every anchor_every-th iteration (and every one below
                        * refine_below) forms p from u.  An incremental iteration never
                        * ends the solve: the convergence test is taken on a pass from
                        * u.  0 forms p from u every iteration.  >= 0.            */
  int32_t reserved;     /* 0                                                         */
} fftc_solver_cfg;

typedef struct {
  int32_t status;             /* FFTC_OK, FFTC_E_NOCONV or FFTC_E_NAN              */
  int32_t iterations;         /* Green solves performed                            */
  double residual;            /* eq (5) at the returned displacement               */
  int32_t contact_updates;    /* active-set updates (contact)                      */
  int32_t anderson_restarts;  /* restarts caused by a changed active set           */
  int32_t contact_nodes;      /* |C| at the end                                    */
  int32_t pad;
  double force_mean_stress;   /* contact: -A0 <sigma_aa> (Section 5.4)              */
  double force_contact;       /* contact: sum of normal contact reactions           */
  double mean_stress[6];      /* <sigma>: xx, yy, zz, yz, xz, xy                   */
} fftc_report;

/* Discrete gradient (Section 3.1.2).  FFTC_TETRA2: two tetrahedra per voxel, two integration
 * points of weight 1/2.  FFTC_HEX1: the gradient of the trilinear interpolant at the voxel
 * centre, one integration point of weight 1; its hourglass modes (zero centre gradient in every
 * voxel) get no Green correction, and single-node conditions excite them (Section 4.2.3: use
 * average relations).  HEX1 runs in FP64 and without contact (FFTC_E_UNSUPPORTED at binding). */
#define FFTC_TETRA2 0
#define FFTC_HEX1 1

/* Create a problem on n[3] voxels of edge h (all lengths at the ABI -- prescribed values,
 * sphere, displacements, gaps -- are in the unit of h; forces are stress times that unit
 * squared; the kernels work in voxel units).  scheme: FFTC_TETRA2 or FFTC_HEX1.
 * Errors: FFTC_E_ARG (n_J < 2 or > 4096, h not positive), FFTC_E_UNSUPPORTED (axis length
 * with a prime factor other than 2, 3, 5, 7, 11, 13, unknown scheme or precision, more than
 * 2^31 DOFs). */
int fftc_create(fftc_h* out, const int32_t n[3], double h, int32_t scheme, int32_t precision);
void fftc_destroy(fftc_h h);

/* Boundary table bc_host[comp*6 + axis*2 + face] (Section 3.2.1, Table 1; Section 3.2.2,
 * Table 2 gives the transform of each (component, axis)).  Periodic must hold on both
 * faces of an axis for all components, else FFTC_E_BC.  Must precede constraints. */
int fftc_set_bc(fftc_h h, const int8_t* bc_host);

/* Reference medium R0 (Section 3.2.3, eq 3-4).  kind FFTC_REF_PAUX: the medium of Paux et
 * al., R0 : grad u = lam0 (grad u o I) + 2 mu0 grad u, one diagonal symbol per component, any
 * boundary table.  FFTC_REF_ISO: the isotropic medium lam0 tr(eps) I + 2 mu0 eps, whose symbol
 * couples the three components (a 3x3 solve per frequency, complex coefficients over periodic
 * axes, Section 3.2.4); it needs the HEX1 scheme, FP64, and either all three axes periodic or
 * normal-mixed faces: no periodic axis and, on every face, the normal component held at 0
 * with both tangential ones free or the reverse (then each component's DTT also diagonalises
 * the coupled medium).  Other tables: FFTC_E_UNSUPPORTED at binding.  Requires mu0 > 0 and lam0 + 2 mu0 > 0 (FFTC_E_ARG).  The
 * kind is fixed at binding (FFTC_E_STATE afterwards).  Default: Paux, max(lam), max(mu). */
#define FFTC_REF_PAUX 0
#define FFTC_REF_ISO 1
int fftc_set_reference(fftc_h h, int32_t kind, double lam0, double mu0);

/* Reference medium as a multiple of the stiffness field: (lam0, mu0) = factor * (max lam,
 * max mu), evaluated by fftc_set_stiffness (the default: Paux, factor 1). */
int fftc_set_reference_factor(fftc_h h, int32_t kind, double factor);

/* Strong nodal constraints u[comp[k]](node[k]) = value[k] (Section 4.1, eq 8-9).
 * node_host: m triples (i, j, k).  set_id groups DOFs for reaction totals (0..63; several
 * calls may share one).  The arrays of this call and of fftc_add_average / fftc_add_smooth may
 * be host or device memory (device arrays are copied to the host).
 * Errors: FFTC_E_ARG (index out of range, DOF constrained twice), FFTC_E_BC (nonzero
 * value on an eliminated DOF; zero values there are dropped). */
int fftc_add_dirichlet(fftc_h h, int64_t m, const int64_t* node_host, const int8_t* comp_host,
                       const double* value_host, int32_t set_id);

/* Kinematic relations: mean of u[comp[r]] over the k nodes of support r equals value[r]
 * (Section 4.2.1, eq 10-14: k = 8 voxel corners or k = 4 face corners; Section 4.2.3: the 44
 * nodes of a line of ten voxels; any 2 <= k <= 64; calls of different k may be combined).
 * proj_U moves the support by the same amount (eq 11), proj_P removes the mean of the
 * boundary-weighted residual 2^-b p from it (eq 14).  support_host: m*k triples.
 * Errors: FFTC_E_ARG (k or index out of range), FFTC_E_BC (support node eliminated for comp),
 * FFTC_E_OVERLAP (a DOF in two supports or also constrained otherwise). */
int fftc_add_average(fftc_h h, int64_t m, int32_t k, const int64_t* support_host,
                     const int8_t* comp_host, const double* value_host, int32_t set_id);

/* Smoothly applied conditions (Section 4.2.2, eq 15-17, Table 2): u[comp[r]] at node r equals
 * value[r] (proj_U, eq 15), and the node's reaction is spread over its neighbours (proj_P,
 * eq 17): a node on no non-periodic face spreads over the 26 nodes of the 2x2x2-voxel cell
 * around it (weights 1/2 middle of faces, 1/4 middle of edges, 1/8 corners, total 8 times
 * the node's multiplier); a node on one face over the 8 nodes of the 2x2 face cell around it
 * in the face plane (1/2, 1/4, total 4).  node_host: m triples (i, j, k).  The reaction
 * reported per condition is the total force.  Errors: FFTC_E_ARG (index out of range),
 * FFTC_E_UNSUPPORTED (node on an edge or corner of the cell), FFTC_E_BC (support reaches a
 * DOF held at 0 by a Dirichlet face), FFTC_E_OVERLAP (support shares a constrained DOF). */
int fftc_add_smooth(fftc_h h, int64_t m, const int64_t* node_host, const int8_t* comp_host,
                    const double* value_host, int32_t set_id);

/* Rigid sphere obstacle (Section 5): every node of face (axis*2 + side) is a potential
 * contact node.  Errors: FFTC_E_ARG (radius <= 0, face out of range, periodic axis). */
int fftc_set_sphere(fftc_h h, const double center_host[3], double radius, int32_t face);

/* Kinematics of the behaviour law (Section 5.2, eq 29, Algorithm 3).  FFTC_SMALL_STRAIN (the
 * default): sigma = C : eps.  FFTC_FINITE_STRAIN: the first Piola-Kirchhoff stress
 * P = F S of the Saint-Venant-Kirchhoff law (Section 5.4: S = lam tr(E) I + 2 mu E,
 * E = (F^T F - I)/2, F = I + grad u) replaces sigma in the residual, in the equilibrium
 * measure (eq 5: ||P||), in the contact reactions and in mean_stress (<P>: xx, yy, zz, yz, xz,
 * xy); the reference medium and the projections are unchanged.  Any time before a solve. */
#define FFTC_SMALL_STRAIN 0
#define FFTC_FINITE_STRAIN 1
int fftc_set_kinematics(fftc_h h, int32_t kind);

/* Solver settings; defaults {1e-6, 2000, FFTC_ACV_P, 4, 2, 1e-2, 1e-5, 16, 0}.  FFTC_E_ARG for
 * a negative tolerance, max_iter, refine_below or anchor_every, a period below 1 or an
 * unknown acv. */
int fftc_set_solver(fftc_h h, const fftc_solver_cfg* cfg);

/* Device workspace needed by the current set-up (grid, precision, constraints). */
int fftc_workspace_bytes(fftc_h h, size_t* bytes);

/* Bind caller-owned device memory (256-byte aligned) and the HIP stream (hipStream_t,
 * NULL = default stream).  Uploads tables and constraints.  FFTC_E_WORKSPACE if small. */
int fftc_bind_workspace(fftc_h h, void* ws_dev, size_t bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): fftc_bind_workspace on a workspace the
 * library holds itself, one array of FFTC_STATIC_WORKSPACE_BYTES per device, kept until the
 * process ends.  The call allocates nothing (no hipMalloc, hipFree or allocating library
 * routine) and times no block sizes: every transform pass takes its larger block.  All
 * handles bound this way on one device share that device's array: a new binding replaces
 * the previous one, whose later calls return FFTC_E_STATE, and calls on two such handles
 * that overlap in time race.  Errors: FFTC_E_WORKSPACE (the problem needs more than
 * FFTC_STATIC_WORKSPACE_BYTES, see fftc_workspace_bytes), FFTC_E_HIP. */
#define FFTC_STATIC_WORKSPACE_BYTES ((size_t)128 << 20)
int fftc_bind_workspace_static(fftc_h h, void* stream);

/* Per-voxel isotropic stiffness (paper eq 1: sigma = C : eps), device arrays [nz][ny][nx] of
 * dtype FFTC_F64 or FFTC_F32, copied into the workspace in the working precision.
 * fftc_set_stiffness takes the Lame constants (lam = mu = 0 marks void voxels);
 * fftc_set_stiffness_Enu Young's modulus and Poisson's ratio (E = 0: void).  Errors:
 * FFTC_E_NAN (non-finite), FFTC_E_ARG (mu < 0 or 3 lam + 2 mu < 0; E < 0 or nu outside
 * (-1, 1/2); unknown dtype), FFTC_E_STATE (no workspace). */
#define FFTC_F64 0
#define FFTC_F32 1
int fftc_set_stiffness(fftc_h h, const void* lam_dev, const void* mu_dev, int32_t dtype);
int fftc_set_stiffness_Enu(fftc_h h, const void* E_dev, const void* nu_dev, int32_t dtype);

/* Algorithm 1.  u_dev: FP64 [3][Nz][Ny][Nx]; on entry the initial guess unless
 * zero_start != 0, on return the last iterate (after the final equilibrium test).
 * With a sphere set, each call is one load increment of Algorithm 2 (start from u_dev,
 * initial active set from the gaps, active-set updates inside the iteration).
 * Returns FFTC_OK, FFTC_E_NOCONV or FFTC_E_NAN (also in rep->status). */
int fftc_solve(fftc_h h, double* u_dev, int32_t zero_start, fftc_report* rep);

/* Move the sphere centre (next increment of Algorithm 2). */
int fftc_move_sphere(fftc_h h, const double center_host[3]);

/* Reactions of the last solve (Section 4.1.3: physical nodal force 2^-b p, sign of eq 8):
 * per_dof_host[m_strong] in the order the strong DOFs were added (dropped zero DOFs
 * excluded), per_relation_host[m_relations] (averages and smooth conditions in the order
 * they were added: the total force each applies), totals_host[nsets*3].  Any pointer may
 * be NULL. */
int fftc_get_reactions(fftc_h h, double* per_dof_host, double* per_relation_host,
                       double* totals_host, int32_t nsets);
int fftc_num_constraints(fftc_h h, int64_t* n_strong, int64_t* n_average);

/* Active set of the last contact solve (Section 5.1, eq 26): mask_host[face nodes] (1 = in C),
 * normal reaction f_nc and gap per face node (face nodes in flat order of the two in-plane
 * axes), the total contact force along the face normal (as fftc_report.force_contact) and the
 * contact area (the face area of the nodes of C, half a voxel face along an edge of the face;
 * its equivalent radius is sqrt(area / pi)).  Any pointer may be NULL. */
int fftc_get_contact(fftc_h h, uint8_t* mask_host, double* fnc_host, double* gap_host, double* force_host,
                     double* area_host);
int fftc_num_face_nodes(fftc_h h, int64_t* count);

/* Stage entry points (one step of the iteration on caller data, for testing):
 * residual: from u, the boundary-weighted residual after proj_P and p~ = p - div(R0:grad u)
 *   (Algorithm 1, stress / divergence / projection / reference term), plus
 *   sums[0] = ||p||^2, sums[1] = sum (1/2) sigma:sigma.  p_dev or ptil_dev may be NULL.
 * green: u = DT^-1(M^-1 DT(ptil)) (eq 3 right part with the transforms of Table 2).
 * Arrays are FP64 device node fields. */
int fftc_stage_residual(fftc_h h, const double* u_dev, double* p_dev, double* ptil_dev,
                        double* sums_host);
int fftc_stage_green(fftc_h h, const double* ptil_dev, double* u_dev);

/* Stage entry of the FP32 iteration as it runs (the residual form of Algorithm 1: FP64
 * displacement u, FP32 residual-sized fields): one residual pass plus the relation projections
 * and the control step, on caller state.  In: u (FP64), delta = u_i - u_{i-1}, e = the last
 * Green input minus K0 u_{i-1}, p_prev, R_prev (FP64 device node fields converted to FP32;
 * NULL = zero), i_local = the Anderson index of the iteration (R is formed from 1 on, its
 * differences from 2 on), pass_kind = 0 for the pass that forms the stresses of u in FP32, 1
 * for the one that forms them in FP64 (taken once the residual is below refine_below), 2 for
 * the incremental pass (p = p_prev + the divergence term of the stresses of delta; u is not
 * read; small strain without obstacle or singular modes, else FFTC_E_UNSUPPORTED).  Out (FP64
 * device node fields, NULL to skip): p after proj_P,
 * R = p + K0 delta - e, dR = R - R_prev, dY = p - p_prev + K0 delta (all 0 at DOFs held at 0),
 * sums[0] = ||p||^2, sums[1] = sum (1/2) sigma:sigma (0 for pass_kind 2).  FP32 handles only
 * (FFTC_E_UNSUPPORTED); FFTC_E_ARG for a pass_kind outside 0..2. */
int fftc_stage_residual_form(fftc_h h, const double* u_dev, const double* delta_dev, const double* e_dev,
                             const double* pprev_dev, const double* rprev_dev, int32_t i_local, int32_t pass_kind,
                             double* p_dev, double* r_dev, double* dr_dev, double* dy_dev, double* sums_host);

/* Batched form: many independent cells (each a fully set-up, bound handle, possibly of
 * different sizes and boundary tables, FP32 precision) iterated together.  A few iterations
 * of the unfinished cells are captured into a HIP graph whose branches run the cells
 * concurrently; the graph is replayed, and captured again without the cells that have met
 * their own exit test, until every cell has finished.  Results are bitwise those of
 * fftc_solve on each cell.  stream: hipStream_t on which the batch runs (cells' own
 * streams are restored afterwards).  The batch creates up to 16 internal streams (default
 * priority) and one pinned host array; it allocates no device memory.
 * Cells with a rigid obstacle (fftc_set_sphere) and FP64 cells are not batched: create
 * returns FFTC_E_UNSUPPORTED (solve them with fftc_solve).
 * batch_solve: u_dev[c] as in fftc_solve (NULL array = zero start for all); reps[count].
 * Returns FFTC_OK if every cell converged, else the first failing status. */
typedef struct fftc_batch* fftc_batch_h;
int fftc_batch_create(fftc_batch_h* out, int32_t count, const fftc_h* cells, void* stream);
int fftc_batch_solve(fftc_batch_h b, double* const* u_dev, int32_t zero_start, fftc_report* reps);
void fftc_batch_destroy(fftc_batch_h b);
const char* fftc_batch_last_error(fftc_batch_h b);

const char* fftc_status_str(int status);
const char* fftc_last_error(fftc_h h);

/* Fixed-count iterations: enqueue exactly `iters` further iterations of the current solve on the
 * handle's stream without an exit test and without host synchronisation (the fields, Anderson
 * history and counters continue from the previous fftc_solve).  The caller synchronises the
 * stream.  Used to time the hot loop. */
int fftc_iterate(fftc_h h, int32_t iters);

/* Per-stage timing: runs `iters` more iterations (no exit test) after a solve and returns the
 * mean time in ms of each stage, measured with HIP events on the handle's stream:
 * [0] residual pass, [1] average-relation projection + control, [2] Anderson store/Gram/LS,
 * [3] x forward DTT (+ Anderson combination), [4] y forward DTT, [5] z forward DTT + Green +
 * z inverse DTT, [6] y inverse DTT, [7] x inverse DTT, [8] proj_U.  The fields keep evolving. */
int fftc_profile_stages(fftc_h h, int32_t iters, double* ms_host, int32_t nstages);

#ifdef __cplusplus
}
#endif
#endif
