/*
 * kfbi.h -- C ABI of the MI355X (gfx950) correction-function KFBI library.
 *
 * The library solves the elliptic interface problem of Zhou & Ying,
 * "A correction function-based kernel-free boundary integral method for
 * elliptic PDEs with implicitly defined interfaces" (arXiv 2309.05965),
 * Sec. 2.2 (eqs. IFP, IFP-bc), divided by the coefficients as in Sec. 3.2
 * (eq. bie-ifp-2):
 *
 *     Lap u - kappa u = fhat_s   in region s,
 *     [u] = g1,  [beta d_n u] = g2   on every interface (interior - exterior),
 *     u = gB   on the boundary of the box [lo, hi]^d,
 *
 * with beta = beta_in inside every interface and beta_out outside.  The
 * unknown density psi = [d_n u] lives on the primary surface points and
 * solves the second-kind BIE  psi/2 + mu K' psi = rhs  (Sec. 3.2) by GMRES
 * (Alg. 1), whose matrix-vector product is one "simple interface problem"
 * solve on the Cartesian grid (Sec. 4, eq. equi-ifp; Sec. 5): collocation
 * for the local correction functions (Secs. 5.3, 5.4), the corrected
 * compact finite-difference right-hand side (Sec. 5.2, eqs. corrected-FDS,
 * crc-formula), a box solve, and corrected interpolation of the normal
 * derivative at the surface points (Sec. 5.5).
 *
 * Conventions
 *  - All array arguments are DEVICE pointers owned by the caller, FP64
 *    unless stated, and all work is ordered on the stream given to
 *    kfbi_plan_create.  Functions return after enqueueing work, except
 *    where a count or a convergence test needs the device (plan set-up,
 *    kfbi_solve): those wait for the values they need, which a small
 *    kernel writes into pinned host memory, not for the whole stream, so
 *    work they enqueue after their last wait (the set-up's operator folds,
 *    the solve's final solve) may still run when they return.
 *  - Grid arrays have (N+1)^d entries in node order i0 + (N+1) i1
 *    (+ (N+1)^2 i2) (x fastest); node x_i = lo + i h, h = (hi - lo)/N.
 *  - Surface arrays are indexed by the surface-point table of the plan
 *    (n_surf entries, canonical order: family r, line, segment, interface).
 *    Density arrays (psi) are indexed by the primary points (n_dof entries,
 *    the primary subsequence of the surface table).
 *  - Errors: every call returns a kfbi_status; kfbi_last_error() gives a
 *    thread-local message.  No exception crosses the ABI.  A plan whose
 *    set-up failed must still be destroyed.
 */
#ifndef KFBI_H
#define KFBI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  KFBI_OK = 0,
  KFBI_E_INVALID = 1,        /* bad argument or geometry (overlap, too close to the box) */
  KFBI_E_UNRESOLVED = 2,     /* no valid collocation / interpolation stencil */
  KFBI_E_SINGULAR = 3,       /* a collocation matrix is singular (cond > 1e10) */
  KFBI_E_NOT_CONVERGED = 4,  /* GMRES reached max_iter */
  KFBI_E_NONFINITE = 5,      /* NaN or Inf in the data */
  KFBI_E_DEVICE = 6,         /* HIP runtime error */
  KFBI_E_OOM = 7             /* device allocation failed */
} kfbi_status;

/* Level-set families (Sec. 5.1: Gamma = {H = 0}, H < 0 inside, outward
 * normal grad H / |grad H|).  Parameter layouts:
 *   ELLIPSE2D   p = [cx, cy, c, s, a, b]: X = c dx + s dy, Y = c dy - s dx,
 *               H = (X/a)^2 + (Y/b)^2 - 1
 *   STAR2D      p = [cx, cy, c0, A1..A8, B1..B8]:
 *               H = rho - (c0 + sum_k A_k cos k theta + B_k sin k theta)
 *   SPHERE3D    p = [cx, cy, cz, r]:  H = |x - c|^2 - r^2
 *   ELLIPSOID3D p = [cx, cy, cz, a0, a1, a2, R00..R22]: X = R^T (x - c)
 *               (R row-major), H = sum_j (X_j / a_j)^2 - 1
 *   TORUS3D     p = [cx, cy, cz, R, r]: H = (sqrt(dx^2+dy^2) - R)^2 + dz^2 - r^2
 *   PRODUCT3D   p = [cx, cy, cz, s]: X = s dx, Y = s dy, Z = s dz,
 *               H = (1+X^2)(1+Y^2)(1+Z^2) + 8XYZ + X^2 + Y^2 + Z^2 - 3
 *               (s = 2: the domain of the 3D Dirichlet example of Sec. 6.2.2)
 *   MOLECULE3D  p = [c, r, m, x1, y1, z1, ..., xm, ym, zm], 1 <= m <= 8:
 *               H = c - sum_k E(-|x - x_k|^2 / r^2), the molecular surface of
 *               Sec. 6.2.3, with E(t) = P(t/1024)^1024, P the degree-12 Taylor
 *               polynomial of exp (Horner), ten squarings: exp to a relative
 *               1e-13 on [-40, 0] from +, -, *, / only
 *   GRID        p = [q] (3 or 5), 2D or 3D: the level set known only at the
 *               grid nodes (Sec. 7), from kfbi_problem.samples[k]: H is the
 *               tensor-product Lagrange interpolant of degree q on the
 *               (q+1)^d nodes around the point's cell (per axis base
 *               floor(t) - (q-1)/2 clamped to [0, N-q], t = (x - lo)/h
 *               snapped to the nearest integer within 1e-9), grad H the
 *               gradient of the same polynomial; H at a node is its sample */
enum {
  KFBI_LS_ELLIPSE2D = 1,
  KFBI_LS_STAR2D = 2,
  KFBI_LS_SPHERE3D = 3,
  KFBI_LS_ELLIPSOID3D = 4,
  KFBI_LS_TORUS3D = 5,
  KFBI_LS_PRODUCT3D = 6,
  KFBI_LS_MOLECULE3D = 7,
  KFBI_LS_GRID = 8
};

/* Boundary integral equation of a problem (Sec. 3):
 *   INTERFACE  the interface problem, unknown psi = [d_n u], psi/2 + mu K' psi
 *              (Sec. 3.2, with beta_in inside every interface, beta_out outside);
 *   DIRICHLET  the interior Dirichlet problem u = gD on Gamma (eq. bie-D):
 *              unknown phi = [u] of u = D phi + N fhat, (1/2 + K) phi = gD - G fhat;
 *   NEUMANN    the interior Neumann problem d_n u = gN on Gamma (eq. bie-N,
 *              gN = sigma^-1 times the paper's g_N): unknown psi = [d_n u] of
 *              u = -S psi + N fhat, (1/2 - K') psi = gN - d_n G fhat.
 * For DIRICHLET and NEUMANN the domain Omega is the union of the interiors,
 * the equation there is Lap u - kappa u = fhat (divided by sigma), the
 * volume potential extends fhat by zero outside Omega (Sec. 4), and the box
 * Green's function vanishes on the box boundary; beta_in and beta_out are
 * not used.  With kappa = 0 the Neumann operator has a one-dimensional null
 * space (u is fixed up to a constant): the right-hand side and every
 * product are shifted to zero mean over the DOFs (Sec. 6.2.1).
 *   TWO_DENSITY the interface problem with different reduced reaction
 *              coefficients on the two sides, kappa = kappa_1 / sigma_1
 *              inside and kappa_out = kappa_2 / sigma_2 outside (sigma_1 =
 *              beta_in, sigma_2 = beta_out): the system of eq. bie-ifp-1 in
 *              phi = u_1 and psi = sigma_2 d_n u_2 on Gamma, of 2 n_dof
 *              unknowns (phi then psi).  Each product takes one simple solve
 *              per Green's function (the superposition remark after Alg. 1);
 *              the plan keeps a second plan of the same geometry for the
 *              exterior operator.  FFT box solver only; no batches, no
 *              learned start. */
enum { KFBI_BIE_INTERFACE = 0, KFBI_BIE_DIRICHLET = 1, KFBI_BIE_NEUMANN = 2, KFBI_BIE_TWO_DENSITY = 3 };

#define KFBI_MAX_IFACE 10
#define KFBI_LS_NPARAM 32

typedef struct {
  int32_t kind;              /* KFBI_LS_* */
  int32_t reserved;
  double p[KFBI_LS_NPARAM];
} kfbi_levelset;

/* Problem descriptor (Secs. 2.1, 2.2).  dim 2|3; order 2 (5/7-point scheme,
 * quadratic correction) or 4 (eqs. 9p-cds / 27p-cds, quartic correction);
 * N a power of two, 8 <= N <= 1024; interiors of the interfaces must be
 * disjoint and stay 3 nodes away from the box boundary; kappa is the
 * reduced reaction coefficient kappa_i / beta_i (equal on both sides);
 * cos_alpha in (0, 1/sqrt(dim)) defines the overlapping surface sets
 * Gamma_r = {|n_r| > cos alpha} (Sec. 5.1); bie one of KFBI_BIE_*;
 * kappa_out the exterior's reduced coefficient (KFBI_BIE_TWO_DENSITY only);
 * samples[k] (KFBI_LS_GRID interfaces only): device array of the (N+1)^dim
 * node values of H_k, x fastest, read by kfbi_plan_create / kfbi_plan_setup
 * (the plan keeps a copy). */
typedef struct {
  int32_t dim, order, N, n_iface;
  int32_t bie, reserved;
  double lo, hi;
  double beta_in, beta_out, kappa, cos_alpha;
  double kappa_out;
  kfbi_levelset iface[KFBI_MAX_IFACE];
  const double* samples[KFBI_MAX_IFACE];
} kfbi_problem;

typedef struct kfbi_plan kfbi_plan;

typedef struct {
  int64_t n_nodes;      /* (N+1)^d */
  int64_t n_surf;       /* surface points (overlapping set Gamma^h) */
  int64_t n_dof;        /* primary points = centres = unknowns */
  int64_t n_irregular;  /* irregular grid nodes (Sec. 5.2) */
  int64_t n_corr;       /* (interface, node) correction entries */
  int32_t n_pde;        /* PDE collocation points per centre */
  int32_t n_dir;        /* Dirichlet collocation points per centre */
  int32_t n_neu;        /* Neumann collocation points per centre */
  int32_t n_coef;       /* polynomial coefficients per centre */
  double h;
  double cond_max;      /* largest 1-norm condition number of the collocation matrices */
} kfbi_sizes;

/* Data of one interface problem (device pointers):
 *   g1, g2  [n_surf]             jumps [u] and [beta d_n u] at the surface points
 *   ftilde  [n_dof][n_pde]       fhat_in - fhat_out at the PDE collocation points
 *   fhat    [n_iface+1][n_nodes] fhat_s at every node for every region s
 *                                (s = 0 exterior, s = k inside interface k)
 *   gB      [n_nodes]            box data; only box-boundary nodes are read
 * Of a Dirichlet or Neumann problem: g2 holds gD resp. gN at the surface
 * points (the DOFs' entries are read), ftilde = fhat at the PDE points,
 * fhat[0] = 0 (the extension by zero), g1 and gB are not read (NULL).
 * Of a two-density problem: g1 = [u], g2 = [sigma d_n u] on the surface
 * points, ftilde [2][n_dof][n_pde] = fhat_1 then fhat_2 at the PDE points
 * (fhat_i = f_i / sigma_i), fhat per region (fhat_2 in region 0), gB. */
typedef struct {
  const double* g1;
  const double* g2;
  const double* ftilde;
  const double* fhat;
  const double* gB;
} kfbi_data;

typedef struct kfbi_mlp kfbi_mlp;

/* Initial density of a solve (Alg. 1 Step 2 gives GMRES an initial guess):
 * zero, the caller's (psi_inout), or predicted by a trained network for an
 * ellipsoid problem (kfbi_learned_start with the fields of kfbi_learned). */
enum { KFBI_START_ZERO = 0, KFBI_START_GIVEN = 1, KFBI_START_LEARNED = 2 };
/* Box solver of a solve: the plan's (kfbi_plan_set_box_solver), or one of
 * KFBI_BOX_FFT / MG64 / MG32 (as 1 + KFBI_BOX_*) set on the plan first. */
enum { KFBI_SOLVER_PLAN = 0, KFBI_SOLVER_FFT = 1, KFBI_SOLVER_MG64 = 2, KFBI_SOLVER_MG32 = 3 };

typedef struct {
  kfbi_mlp* mlp;        /* network 15 -> ... -> 4 x 81 (kfbi_learned_start) */
  int32_t nb;           /* jump coefficients, 32 */
  const double* geom;   /* [15] device: centre, semi-axes, orientation Q row-major */
  const double* jumps;  /* [nb] device: a_1[8], a_2[8], b_1[8], b_2[8] */
  double scale;         /* scale of the network's output */
} kfbi_learned;

/* Options of kfbi_solve.  Zero-initialised apart from tol and max_iter,
 * they give the plain solve: zero start with the plan's box solver. */
typedef struct {
  double tol;           /* GMRES stop: |r_k| <= tol |b| (default 1e-10) */
  int32_t max_iter;     /* unrestarted GMRES length (<= 512) */
  int32_t start;        /* KFBI_START_*: zero, psi_inout as given, or learned from *learned */
  int32_t solver;       /* KFBI_SOLVER_*: with other than PLAN the plan's box solver becomes this one
                           with eps_in, max_cycles and relax (kept for later solves; as
                           kfbi_plan_set_box_solver and kfbi_plan_set_box_relaxation) */
  int32_t max_cycles;   /* multigrid correction cap, 1..64 (0: 40) */
  double eps_in;        /* multigrid tolerance |F - A_h v| <= eps_in |F| (0: 1e-12) */
  double relax;         /* relaxed multigrid tolerance inside GMRES, >= 0 (0: off) */
  const kfbi_learned* learned;   /* KFBI_START_LEARNED: the network and the problem's geometry and jumps */
} kfbi_opts;

typedef struct {
  int32_t iters;
  int32_t status;       /* kfbi_status of the solve */
  double est_rel_res;   /* GMRES residual estimate / |b| */
  double true_rel_res;  /* |b - A psi| / |b| recomputed with a fresh matvec */
} kfbi_info;

/* Step S0 + S1: build the plan of one problem (geometry on the device:
 * regions, surface points, stencils, irregular nodes, correction entries and
 * their closest centres; then factor every collocation matrix).  `stream`
 * is a hipStream_t (NULL = default stream).  On failure *out is still set
 * (destroy it) unless the status is KFBI_E_OOM or KFBI_E_INVALID from the
 * descriptor check. */
kfbi_status kfbi_plan_create(const kfbi_problem* prob, void* stream, kfbi_plan** out);

/* Re-run S0 + S1 for another problem with the same dim, order, N and bie,
 * reusing the plan's buffers (they grow when the new geometry needs more). */
kfbi_status kfbi_plan_setup(kfbi_plan* plan, const kfbi_problem* prob);

kfbi_status kfbi_plan_sizes(const kfbi_plan* plan, kfbi_sizes* out);
/* The stream the plan orders its work on (the one it was created with). */
kfbi_status kfbi_plan_stream(const kfbi_plan* plan, void** stream);

/* Copy a plan table to caller memory (device pointer, `bytes` available).
 * Layouts (int32 unless stated):
 *   REGION     int8 [n_nodes]             region id per node
 *   SURF_POS   double [n_surf][dim]       surface points
 *   SURF_NRM   double [n_surf][dim]       unit normals
 *   SURF_META  int32 [n_surf][5]          family, line id, segment, interface, primary
 *   DOF_SURF   [n_dof]                    surface index of every primary point
 *   STENCIL_D  [n_dof][n_dir]             Dirichlet points (surface indices)
 *   STENCIL_N  [n_dof][n_neu]             Neumann points (surface indices)
 *   EXT_IDX    [n_surf][p]                density extension: primary indices
 *   EXT_W      double [n_surf][p]         density extension weights
 *   PDE_PTS    double [n_dof][n_pde][dim] PDE collocation points
 *   IRREGULAR  [n_irregular]              irregular node indices
 *   CORR       [n_corr][3]                interface, node, owner centre
 *   COND       double [n_dof]             collocation 1-norm condition numbers
 *   DOF_POS    double [n_dof][dim]        primary points
 * The copy is ordered on the plan's stream (no host wait). */
enum {
  KFBI_EXPORT_REGION = 0,
  KFBI_EXPORT_SURF_POS = 1,
  KFBI_EXPORT_SURF_NRM = 2,
  KFBI_EXPORT_SURF_META = 3,
  KFBI_EXPORT_DOF_SURF = 4,
  KFBI_EXPORT_STENCIL_D = 5,
  KFBI_EXPORT_STENCIL_N = 6,
  KFBI_EXPORT_EXT_IDX = 7,
  KFBI_EXPORT_EXT_W = 8,
  KFBI_EXPORT_PDE_PTS = 9,
  KFBI_EXPORT_IRREGULAR = 10,
  KFBI_EXPORT_CORR = 11,
  KFBI_EXPORT_COND = 12,
  KFBI_EXPORT_DOF_POS = 13
};
kfbi_status kfbi_plan_export(const kfbi_plan* plan, int which, void* dst, int64_t bytes);

/* Box solver of the plan (Alg. 1 Step 3.3; the paper uses the FFT):
 *   KFBI_BOX_FFT   exact solve by the type-I sine transform (default);
 *   KFBI_BOX_MG64  multigrid: FP64 two-grid cycles (two damped-Jacobi
 *                  steps before and after the coarse correction, full
 *                  weighting, linear interpolation, the operator
 *                  rediscretised on the grid N/2 and solved there exactly
 *                  by the sine transform in FP64) inside FP64 defect
 *                  correction; needs N >= 16;
 *   KFBI_BOX_MG32  the same cycles with the fine-grid work in FP32 inside
 *                  the FP64 defect correction (residual r = F - A_h v
 *                  always in FP64, the coarse solve in FP64).
 * The multigrid loop stops when |F - A_h v|_2 <= eps_in |F|_2 or after
 * max_cycles corrections (1..64).  Every later box solve, simple solve,
 * matvec and solve of the plan uses this solver; a re-setup keeps it.
 * Allocates three fine grids (FP32 or FP64) and four coarse FP64 grids on
 * the first multigrid request.  Returns KFBI_E_INVALID for an unknown
 * solver, eps_in <= 0, max_cycles out of range or N < 16. */
enum { KFBI_BOX_FFT = 0, KFBI_BOX_MG64 = 1, KFBI_BOX_MG32 = 2 };
kfbi_status kfbi_plan_set_box_solver(kfbi_plan* plan, int solver, double eps_in, int max_cycles);

/* Relaxed multigrid tolerance inside GMRES (inexact Krylov; not in the
 * paper, whose box solve is exact): with relax > 0, the box solve of the
 * matvec at GMRES step j stops at
 *   eps_j = min(1e-1, max(eps_in, relax * tol * |b| / |r_j|)),
 * |r_j| the current GMRES residual estimate, |b| the right-hand side norm
 * and tol the solve's tolerance, all read on the device from the GMRES
 * control data, so the captured iterations stay valid.  The right-hand
 * side, the final solve and the true-residual matvec keep eps_in; the
 * reported true residual judges the result.  relax = 0 (the default)
 * turns it off; no effect with the FFT solver.  Returns KFBI_E_INVALID for
 * a negative or non-finite relax. */
kfbi_status kfbi_plan_set_box_relaxation(kfbi_plan* plan, double relax);

/* Corrections used by, and relative residual |F - A_h v| / |F| reached in,
 * the last multigrid box solve of the plan (synchronises the plan's
 * stream).  For the FFT solver both are 0. */
kfbi_status kfbi_plan_box_stats(kfbi_plan* plan, int32_t* cycles, double* rel_res);

/* Box solve alone (step S3; Alg. 1 Step 3.3): A_h v = F on the interior
 * nodes with v = 0 on the box boundary, A_h the plan's scheme, by the
 * plan's box solver (exact with the FFT; to eps_in with multigrid).
 * F, v: [n_nodes] (interior of F read; all of v written).  F and v may not
 * alias. */
kfbi_status kfbi_box_solve(kfbi_plan* plan, const double* F, double* v);

/* Box solve without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the FFT box solve of kfbi_box_solve
 * (the same kernels) on the grid [lo, hi]^dim with N intervals per axis,
 * scheme `order` (2 or 4) and reduced reaction coefficient kappa, without
 * a plan.  v = A_h^-1 F on the interior, v = 0 on the box boundary;
 * F, v: [(N+1)^dim] device arrays of the caller (distinct), x fastest.
 * Work is ordered on `stream` (a hipStream_t of the current device; NULL =
 * default stream) and the call returns after enqueueing it.
 * Limits: N a power of two, 8 <= N <= 1024 in 2D and <= 128 in 3D; larger
 * grids return KFBI_E_INVALID.  The two intermediate grids and the FFT
 * tables live in one static device array of 34.4 MB per device (2 x
 * 2,146,720 + 5,376 doubles), held from the first call on a device until
 * the process ends; the call allocates nothing (no hipMalloc, hipFree or
 * allocating library routine).  Every call on a device shares that array:
 * calls that overlap on one device (two streams, two threads) race and
 * must be serialised by the caller. */
/* Lines per tile of the sine-transform passes (S3) on a grid (dim, N): the
 * caller's override (kfbi_set_tile_lines), else the autotuner's choice (at
 * the first plan of that grid in the process the library times the x pass
 * and the most strided pass for every candidate tile and keeps the fastest
 * unless it is within 10% of the built-in rule's tile; KFBI_TILE_AUTOTUNE=0 in the
 * environment keeps the rule), else the rule.  Results do not depend on it:
 * every even tile pairs the lines the same way and each line's transform is
 * the same.  Returns 0 for an invalid grid. */
int kfbi_tile_lines(int dim, int N);
/* Override the tile lines of a grid: an even TL of 2..8 that fits the LDS
 * (twice per compute unit) and leaves at least 256 tiles; 0 removes the
 * override.  The 2D grids of 512 and 1024 run their own kernels with fixed
 * tiles and take no override.  Affects launches made after the call. */
kfbi_status kfbi_set_tile_lines(int dim, int N, int TL);

kfbi_status kfbi_box_solve_noalloc(int dim, int order, int N, double lo, double hi, double kappa,
                                   const double* F, double* v, void* stream);

/* One simple interface problem (eq. con-ifp with box data; Secs. 4, 5):
 * w with [w] = a, [d_n w] = b, Lap w - kappa w = fhat_s, w = gB on the box.
 * a, b: [n_surf] (NULL = 0); ftilde [n_dof][n_pde], fhat, gB as in
 * kfbi_data (NULL = 0).  Outputs: v [n_nodes] (may be NULL), and at the
 * primary points [n_dof] (may be NULL) the one-sided limits of the
 * corrected interpolation (Sec. 5.5): d_n w_in and d_n w_out, or, on a
 * plan of a Dirichlet problem, the values w_in and w_out. */
kfbi_status kfbi_simple_solve(kfbi_plan* plan, const double* a, const double* b,
                              const double* ftilde, const double* fhat, const double* gB,
                              double* v, double* dn_in, double* dn_out);

/* The BIE operator (hot path, steps S2-S5): Apsi = J[w(0, E psi, 0, 0, 0)] /
 * (beta_in + beta_out), J = beta_in d_n w_in - beta_out d_n w_out, E the
 * density extension to the surface table.  Equals psi/2 + mu K' psi of
 * Sec. 3.2 with mu = (beta_out - beta_in)/(beta_out + beta_in).
 * Dirichlet problem: Aphi = w_in(E phi, 0, 0, 0, 0), the interior value,
 * = (1/2 + K) phi (eq. bie-D); Neumann problem: Apsi = d_n w_in(0, E psi,
 * 0, 0, 0) = (1/2 - K') psi (eq. bie-N), shifted to zero mean when kappa = 0.
 * Two-density problem: the operator of eq. bie-ifp-1 on [phi; psi].
 * psi, Apsi: [n_dof] ([2 n_dof] for a two-density plan), distinct buffers. */
kfbi_status kfbi_matvec(kfbi_plan* plan, const double* psi, double* Apsi);

/* BIE right-hand side (Alg. 1 Step 1):
 * b = (g2 - J[w(g1, 0, ftilde, fhat, gB)]) / (beta_in + beta_out), b [n_dof];
 * Dirichlet: b = gD - w_in(0, 0, ftilde, fhat, 0); Neumann: b = gN -
 * d_n w_in(0, 0, ftilde, fhat, 0) (zero mean when kappa = 0); two-density:
 * the right-hand side of eq. bie-ifp-1, b [2 n_dof]. */
kfbi_status kfbi_rhs(kfbi_plan* plan, const kfbi_data* data, double* b);

/* Full solve (Alg. 1): b, GMRES on kfbi_matvec to opts->tol, then
 * u = w(g1, E psi, ftilde, fhat, gB) (Dirichlet: w(E phi, 0, ftilde, fhat,
 * 0), Neumann: w(0, E psi, ftilde, fhat, 0); the solution is u on the nodes
 * of Omega, the Neumann one up to an additive constant; a learned start is
 * for interface problems only).  A two-density plan solves eq. bie-ifp-1
 * by GMRES with classical Gram-Schmidt applied twice (host Hessenberg, one
 * host wait per orthogonalisation pass), psi_inout holding [phi; psi]
 * (2 n_dof), u = u_1 = W_1(phi, (psi + g2)/sigma_1, ...) inside and u_2 =
 * W_2(g1 - phi, -psi/sigma_2, ...; gB) outside.  psi_inout [n_dof] (initial guess
 * with KFBI_START_GIVEN; with KFBI_START_LEARNED the predicted density is
 * written there first; density on return); u_out [n_nodes] (may be NULL).
 * With a multigrid box solver, u is the step-1 grid solution plus the box
 * solution of the true residual's matvec (the solution is linear in the
 * data and the density), and that box solve starts from the iterations'
 * stored box solutions combined with the GMRES coefficients.
 * The host waits for the device between batches of captured GMRES
 * iterations and for the true residual; on a plan solved before (same graph
 * key), without relaxation and from a zero start, the update, the true
 * residual and the final solve are enqueued behind the first batch, so a
 * solve that converges within it waits once.  The iterations run
 * as captured HIP graphs: on a plan created with a stream of the caller's
 * own they are captured and launched on that stream; on a default stream
 * (NULL, legacy or per-thread) the solve runs on a private stream of the
 * plan, ordered after and before the caller's stream by events (which costs
 * a few tens of microseconds per solve).  Returns KFBI_E_NOT_CONVERGED (with
 * psi and u of the last iterate) if max_iter is reached. */
kfbi_status kfbi_solve(kfbi_plan* plan, const kfbi_data* data, const kfbi_opts* opts,
                       double* psi_inout, double* u_out, kfbi_info* info);

/* Event timing of the box-solve kernels (tracing aid).  With enable = 1
 * every subsequent FFT box solve of the plan is bracketed by two HIP events
 * on the plan's stream; with enable = 2 the finest-level post-smoothing
 * sweeps of every multigrid cycle that are not fused with the update (one
 * on 3D grids up to 128^3, two otherwise), with enable = 3 the passes of
 * every cycle's exact coarse solve (five in 3D, three in 2D); modes 2 and 3
 * trace the multigrid solves outside GMRES iterations, which are then
 * enqueued kernel by kernel instead of as graphs.  kfbi_plan_timing synchronises the stream
 * and returns the number of bracketed intervals and kernel launches
 * recorded since enabling and their total elapsed milliseconds (launches
 * are back to back, so ms / launches is the average launch duration).
 * enable = 0 stops and clears the record. */
kfbi_status kfbi_plan_profile(kfbi_plan* plan, int enable);
kfbi_status kfbi_plan_timing(kfbi_plan* plan, int64_t* solves, int64_t* launches, double* ms);

kfbi_status kfbi_plan_destroy(kfbi_plan* plan);

/* ----------------------------------------------------------------------
 * Many independent problems (batched solves, Alg. 1 per problem).  Two
 * ways to give the data, both with n_workers host threads that each own a
 * stream and take problems largest first:
 *   set up, then solve: kfbi_batch_setup builds one plan per problem;
 *     the caller reads each plan's query points (kfbi_batch_plan, then
 *     kfbi_plan_sizes / kfbi_plan_export) and passes every problem's
 *     kfbi_data and density buffer to kfbi_batch_solve;
 *   streaming: kfbi_batch_solve_stream keeps one plan per grid shape per
 *     worker, sets it up for each problem in turn and asks a callback for
 *     the problem's data (memory bounded by the workers, not the batch).
 * -------------------------------------------------------------------- */
typedef struct kfbi_batch kfbi_batch;

/* A batch of n problems (copied) with n_workers (1..16) workers.  Device
 * of the calling thread. */
kfbi_status kfbi_batch_create(const kfbi_problem* probs, int n, int n_workers, kfbi_batch** out);
/* Number of problems and sum of their node counts (the length of u_all). */
kfbi_status kfbi_batch_sizes(const kfbi_batch* batch, int64_t* n_problems, int64_t* total_nodes);

/* S0 + S1 of every problem, one plan each (kept until kfbi_batch_destroy;
 * a plan is ordered on the stream of the worker that built it).  infos
 * (host, [n], may be NULL): status of each set-up in .status (e.g.
 * KFBI_E_UNRESOLVED for a geometry the grid does not resolve); seconds
 * (host, [n], may be NULL): wall time of each set-up.  Returns KFBI_OK if
 * every set-up succeeded, else the first failure's status with its
 * message; the other problems are set up all the same.  Waits for the
 * device. */
kfbi_status kfbi_batch_setup(kfbi_batch* batch, kfbi_info* infos, double* seconds);
/* The plan of problem i after kfbi_batch_setup (owned by the batch; NULL
 * with the set-up's status if it failed). */
kfbi_status kfbi_batch_plan(kfbi_batch* batch, int i, kfbi_plan** plan);
/* Solve every set-up problem with opts (box solver, tolerance, start; a
 * learned start is per problem and is rejected here), on the worker and
 * stream that set it up: data [n] (host array of kfbi_data with device
 * arrays at each plan's query points), psi [n] (host array of device
 * arrays of n_dof doubles: the density out, and the initial guess with
 * KFBI_START_GIVEN; psi or an entry may be NULL to discard it), u_all
 * (device, may be NULL): the solutions concatenated in problem order,
 * (N_i+1)^d values each.  infos (host, [n]) and seconds (host, [n], may be
 * NULL) are filled for every problem (a problem whose set-up failed keeps
 * that status).  Returns KFBI_OK only if every problem is OK, else the
 * first failure's status with its message.  Waits for the device. */
kfbi_status kfbi_batch_solve(kfbi_batch* batch, const kfbi_opts* opts, const kfbi_data* data, double* const* psi,
                             double* u_all, kfbi_info* infos, double* seconds);

/* Streaming data: once a worker's plan is set up for a problem (its query
 * points are then known: kfbi_plan_sizes, kfbi_plan_export), the callback
 * is called on the worker's host thread with the plan and its stream; work
 * it enqueues must go on that stream.  It fills *data with device arrays
 * laid out as kfbi_data for that plan, which must stay valid until the same
 * worker calls it again or the solve returns, and sets *psi_out to a device
 * array of n_dof doubles for the problem's density (the initial guess too
 * with KFBI_START_GIVEN), or to NULL to discard it.  A status other than
 * KFBI_OK fails the problem with that status. */
typedef kfbi_status (*kfbi_batch_data_fn)(void* ctx, int problem, kfbi_plan* plan, void* stream, kfbi_data* data,
                                          double** psi_out);
/* Set up and solve every problem, streaming (see above): u_all, infos and
 * seconds as in kfbi_batch_solve (seconds include the set-up and the
 * callback).  Independent of kfbi_batch_setup's plans. */
kfbi_status kfbi_batch_solve_stream(kfbi_batch* batch, const kfbi_opts* opts, kfbi_batch_data_fn data_fn, void* ctx,
                                    double* u_all, kfbi_info* infos, double* seconds);
kfbi_status kfbi_batch_destroy(kfbi_batch* batch);

/* ----------------------------------------------------------------------
 * Learned initial density for GMRES (Alg. 1 Step 2 gives GMRES an initial
 * guess; this predicts one).  All pointers are device pointers ordered on
 * the given stream (the plan's stream for the plan calls); the MLP object
 * and its buffers are library-owned.
 * -------------------------------------------------------------------- */
/* MLP widths[0] -> widths[1] -> ... -> widths[n_layers], ReLU after every
 * layer but the last.  Weights are bf16 copies of fp32 master weights
 * (all zero until kfbi_mlp_set_params); GEMMs accumulate in fp32.
 * Parameter pack (fp32): for each layer W_l [widths[l] x widths[l+1]]
 * row-major, then b_l [widths[l+1]]. */
kfbi_status kfbi_mlp_create(int n_layers, const int* widths, void* stream, kfbi_mlp** out);
kfbi_status kfbi_mlp_sizes(const kfbi_mlp* mlp, int64_t* n_params);
/* Copy a parameter pack in (resets the Adam state) or out. */
kfbi_status kfbi_mlp_set_params(kfbi_mlp* mlp, const float* params);
kfbi_status kfbi_mlp_get_params(const kfbi_mlp* mlp, float* params);
/* Y [B x widths[L]] = MLP(X [B x widths[0]]), fp32 in and out. */
kfbi_status kfbi_mlp_forward(kfbi_mlp* mlp, const float* X, int B, float* Y);
/* loss = mean over all entries of (MLP(X) - Yt)^2 (device float) and its
 * gradient with respect to the parameter pack (grads may be NULL). */
kfbi_status kfbi_mlp_loss_grad(kfbi_mlp* mlp, const float* X, const float* Yt, int B, float* loss,
                               float* grads);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8, bias-corrected) on the same
 * loss; loss of the batch before the step written to *loss (device). */
kfbi_status kfbi_mlp_train_step(kfbi_mlp* mlp, const float* X, const float* Yt, int B, float lr, float* loss);
kfbi_status kfbi_mlp_destroy(kfbi_mlp* mlp);

/* Linear head (the density is linear in the jump coefficients when the
 * source and box data vanish, Sec. 3.2 with fhat = 0, gB = 0): X holds B
 * examples of R consecutive rows; the network's output of example b, its R
 * rows read as one row of R widths[L] entries, holds nb basis vectors of
 * K = R widths[L] / nb entries, and the head is y[b][k] = sum_j C[b][j]
 * out[b][j K + k].  C [B x nb] fp32; Y, Yt [B x K] fp32.  loss_grad_lin /
 * train_step_lin use the loss mean over all entries of (y - Yt)^2 (the head
 * in fp32, its gradient C[b][j] dy[b][k] back-propagated through the
 * network); train_step_lin takes one Adam step as kfbi_mlp_train_step.
 * KFBI_E_INVALID if nb does not divide R widths[L]. */
kfbi_status kfbi_mlp_forward_lin(kfbi_mlp* mlp, const float* X, int B, int R, const float* C, int nb, float* Y);
kfbi_status kfbi_mlp_loss_grad_lin(kfbi_mlp* mlp, const float* X, int B, int R, const float* C, int nb,
                                   const float* Yt, float* loss, float* grads);
kfbi_status kfbi_mlp_train_step_lin(kfbi_mlp* mlp, const float* X, int B, int R, const float* C, int nb,
                                    const float* Yt, float lr, float* loss);

/* C [M x N] (fp32, row stride ldc) = op(A) op(B) with bf16 operands (raw
 * 16-bit storage) and fp32 accumulation on the matrix cores.  transA = 0:
 * A is [M x K] (row stride lda); 1: A is [K x M].  transB = 0: B is
 * [K x N]; 1: B is [N x K].  Both transposed is rejected. */
kfbi_status kfbi_gemm_bf16(int transA, int transB, int M, int N, int K, const uint16_t* A, int lda,
                           const uint16_t* B, int ldb, float* C, int ldc, void* stream);

/* Features of ns interface samples for P ellipsoids: geom [P][15] =
 * centre (3), semi-axes (3), orientation Q row-major (9); jumps [P][32] =
 * a[j][m] (16) then b[j][m] (16) of g_j(x) = sum_m a_jm cos(k_m . x) +
 * b_jm sin(k_m . x), k_m = (pi/2)(m & 1, (m >> 1) & 1, (m >> 2) & 1);
 * S [ns][3] unit directions, sample i at x = c + Q diag(a) S_i.
 * X [P][ns][9] = (x, outward normal, mean curvature, g1, g2), fp32. */
kfbi_status kfbi_ellipsoid_features(const double* geom, const double* jumps, int P, const double* S, int ns,
                                    void* stream, float* X);
/* Training-data augmentation from the linearity of the density in the
 * jump data: in place, for every example r < B, the g1 and g2 features of
 * its ns samples in X [B][ns][9] and its target row Y [B][nout] are
 * multiplied by alpha[r]. */
kfbi_status kfbi_scale_jumps(float* X, float* Y, const float* alpha, int B, int ns, int nout, void* stream);
/* Density at the plan's DOFs from values at the samples: least-squares
 * fit of the 81 real spherical harmonics of degree <= 8 in the body-frame
 * direction diag(1/a) Q^T (x - c) to scale * psi_s (ns >= 81), evaluated
 * at the DOFs.  geom [15] as above (device); psi_dof [n_dof]. */
kfbi_status kfbi_sh_transfer(kfbi_plan* plan, const double* geom, const double* S, int ns, const float* psi_s,
                             double scale, double* psi_dof);
/* Density at the samples from values at the DOFs (the same fit from the
 * DOFs, n_dof >= 81), times scale, fp32.
 * Both transfers are ordered on the plan's stream without a host wait and
 * use a workspace the plan keeps (grown on demand, freed with the plan);
 * concurrent transfers on one plan are not allowed. */
kfbi_status kfbi_sh_sample(kfbi_plan* plan, const double* geom, const double* psi_dof, const double* S, int ns,
                           double scale, float* psi_s);
/* Network input of the linear-head start for P ellipsoids, geom [P][15] as
 * above: X [P][8][15] fp32, one row per Fourier mode m of the jump data:
 * (a_k - 0.5) / 0.2 for the three semi-axes, the mode's wave vector in the
 * scaled body frame diag(a) Q^T k_m (3), and the nine entries of Q. */
kfbi_status kfbi_geometry_input(const double* geom, int P, void* stream, float* X);
/* Least-squares coefficients coef [81] (device, FP64) of scale * psi_dof in
 * the 81 real spherical harmonics of the body-frame direction of the plan's
 * DOFs (n_dof >= 81), on the plan's stream (targets of the linear head). */
kfbi_status kfbi_sh_coefficients(kfbi_plan* plan, const double* geom, const double* psi_dof, double scale,
                                 double* coef);
/* The expansion sum_i coef[i] Y_i (81 harmonics of the body-frame
 * direction) at the plan's DOFs, times scale: psi_dof [n_dof]. */
kfbi_status kfbi_sh_expand(kfbi_plan* plan, const double* geom, const double* coef, double scale, double* psi_dof);
/* Learned initial density of one ellipsoid problem (Alg. 1 Step 2 with a
 * predicted start): the network (15 -> ... -> 4 x 81, one row per Fourier
 * mode, kfbi_geometry_input(geom)) gives for every mode m the SH
 * coefficients of the four basis densities of a_1m, a_2m, b_1m, b_2m; the
 * head contracts them with jumps [nb = 32] (device FP64, packed as a_1[8],
 * a_2[8], b_1[8], b_2[8] like kfbi_ellipsoid_features), times scale, and
 * the expansion is evaluated at the plan's DOFs into psi_dof [n_dof].
 * Ordered on the plan's stream (the network's kernels too); uses the plan's
 * transfer workspace; the network must not be used by another thread
 * meanwhile. */
kfbi_status kfbi_learned_start(kfbi_plan* plan, kfbi_mlp* mlp, int nb, const double* geom, const double* jumps,
                               double scale, double* psi_dof);
/* The 81 real orthonormal spherical harmonics (no Condon-Shortley phase,
 * index l^2 + l + m) at n directions: Y [81][n]. */
kfbi_status kfbi_real_sh(const double* dirs, int n, void* stream, double* Y);

/* Thread-local message of the last failing call (never NULL). */
const char* kfbi_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* KFBI_H */
