// Internal definitions of the KFBI library: the plan, device buffers and the
// host launchers of every kernel translation unit.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <shared_mutex>
#include <string>
#include <vector>

#include "../../include/kfbi.h"

#define KFBI_BLOCK 256
#define KFBI_MAXC 35       // max polynomial coefficients (3D, degree 4)
#define KFBI_MAXP 10       // max PDE collocation points
#define KFBI_MAXD 15       // max Dirichlet points
#define KFBI_MAXN 10       // max Neumann points
#define KFBI_GMRES_MAX 512
#define KFBI_NGRAPH 5      // captured GMRES graphs of 1, 2, 4, 8 and 16 iterations
#define KFBI_MG_GRAPHS 48  // captured multigrid box solves kept per plan

// device-side status bits (OR-ed into plan->d_flags)
enum {
  FLAG_OVERLAP = 1,
  FLAG_MARGIN = 2,
  FLAG_UNRESOLVED_STENCIL = 4,
  FLAG_UNRESOLVED_EXT = 8,
  FLAG_UNRESOLVED_OWNER = 16,
  FLAG_SINGULAR = 32,
  FLAG_NONFINITE = 64
};

struct GridDesc {           // plain-value grid/problem description for kernels
  int d, order, p, N, n1, K;
  int bie;                  // KFBI_BIE_*: what the density is and what the interpolation returns
  double lo, hi, h, kappa, cos_alpha, beta_in, beta_out;
  int64_t n_nodes;
};

// Pinned host block that the device posts small results into (k_post): the
// values, then the sequence word with a system-scope release store.
struct KfbiMailbox {
  unsigned seq;
  int iv[8];
  unsigned long long dv[9];      // bit patterns of doubles
};

// What k_post copies: up to 8 ints and 8 doubles from device memory and,
// if nmax > 0, the maximum of maxsrc[0..nmax) (a NaN wins) as double nd.
struct PostReq {
  const int* isrc[8];
  int ni;
  const double* dsrc[8];
  int nd;
  const double* maxsrc;
  int64_t nmax;
};

struct kfbi_plan {
  kfbi_problem prob;
  GridDesc g;
  hipStream_t stream;
  int nP, nD, nN, nC;            // collocation sizes
  int64_t n_seg;                 // grid segments = d N (N+1)^(d-1)
  int64_t n_lines;               // d (N+1)^(d-1)
  int64_t n_cand, n_surf, n_dof, n_irr, n_corr;
  int64_t ncell_axis, ncell;     // closest-centre bins (per interface)
  double cond_max;
  bool ready;

  // capacities (elements) of the count-dependent buffers
  int64_t cap_cand, cap_surf, cap_dof, cap_irr, cap_corr;

  // grid-sized
  int8_t* region;
  uint8_t* need;                 // [K][n_nodes] correction-entry flags
  double* Cg;                    // [K][n_nodes] correction values
  double *Fs, *T1, *T2, *vbuf, *vsbuf;   // simple-solve RHS, box-solve pass buffers, grid solutions
                                 // (vbuf's box boundary stays zero: the box solves write interior nodes)
  // candidates
  int *c_r, *c_lid, *c_seg, *c_k, *c_ina;
  double *c_pos, *c_nrm;
  int* c_acc;
  // surface table
  double *s_pos, *s_nrm;
  int *s_meta;                   // [n_surf][5]: fam, lid, seg, iface, prim
  int *s2d, *d2s;
  uint8_t* s_need;
  int *line_start, *line_end;
  // centres
  int *stD, *stN;
  int* ext_idx;
  double* ext_w;
  double* MinvT;                 // [n_dof][nC][nC], element (alpha, j) at j*nC + alpha
  double* MT;                    // [n_dof][nC][nC], M element (j, alpha) at alpha*nC + j
  double* cond;
  double *psiS, *aS, *U, *dn_in, *dn_out;
  // irregular nodes and correction entries
  int* irr;
  int *ce_k, *ce_node, *ce_owner;
  // closest-centre bins
  int *cell_count, *cell_start, *cell_items;
  int* cell_cursor;              // per-cell fill cursor of the binning
  // scan scratch
  uint8_t* flags8;               // predicate per item, max(d N (N+1)^(d-1) K, n_nodes)
  int *blk, *blk_total;
  int64_t cap_blk;
  uint8_t* flags8b;              // irregular-node predicate per node (compacted beside the candidates)
  int* blk2;                     // scan scratch of that compaction and of the correction entries
  int64_t cap_blk2;
  int* blk3;                     // scan scratch of the centre count over the candidates
  int64_t cap_blk3;
  int* d_flags;
  int* h_pinned;                 // pinned host scratch for counts
  double* h_dpinned;
  // box solver tables
  double *tw, *eig1;
  // GMRES
  double *V, *Hm, *gv, *cs, *sn, *work, *work2, *bvec, *scal;
  int gm_cap;
  int last_iters;                // GMRES iterations of the plan's previous solve
  double* gm_part;               // Arnoldi partial sums [3][gm_pb][gm_cap + 2]
  int gm_pb;
  int64_t gm_n;
  // folded operators of the matvec (set-up products of the inverses with the
  // density extension): C at entry e = sum_t FW[e][t] psi[FI[e][t]],
  // d_n C at centre c = sum_t GW[c][t] psi[GI[c][t]], own-polynomial part of
  // the interpolation at centre c = sum_t HW[c][t] psi[GI[c][t]]
  // (nF = nN p terms)
  int nF, maxpairs;
  int *FI, *GI;
  double *FW, *GW, *HW, *IW;     // IW: [n_dof][(q+1)^d] normal-derivative weights
  double* TI;                    // [n_dof][nC] sum over the block nodes outside the
                                 // centre's region of IW * monomials (own polynomial)
  double* Cv;                    // [n_corr] correction values of the current matvec
  double* sh_ws;                 // spherical-harmonic transfer workspace (learned start)
  int64_t sh_ws_cap;
  double* Firr;                  // [n_irr] corrected right-hand side at the irregular nodes (many pairs)
  double* ls_samples;            // [K][n_nodes] the plan's copy of sampled level sets
  // two-density BIE (eq. bie-ifp-1): value interpolation weights, the plan
  // of the exterior operator (same geometry, Lap - kappa_out), one-sided
  // values at the DOFs, GMRES over [phi; psi]
  double *IWv, *TIv;             // [n_dof][(q+1)^d] value weights, [n_dof][nC] their own-polynomial sums
  double *GWv, *HWv;             // [n_dof][nF] folds of C_c(p_c) and of the value interpolation's own term
  kfbi_plan* aux;
  bool is_aux;
  double *tv_in, *tv_out;        // [cap_dof]
  int64_t td_cap_dof;
  double *td_V, *td_b, *td_w, *td_part, *td_h;   // basis [(m+1)][2 n], right-hand side, work, dot partials
  double* h_td;                  // pinned host copy of the dots
  int td_m;
  int64_t td_n;
  int* IB;                       // [n_dof] first node of the interpolation block
  int* IE2;                      // [n_dof][(q+1)^d] entry of C^(reg q) at block nodes
                                 // inside another interface, -1 elsewhere
  double* PA;                    // [n_irr][maxpairs] stencil coefficients of the cut neighbours
  int *PE1, *PE2;                // [n_irr][maxpairs] entries of C^(reg P), C^(reg Q)
  int *EI;                       // [K][n_nodes] entry index of (interface, node), -1 if none
  int *row_start, *row_end;      // irregular nodes of every x-line
  int64_t cap_fold_corr, cap_fold_dof, cap_fold_irr;
  // box solver: FFT, or multigrid V-cycles (FP64 or FP32) inside FP64
  // defect correction to |F - A v| <= mg_eps |F|, at most mg_maxit cycles
  int box_solver;
  double mg_eps;
  double mg_eps_out;             // inside kfbi_solve: tolerance of the box solves outside the GMRES iterations
  int mg_maxit;
  double mg_c[27];                // A_h on the 3^d cube (fine grid)
  double mg_w;                   // Jacobi weight of the fine grid
  void *mg_u, *mg_t, *mg_f;      // fine-grid arrays (float or double), boundaries zero
  int64_t mg_bytes;
  // coarse grid N/2 of the two-grid cycle, solved exactly by the sine
  // transform in FP64: right-hand side, solution, two pass buffers, tables
  GridDesc mg_gc;
  double *mg_Fc, *mg_Uc, *mg_T1c, *mg_T2c, *mg_twc, *mg_eigc;
  int64_t mg_nc;                 // (N/2 + 1)^d the coarse arrays hold
  double* mg_part;               // partial sums of the outer residual
  int* mg_ctl;                   // [done, corrections, most corrections since the solve began,
                                 //  box solves stopped by the cap above eps, then per GMRES
                                 //  iteration j the corrections of its box solve at 4 + j]
  int mg_cap_eff;                // cap used inside kfbi_solve: observed need + 2 (0: unknown)
  int mg_run_cap;                // cap of the box solves being enqueued (0: mg_maxit)
  bool mg_guess;                 // the box solve being enqueued starts from v as it stands
  // box solutions of a solve's matvecs (multigrid): slot 0 the initial
  // iterate's, slot 1 + j GMRES iteration j's.  The iterate x0 + sum y_j v_j
  // has the same combination of them as its box solution, which starts the
  // box solve of the true residual.
  double* ustore;
  int ustore_slots;              // slots allocated (0: none)
  int64_t ustore_n;              // nodes per slot
  // captured multigrid box solves, one per (right-hand side, solution,
  // GMRES control word, cap, start, tolerance), valid while the multigrid configuration
  // key mg_sg_key holds: they do not depend on the interfaces, so every
  // geometry on the same grid reuses them
  struct MgSolveGraph {
    const double* F;
    double* v;
    const int* gctl;
    int cap, guess;
    double eps;
    hipGraph_t g;
    hipGraphExec_t e;
  };
  MgSolveGraph mg_sg[KFBI_MG_GRAPHS];
  int mg_sg_n;
  uint64_t mg_sg_key[48];
  bool mg_graphs_off;            // a capture failed: solves are enqueued kernel by kernel
  double mg_relax;               // inexact-Krylov relaxation of eps inside GMRES (0: off)
  double relax_word;             // host copy of the factor last written to GMRES scal[7] (NaN: none)
  double* mg_scal;               // [|F|, last relative residual]
  double* Fmg;                   // matvec right-hand side (full grid), zero off the irregular nodes
  // GMRES iteration on the device: control word [j, done, k, max_iter] and a
  // captured graphs of 2^g iterations (matvec + Arnoldi step each)
  int* ctl;
  const int* ctl_active;         // non-null while the iteration is captured
  hipStream_t gstream;           // private stream of kfbi_solve (graph launches)
  hipEvent_t ev_in, ev_out;
  hipGraph_t graphs[KFBI_NGRAPH];
  hipGraphExec_t graph_execs[KFBI_NGRAPH];  // graph g runs 2^g iterations
  hipGraph_t graph_x;            // graph_xn iterations (a repeated first batch that is no power of two)
  hipGraphExec_t graph_xe;
  int graph_xn;
  uint64_t graph_key[20];
  int graph_uses;                // solves run with the current graph key
  int* h_ctl;
  KfbiMailbox* mbox;             // pinned; see kfbi_post_wait
  PostReq colloc_req;            // the collocation's status post, collected after the folds are enqueued
  unsigned colloc_seq;
  unsigned mseq;
  // box-solve event timing
  int prof_on;
  std::vector<hipEvent_t>* prof_ev;
  int64_t prof_launches;
};

// ---------------------------------------------------------------- errors
void kfbi_set_error(const char* fmt, ...);
kfbi_status kfbi_hip_status(hipError_t e, const char* what);
kfbi_status kfbi_flags_status(int flags);

#define HIPCHK(call)                                              \
  do {                                                            \
    hipError_t e_ = (call);                                       \
    if (e_ != hipSuccess) return kfbi_hip_status(e_, #call);      \
  } while (0)

#define KCHK(call)                                                \
  do {                                                            \
    kfbi_status s_ = (call);                                      \
    if (s_ != KFBI_OK) return s_;                                 \
  } while (0)

// ---------------------------------------------------------------- launchers
// api.hip: enqueue k_post on the plan's stream and wait for its values by
// spinning on the pinned sequence word (a few microseconds sooner than a
// device-to-host copy and a stream synchronisation); after 2 ms of spinning
// it falls back to a stream synchronisation, which also reports a device
// error.  iout / dout receive r.ni ints and r.nd (+1 with a maximum) doubles.
kfbi_status kfbi_post_wait(kfbi_plan* pl, const PostReq& r, int* iout, double* dout);
// the two halves of kfbi_post_wait: enqueue k_post (returns its sequence
// number), and wait for it (other work may be enqueued in between)
kfbi_status kfbi_post_launch(kfbi_plan* pl, const PostReq& r, unsigned* seq);
kfbi_status kfbi_post_collect(kfbi_plan* pl, const PostReq& r, unsigned seq, int* iout, double* dout);

// geometry.hip (step S0)
kfbi_status geo_setup(kfbi_plan* pl);
// collocation.hip (step S1)
kfbi_status colloc_factor(kfbi_plan* pl);      // enqueues the factorisation and its status post
kfbi_status colloc_finish(kfbi_plan* pl);      // waits for that post: status flags, largest condition number
// operator.hip (steps S2, S4, S5 and right-hand sides)
void op_extend(kfbi_plan* pl, const double* psi, double* psiS);
void op_coefficients(kfbi_plan* pl, const double* a, const double* b, const double* ftilde,
                     double bscale = 1.0, double fscale = 1.0);
void op_correction_values(kfbi_plan* pl);
// fsel: fhat of every region (0), of the interiors only (1), of the exterior only (2)
void op_rhs_base(kfbi_plan* pl, const double* fhat, const double* gB, double* F, bool corrected = false,
                 int fsel = 0);
// one-sided values at the DOFs with the value weights (two-density plans)
void op_values(kfbi_plan* pl, const double* v, double* v_in, double* v_out);
// folded interpolation of the density x (values or normal derivatives)
void op_interp_folded(kfbi_plan* pl, const double* v, const double* x, double* t_in, double* t_out, bool values);
void dst_solve_corrections(kfbi_plan* pl, const double* psi, double* v);
void op_rhs_correct(kfbi_plan* pl, double* F, bool overwrite);
void op_boundary(kfbi_plan* pl, const double* gB, double* v);
void op_normal_derivatives(kfbi_plan* pl, const double* v, double* dn_in, double* dn_out,
                           double* Apsi);
kfbi_status op_fold(kfbi_plan* pl);
void op_matvec(kfbi_plan* pl, const double* psi, double* Apsi);
void op_matvec_head(kfbi_plan* pl, const double* psi);
void op_matvec_tail(kfbi_plan* pl, const double* psi, double* Apsi);
bool op_zero_mean_used(const kfbi_plan* pl);
void op_bie_rhs(kfbi_plan* pl, const double* g2, const double* dn_in, const double* dn_out,
                double* b);
// twodensity.hip (eq. bie-ifp-1)
kfbi_status td_setup(kfbi_plan* pl);
void td_free(kfbi_plan* pl);
kfbi_status td_matvec(kfbi_plan* pl, const double* x, double* out);
kfbi_status td_rhs(kfbi_plan* pl, const kfbi_data* d, double* b);
kfbi_status td_solve(kfbi_plan* pl, const kfbi_data* d, const kfbi_opts* o, double* x, double* u, kfbi_info* info);
// api.hip: plan creation without the capture lock (for a plan made inside
// another's set-up), the box solve of the plan's solver, a plan's release
kfbi_status plan_create_impl(const kfbi_problem* prob, hipStream_t stream, kfbi_plan** out, bool is_aux = false);
void plan_box_solve(kfbi_plan* pl, const double* F, double* v);
kfbi_status plan_resetup(kfbi_plan* pl, const kfbi_problem* prob);   // S0 + S1 for another problem
void plan_release(kfbi_plan* pl);
// dst.hip (step S3)
kfbi_status dst_init(kfbi_plan* pl);
// the tile autotuner of the sine-transform passes of grid g (once per grid
// and process), on that grid's tables and pass buffers
kfbi_status dst_autotune_grid(const GridDesc& g, const double* tw, const double* eig1, double* T1, double* T2,
                              hipStream_t st);
void dst_solve(kfbi_plan* pl, const double* F, double* v);
// Graph capture takes this exclusively; plan creation, set-up, buffer
// growth and destruction (allocations, frees and host copies, which may
// synchronise with other streams) take it shared, so several host threads
// can drive their own plans while one of them captures.
extern std::shared_mutex kfbi_capture_mutex;

// capacity for n elements when a plan's buffer grows: twice the need, so
// that a plan set up again for problems of varying size reallocates (and
// synchronises the device on the frees) a few times, not at every new
// largest problem
inline int64_t kfbi_headroom(int64_t n) { return 2 * n + 64; }

kfbi_status mg_configure(kfbi_plan* pl, int solver, double eps, int maxit);
// exact solve A_h v = F (zero box data) of the grid g by the sine transform
// with the given tables and pass buffers; skipped when ctl[1] (GMRES
// converged) or mctl[0] (multigrid converged) is set.  With rsrc (3D only)
// F is not read: the first pass forms F on load as the full weighting of
// the fine residual rsrc (FP32 if rsrc_f32, else FP64; n1f nodes per axis,
// the fine grid twice g's), in that precision, taken to FP64
void dst_solve_grid(const GridDesc& g, const double* tw, const double* eig1, double* T1, double* T2,
                    const double* F, double* v, const int* ctl, const int* mctl, hipStream_t st,
                    const void* rsrc = nullptr, int rsrc_f32 = 0, int n1f = 0);
// twiddles exp(-2 pi i m / 2N) (m < 2N, interleaved re, im) and the 1D
// eigenvalues s_k = -4/h^2 sin^2(k pi / 2N) (k <= N) of the sine transform
void dst_host_tables(int N, double h, double* tw, double* eig1);
// v = A_h^-1 F to eps_in (at most mg_run_cap corrections), sent as a
// captured graph when the stream is not being captured itself
void mg_solve(kfbi_plan* pl, const double* F, double* v);
void mg_graphs_clear(kfbi_plan* pl);
void mg_matvec_rhs(kfbi_plan* pl);
// the box-solution store of a solve (see kfbi_plan::ustore)
kfbi_status mg_store_reserve(kfbi_plan* pl);
void mg_store_solution(kfbi_plan* pl, const double* v);
void mg_guess_from_store(kfbi_plan* pl, int k, int use_x0, const double* y, double* v);
void mg_sum(kfbi_plan* pl, const double* a, const double* b, double* out);
// out = a - b over n entries; v = 0 over the grid (fill kernels, safe under capture)
void vec_diff(kfbi_plan* pl, int64_t n, const double* a, const double* b, double* out);
void grid_zero(kfbi_plan* pl, double* v);
void dst_solve_corrections(kfbi_plan* pl, const double* psi, double* v);
// the matvec box solves of G plans of one grid shape (FFT solver) as one
// launch per pass; each plan's GMRES control word stops its own work
struct DstBatch;
DstBatch* dst_batch_create(kfbi_plan* const* pls, int G, hipStream_t st, kfbi_status* status);
void dst_batch_corrections(DstBatch* b, hipStream_t st);
void dst_batch_destroy(DstBatch* b);
// Alg. 1 for G set-up plans of one grid shape with the FFT box solver,
// their GMRES iterations in lockstep with batched box-solve passes, on st
// (api.hip); psi[p] (n_dof) and u[p] ((N+1)^d) device arrays per problem;
// infos[p] filled for every problem.
kfbi_status kfbi_solve_group(kfbi_plan* const* pls, int G, const kfbi_data* data, double* const* psi,
                             double* const* u, const kfbi_opts* opts, hipStream_t st, kfbi_info* infos);
// gmres.hip (step S6)
void gm_residual_start(kfbi_plan* pl, const double* b, const double* Ax0, int use_x0, double tol, int maxit);
void gm_arnoldi(kfbi_plan* pl);
int gm_part_blocks(int64_t n);
void gm_update(kfbi_plan* pl, int k, double* x, int use_x0);
void gm_update_device(kfbi_plan* pl, double* x, int use_x0);
void gm_true_residual(kfbi_plan* pl, const double* b, const double* Ax, double* out2);

// ---------------------------------------------------------------- device helpers
__host__ __device__ inline int kfbi_ncoef(int d, int p) {
  return d == 2 ? (p + 1) * (p + 2) / 2 : (p + 1) * (p + 2) * (p + 3) / 6;
}

// the FFT matvec precomputes F at the irregular nodes (one 32-lane group
// per node) when the pair tables are long (3D, 4th order: up to 26 pairs)
inline bool kfbi_irr_rhs_used(const kfbi_plan* pl) { return pl->maxpairs > 8 && pl->maxpairs <= 32; }

// The work groups of a launch are dealt to the chip's 8 XCDs in turn (group
// b runs on XCD b mod 8) and every XCD has an L2 of its own.  This maps b to
// a logical index under which each XCD takes one contiguous range, so that
// neighbouring tiles, which share cache lines, meet in the same L2.  A
// bijection of [0, nb) for every nb.
__device__ __forceinline__ int kfbi_xcd_block(int b, int nb) {
  const int q = nb >> 3, r = nb & 7, x = b & 7;
  return x * q + (x < r ? x : r) + (b >> 3);
}
