// Host side of the C ABI: plan life cycle, table export and the solve
// orchestration (Alg. 1 of the paper: right-hand side, GMRES over the
// simple-interface-problem operator, final solve).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <chrono>
#include <new>

#include "kfbi_internal.h"

void kfbi_pde_lattice(int d, int p, int (*off)[3], int* n);
void kfbi_dn_lattice(int D, int m, int (*off)[2], int* n);

std::shared_mutex kfbi_capture_mutex;

namespace {

thread_local char g_err[512] = "no error";

void destroy_graphs(kfbi_plan* pl);

template <class T>
kfbi_status dalloc(T** p, int64_t n) {
  *p = nullptr;
  if (n <= 0) n = 1;
  if (hipMalloc((void**)p, (size_t)n * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    kfbi_set_error("device allocation of %lld bytes failed", (long long)(n * sizeof(T)));
    return KFBI_E_OOM;
  }
  return KFBI_OK;
}

template <class T>
void dfree(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

kfbi_status check_problem(const kfbi_problem* pr) {
  if (!pr) {
    kfbi_set_error("problem descriptor is NULL");
    return KFBI_E_INVALID;
  }
  if (pr->dim != 2 && pr->dim != 3) {
    kfbi_set_error("dim must be 2 or 3 (got %d)", pr->dim);
    return KFBI_E_INVALID;
  }
  if (pr->order != 2 && pr->order != 4) {
    kfbi_set_error("order must be 2 or 4 (got %d)", pr->order);
    return KFBI_E_INVALID;
  }
  if (pr->N < 8 || pr->N > 1024 || (pr->N & (pr->N - 1))) {
    kfbi_set_error("N must be a power of two in [8, 1024] (got %d)", pr->N);
    return KFBI_E_INVALID;
  }
  if (pr->n_iface < 1 || pr->n_iface > KFBI_MAX_IFACE) {
    kfbi_set_error("n_iface must be in [1, %d] (got %d)", KFBI_MAX_IFACE, pr->n_iface);
    return KFBI_E_INVALID;
  }
  if (pr->bie != KFBI_BIE_INTERFACE && pr->bie != KFBI_BIE_DIRICHLET && pr->bie != KFBI_BIE_NEUMANN &&
      pr->bie != KFBI_BIE_TWO_DENSITY) {
    kfbi_set_error("bie must be KFBI_BIE_INTERFACE, _DIRICHLET, _NEUMANN or _TWO_DENSITY (got %d)", pr->bie);
    return KFBI_E_INVALID;
  }
  const bool ifc = pr->bie == KFBI_BIE_INTERFACE || pr->bie == KFBI_BIE_TWO_DENSITY;
  const bool betas = !ifc || (pr->beta_in > 0.0 && pr->beta_out > 0.0);
  if (!(pr->hi > pr->lo) || !betas || !(pr->kappa >= 0.0) ||
      (pr->bie == KFBI_BIE_TWO_DENSITY && !(pr->kappa_out >= 0.0))) {
    kfbi_set_error("need hi > lo, beta_in > 0, beta_out > 0 (interface problems), kappa >= 0, kappa_out >= 0");
    return KFBI_E_INVALID;
  }
  if (!(pr->cos_alpha > 0.0) || !(pr->cos_alpha * pr->cos_alpha * pr->dim < 1.0)) {
    kfbi_set_error("cos_alpha must lie in (0, 1/sqrt(dim))");
    return KFBI_E_INVALID;
  }
  for (int k = 0; k < pr->n_iface; ++k) {
    int kind = pr->iface[k].kind;
    if (kind == KFBI_LS_GRID) {
      const double q = pr->iface[k].p[0];
      if (!(q == 3.0 || q == 5.0) || !pr->samples[k]) {
        kfbi_set_error("level set %d: a sampled level set needs degree 3 or 5 and samples", k);
        return KFBI_E_INVALID;
      }
      continue;
    }
    bool two = kind == KFBI_LS_ELLIPSE2D || kind == KFBI_LS_STAR2D;
    bool three = kind == KFBI_LS_SPHERE3D || kind == KFBI_LS_ELLIPSOID3D || kind == KFBI_LS_TORUS3D ||
                 kind == KFBI_LS_PRODUCT3D || kind == KFBI_LS_MOLECULE3D;
    if ((pr->dim == 2 && !two) || (pr->dim == 3 && !three)) {
      kfbi_set_error("level set %d: kind %d does not fit dim %d", k, kind, pr->dim);
      return KFBI_E_INVALID;
    }
    if (kind == KFBI_LS_MOLECULE3D) {
      const double m = pr->iface[k].p[2];
      if (!(m >= 1.0 && m <= 8.0 && m == (double)(int)m) || !(pr->iface[k].p[1] > 0.0)) {
        kfbi_set_error("level set %d: a molecule needs 1..8 atoms and r > 0", k);
        return KFBI_E_INVALID;
      }
    }
  }
  return KFBI_OK;
}

void free_plan(kfbi_plan* pl) {
  td_free(pl);
  dfree(pl->ls_samples);
  dfree(pl->region);
  dfree(pl->need);
  dfree(pl->Cg);
  dfree(pl->Fs);
  dfree(pl->T1);
  dfree(pl->T2);
  dfree(pl->vbuf);
  dfree(pl->vsbuf);
  dfree(pl->c_r);
  dfree(pl->c_lid);
  dfree(pl->c_seg);
  dfree(pl->c_k);
  dfree(pl->c_ina);
  dfree(pl->c_pos);
  dfree(pl->c_nrm);
  dfree(pl->c_acc);
  dfree(pl->s_pos);
  dfree(pl->s_nrm);
  dfree(pl->s_meta);
  dfree(pl->s2d);
  dfree(pl->d2s);
  dfree(pl->s_need);
  dfree(pl->line_start);
  dfree(pl->line_end);
  dfree(pl->stD);
  dfree(pl->stN);
  dfree(pl->ext_idx);
  dfree(pl->ext_w);
  dfree(pl->MinvT);
  dfree(pl->MT);
  if (pl->mg_u) (void)hipFree(pl->mg_u);
  if (pl->mg_t) (void)hipFree(pl->mg_t);
  if (pl->mg_f) (void)hipFree(pl->mg_f);
  dfree(pl->mg_Fc);
  dfree(pl->mg_Uc);
  dfree(pl->mg_T1c);
  dfree(pl->mg_T2c);
  dfree(pl->mg_twc);
  dfree(pl->mg_eigc);
  dfree(pl->mg_part);
  dfree(pl->mg_ctl);
  dfree(pl->mg_scal);
  dfree(pl->Fmg);
  dfree(pl->ustore);
  pl->ustore_slots = 0;
  pl->ustore_n = 0;
  dfree(pl->cond);
  dfree(pl->psiS);
  dfree(pl->aS);
  dfree(pl->U);
  dfree(pl->dn_in);
  dfree(pl->dn_out);
  dfree(pl->irr);
  dfree(pl->ce_k);
  dfree(pl->ce_node);
  dfree(pl->ce_owner);
  dfree(pl->cell_count);
  dfree(pl->cell_start);
  dfree(pl->cell_items);
  dfree(pl->cell_cursor);
  dfree(pl->blk);
  dfree(pl->blk_total);
  dfree(pl->d_flags);
  dfree(pl->tw);
  dfree(pl->eig1);
  dfree(pl->V);
  dfree(pl->gm_part);
  dfree(pl->Hm);
  dfree(pl->gv);
  dfree(pl->cs);
  dfree(pl->sn);
  dfree(pl->work);
  dfree(pl->work2);
  dfree(pl->bvec);
  dfree(pl->scal);
  dfree(pl->FI);
  dfree(pl->FW);
  dfree(pl->Cv);
  dfree(pl->GI);
  dfree(pl->GW);
  dfree(pl->IW);
  dfree(pl->IB);
  dfree(pl->HW);
  dfree(pl->TI);
  dfree(pl->IE2);
  dfree(pl->PA);
  dfree(pl->Firr);
  dfree(pl->sh_ws);
  dfree(pl->PE1);
  dfree(pl->PE2);
  dfree(pl->EI);
  dfree(pl->flags8);
  dfree(pl->flags8b);
  dfree(pl->blk2);
  dfree(pl->blk3);
  dfree(pl->row_start);
  dfree(pl->row_end);
  if (pl->prof_ev) {
    for (hipEvent_t e : *pl->prof_ev) (void)hipEventDestroy(e);
    delete pl->prof_ev;
    pl->prof_ev = nullptr;
  }
  destroy_graphs(pl);
  mg_graphs_clear(pl);
  if (pl->gstream) (void)hipStreamDestroy(pl->gstream);
  if (pl->ev_in) (void)hipEventDestroy(pl->ev_in);
  if (pl->ev_out) (void)hipEventDestroy(pl->ev_out);
  pl->gstream = nullptr;
  pl->ev_in = pl->ev_out = nullptr;
  dfree(pl->ctl);
  if (pl->h_ctl) (void)hipHostFree(pl->h_ctl);
  pl->h_ctl = nullptr;
  if (pl->h_pinned) (void)hipHostFree(pl->h_pinned);
  if (pl->h_dpinned) (void)hipHostFree(pl->h_dpinned);
  if (pl->mbox) (void)hipHostFree(pl->mbox);
  pl->mbox = nullptr;
  pl->h_pinned = nullptr;
  pl->h_dpinned = nullptr;
}

GridDesc make_grid(const kfbi_problem& pr) {
  GridDesc g;
  g.d = pr.dim;
  g.order = pr.order;
  g.p = pr.order == 4 ? 4 : 2;
  g.N = pr.N;
  g.n1 = pr.N + 1;
  g.K = pr.n_iface;
  g.lo = pr.lo;
  g.hi = pr.hi;
  g.h = (pr.hi - pr.lo) / pr.N;
  g.kappa = pr.kappa;
  g.cos_alpha = pr.cos_alpha;
  g.bie = pr.bie;
  // a boundary value problem's operator is the interior one-sided limit:
  // the interface combination with weights 1 inside and 0 outside
  const bool bvp = pr.bie == KFBI_BIE_DIRICHLET || pr.bie == KFBI_BIE_NEUMANN;
  g.beta_in = bvp ? 1.0 : pr.beta_in;
  g.beta_out = bvp ? 0.0 : pr.beta_out;
  g.n_nodes = 1;
  for (int a = 0; a < g.d; ++a) g.n_nodes *= g.n1;
  return g;
}

// grid-sized and fixed buffers of a plan
kfbi_status alloc_fixed(kfbi_plan* pl) {
  const GridDesc& g = pl->g;
  int64_t n = g.n_nodes;
  KCHK(dalloc(&pl->region, n));
  KCHK(dalloc(&pl->need, (int64_t)g.K * n));
  KCHK(dalloc(&pl->Cg, (int64_t)g.K * n));
  KCHK(dalloc(&pl->Fs, n));
  KCHK(dalloc(&pl->T1, n));
  KCHK(dalloc(&pl->T2, n));
  KCHK(dalloc(&pl->vbuf, n));
  HIPCHK(hipMemsetAsync(pl->vbuf, 0, sizeof(double) * n, pl->stream));   // box boundary: never written again
  KCHK(dalloc(&pl->vsbuf, n));
  KCHK(dalloc(&pl->flags8, pl->n_seg * g.K > n ? pl->n_seg * g.K : n));
  KCHK(dalloc(&pl->EI, (int64_t)g.K * n));
  KCHK(dalloc(&pl->flags8b, n));
  int64_t nrows = g.d == 3 ? (int64_t)g.n1 * g.n1 : g.n1;
  KCHK(dalloc(&pl->row_start, nrows));
  KCHK(dalloc(&pl->row_end, nrows));
  KCHK(dalloc(&pl->line_start, pl->n_lines));
  KCHK(dalloc(&pl->line_end, pl->n_lines));
  int64_t nkeys = (int64_t)g.K * pl->ncell;
  KCHK(dalloc(&pl->cell_count, nkeys + 1));
  KCHK(dalloc(&pl->cell_start, nkeys + 1));
  KCHK(dalloc(&pl->cell_cursor, nkeys + 1));
  KCHK(dalloc(&pl->blk_total, 4));
  KCHK(dalloc(&pl->d_flags, 4));
  KCHK(dalloc(&pl->tw, 4 * g.N));
  KCHK(dalloc(&pl->eig1, g.N + 1));
  KCHK(dalloc(&pl->scal, 16 + KFBI_GMRES_MAX + 8));
  KCHK(dalloc(&pl->Hm, (int64_t)(KFBI_GMRES_MAX + 1) * (KFBI_GMRES_MAX + 1)));
  KCHK(dalloc(&pl->gv, KFBI_GMRES_MAX + 1));
  KCHK(dalloc(&pl->cs, KFBI_GMRES_MAX));
  KCHK(dalloc(&pl->sn, KFBI_GMRES_MAX));
  if (hipHostMalloc((void**)&pl->h_pinned, 64 * sizeof(int), 0) != hipSuccess) {
    kfbi_set_error("pinned host allocation failed");
    return KFBI_E_OOM;
  }
  if (hipHostMalloc((void**)&pl->h_dpinned, 64 * sizeof(double), 0) != hipSuccess) {
    kfbi_set_error("pinned host allocation failed");
    return KFBI_E_OOM;
  }
  if (hipHostMalloc((void**)&pl->mbox, sizeof(KfbiMailbox), 0) != hipSuccess) {
    kfbi_set_error("pinned host allocation failed");
    return KFBI_E_OOM;
  }
  memset((void*)pl->mbox, 0, sizeof(KfbiMailbox));
  if (hipHostMalloc((void**)&pl->h_ctl, 16 * sizeof(int), 0) != hipSuccess) {
    kfbi_set_error("pinned host allocation failed");
    return KFBI_E_OOM;
  }
  KCHK(dalloc(&pl->ctl, 8));
  // the private stream of solves on a default stream and its two events
  // are made on first use (a stream costs about 1.5 ms to create)
  return KFBI_OK;
}

kfbi_status run_setup(kfbi_plan* pl) {
  pl->ready = false;
  KCHK(geo_setup(pl));
  KCHK(colloc_factor(pl));
  // the folds go out before the host waits for the collocation's status
  // (they do nothing when a status flag is set)
  KCHK(op_fold(pl));
  KCHK(colloc_finish(pl));
  if (pl->g.bie == KFBI_BIE_TWO_DENSITY && !pl->is_aux) KCHK(td_setup(pl));
  // the multigrid matvec right-hand side is zero away from the irregular nodes
  if (pl->Fmg) HIPCHK(hipMemsetAsync(pl->Fmg, 0, sizeof(double) * pl->g.n_nodes, pl->stream));
  // everything after the set-up is ordered behind it on the plan's stream
  HIPCHK(hipGetLastError());
  pl->ready = true;
  return KFBI_OK;
}

kfbi_status need_ready(const kfbi_plan* pl) {
  if (!pl) {
    kfbi_set_error("plan is NULL");
    return KFBI_E_INVALID;
  }
  if (!pl->ready) {
    kfbi_set_error("plan set-up did not complete");
    return KFBI_E_INVALID;
  }
  return KFBI_OK;
}

kfbi_status ensure_gmres(kfbi_plan* pl, int m) {
  if (m <= pl->gm_cap && pl->n_dof <= pl->gm_n && pl->V) return KFBI_OK;
  dfree(pl->V);
  dfree(pl->gm_part);
  int mm = m > pl->gm_cap ? m : pl->gm_cap;
  KCHK(dalloc(&pl->V, (int64_t)(mm + 1) * pl->cap_dof));
  pl->gm_pb = gm_part_blocks(pl->cap_dof);
  KCHK(dalloc(&pl->gm_part, (int64_t)3 * pl->gm_pb * (mm + 2)));
  pl->gm_cap = mm;
  pl->gm_n = pl->cap_dof;
  return KFBI_OK;
}

void box_solve_any(kfbi_plan* pl, const double* F, double* v) {
  if (pl->box_solver == KFBI_BOX_FFT)
    dst_solve(pl, F, v);
  else
    mg_solve(pl, F, v);
}

void simple_solve_impl(kfbi_plan* pl, const double* a, const double* b, const double* ftilde,
                       const double* fhat, const double* gB, double* v, double* dn_in, double* dn_out) {
  op_coefficients(pl, a, b, ftilde);
  op_correction_values(pl);
  op_rhs_base(pl, fhat, gB, pl->Fs, true);   // corrected at the irregular nodes in the same pass
  box_solve_any(pl, pl->Fs, v);
  op_boundary(pl, gB, v);
  op_normal_derivatives(pl, v, dn_in, dn_out, nullptr);
}

void matvec_impl(kfbi_plan* pl, const double* psi, double* Apsi) { op_matvec(pl, psi, Apsi); }

// Alg. 1 Step 1: the BIE right-hand side into b, its grid solution into
// vsbuf.  A boundary value problem has no jump data and zero box data.
void rhs_impl(kfbi_plan* pl, const kfbi_data& d, double* b) {
  const bool ifc = pl->g.bie == KFBI_BIE_INTERFACE;
  simple_solve_impl(pl, ifc ? d.g1 : nullptr, nullptr, d.ftilde, d.fhat, ifc ? d.gB : nullptr, pl->vsbuf,
                    pl->dn_in, pl->dn_out);
  op_bie_rhs(pl, d.g2, pl->dn_in, pl->dn_out, b);
}

// the grid solution of the density psi: w(g1, E psi, ftilde, fhat, gB); of
// a Dirichlet problem w(E phi, 0, ftilde, fhat, 0) (the density is [u]),
// of a Neumann problem w(0, E psi, ftilde, fhat, 0)
void final_impl(kfbi_plan* pl, const kfbi_data& d, const double* psi, double* u) {
  op_extend(pl, psi, pl->aS);
  if (pl->g.bie == KFBI_BIE_DIRICHLET)
    simple_solve_impl(pl, pl->aS, nullptr, d.ftilde, d.fhat, nullptr, u, pl->dn_in, pl->dn_out);
  else if (pl->g.bie == KFBI_BIE_NEUMANN)
    simple_solve_impl(pl, nullptr, pl->aS, d.ftilde, d.fhat, nullptr, u, pl->dn_in, pl->dn_out);
  else
    simple_solve_impl(pl, d.g1, pl->aS, d.ftilde, d.fhat, d.gB, u, pl->dn_in, pl->dn_out);
}

void destroy_graphs(kfbi_plan* pl) {
  if (pl->graph_xe) (void)hipGraphExecDestroy(pl->graph_xe);
  if (pl->graph_x) (void)hipGraphDestroy(pl->graph_x);
  pl->graph_xe = nullptr;
  pl->graph_x = nullptr;
  pl->graph_xn = 0;
  for (int v = 0; v < KFBI_NGRAPH; ++v) {
    if (pl->graph_execs[v]) (void)hipGraphExecDestroy(pl->graph_execs[v]);
    if (pl->graphs[v]) (void)hipGraphDestroy(pl->graphs[v]);
    pl->graph_execs[v] = nullptr;
    pl->graphs[v] = nullptr;
  }
}

// cap of a relaxed box solve launched when the host's latest GMRES
// residual estimate is res (|b| = nb): its tolerance relax tol |b| / res,
// clamped to [eps_in, 1e-1], reached at the two-grid cycle's contraction
// (0.07 per correction, 0.085 taken).  The device applies the same rule
// with the iteration's own estimate, which is no larger, so it needs no
// more.  0 means the plan-wide cap (no estimate, or no smaller cap).
int relaxed_cap(const kfbi_plan* pl, double tol, double nb, double res) {
  if (pl->box_solver == KFBI_BOX_FFT || !(pl->relax_word > 0.0) || !(res > 0.0) || !(nb > 0.0)) return 0;
  const int full = pl->mg_run_cap > 0 ? pl->mg_run_cap : pl->mg_maxit;
  double e = pl->relax_word * tol * nb / res;
  if (e > 1e-1) e = 1e-1;
  if (e < pl->mg_eps) e = pl->mg_eps;
  const int c = (int)ceil(log(e) / log(0.085));
  return c >= 1 && c < full ? c : 0;
}

// one GMRES iteration with a multigrid box solver, enqueued as it goes: the
// few kernels of the matvec that depend on the interfaces, the captured box
// solve (capped at mg_run_cap corrections), the store of its solution, the
// Arnoldi step.  Every kernel reads j and the stop flag from the device
// control word, so iterations enqueued past convergence do nothing.
void enqueue_mg_iteration(kfbi_plan* pl) {
  pl->ctl_active = pl->ctl;
  op_matvec(pl, nullptr, nullptr);
  mg_store_solution(pl, pl->vbuf);
  gm_arnoldi(pl);
  pl->ctl_active = nullptr;
}

// FFT box solver: captured iterations (matvec + Arnoldi step)
kfbi_status capture_iterations(kfbi_plan* pl, int iters, hipGraph_t* gr_out, hipGraphExec_t* ex_out) {
  HIPCHK(hipStreamBeginCapture(pl->stream, hipStreamCaptureModeThreadLocal));
  pl->ctl_active = pl->ctl;
  for (int it = 0; it < iters; ++it) {
    op_matvec(pl, nullptr, nullptr);
    gm_arnoldi(pl);
  }
  pl->ctl_active = nullptr;
  hipGraph_t gr = nullptr;
  hipError_t e = hipStreamEndCapture(pl->stream, &gr);
  if (e != hipSuccess) return kfbi_hip_status(e, "hipStreamEndCapture");
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(gr);
    return kfbi_hip_status(e, "hipGraphInstantiate");
  }
  *gr_out = gr;
  *ex_out = ex;
  return KFBI_OK;
}

// Graphs of one and of four GMRES iterations (matvec of V[j] into V[j+1],
// Arnoldi step),
// captured on the private stream; every kernel reads j and the stop flag
// from the device control word.  Rebuilt when buffers or sizes change.
// Graph v runs 2^v iterations.  Each graph launch costs a few microseconds
// of idle time at its boundaries, so a batch is sent as few graphs as
// possible, but capturing and instantiating a graph costs about as much as
// launching its kernels, so a graph set is only worth it when the key is
// reused: the first solve with a key captures the graphs of 1 and 4
// iterations, later solves all.  Multigrid iterations are enqueued kernel by
// kernel around captured box solves (enqueue_mg_iteration), which stay
// valid from one geometry to the next.
bool graph_wanted(const kfbi_plan* pl, int v) {
  if (pl->box_solver != KFBI_BOX_FFT) return false;
  return pl->graph_uses > 0 || v == 0 || v == 2;
}

kfbi_status ensure_graph(kfbi_plan* pl) {
  uint64_t bi, bo, ka;
  memcpy(&bi, &pl->g.beta_in, 8);
  memcpy(&bo, &pl->g.beta_out, 8);
  memcpy(&ka, &pl->g.kappa, 8);
  uint64_t key[20] = {bi, bo, ka, (uint64_t)pl->box_solver * 1000003u + (uint64_t)(pl->mg_run_cap > 0 ? pl->mg_run_cap : pl->mg_maxit),(uint64_t)pl->n_dof, (uint64_t)pl->n_surf, (uint64_t)pl->n_corr, (uint64_t)pl->n_irr,
                      (uint64_t)(uintptr_t)pl->V, (uint64_t)(uintptr_t)pl->psiS, (uint64_t)(uintptr_t)pl->Cg,
                      (uint64_t)(uintptr_t)pl->FI, (uint64_t)(uintptr_t)pl->IW, (uint64_t)(uintptr_t)pl->stN,
                      (uint64_t)(uintptr_t)pl->ext_idx, (uint64_t)(uintptr_t)pl->irr,
                      (uint64_t)(uintptr_t)pl->ce_node, (uint64_t)pl->gm_cap, (uint64_t)(uintptr_t)pl->d2s,
                      (uint64_t)(uintptr_t)pl->PA ^ (uint64_t)(uintptr_t)pl->GI ^ (uint64_t)(uintptr_t)pl->mg_u ^
                          (uint64_t)(uintptr_t)pl->ustore};
  if (!pl->graph_execs[0] || memcmp(key, pl->graph_key, sizeof(key)) != 0) {
    destroy_graphs(pl);
    pl->graph_uses = 0;
    memcpy(pl->graph_key, key, sizeof(key));
  }
  bool want[KFBI_NGRAPH], missing = false;
  for (int v = 0; v < KFBI_NGRAPH; ++v) {
    want[v] = graph_wanted(pl, v) && !pl->graph_execs[v];
    missing = missing || want[v];
  }
  ++pl->graph_uses;
  if (!missing) return KFBI_OK;
  std::unique_lock<std::shared_mutex> lock(kfbi_capture_mutex);
  for (int v = 0; v < KFBI_NGRAPH; ++v)
    if (want[v]) KCHK(capture_iterations(pl, 1 << v, &pl->graphs[v], &pl->graph_execs[v]));
  return KFBI_OK;
}


}  // namespace

// ---------------------------------------------------------------- device posts
namespace {
__global__ void __launch_bounds__(1024) k_post(PostReq r, KfbiMailbox* mb, unsigned seq) {
  __shared__ double red[16];
  double mx = 0.0;
  if (r.nmax > 0) {
    for (int64_t i = threadIdx.x; i < r.nmax; i += 1024) {
      const double v = r.maxsrc[i];
      mx = (v > mx || v != v) ? v : mx;
    }
    for (int off = 32; off > 0; off >>= 1) {
      const double v = __shfl_xor(mx, off, 64);
      mx = (v > mx || v != v) ? v : mx;
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  for (int i = 0; i < r.ni; ++i)
    __hip_atomic_store(&mb->iv[i], *r.isrc[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  for (int i = 0; i < r.nd; ++i)
    __hip_atomic_store(&mb->dv[i], (unsigned long long)__double_as_longlong(*r.dsrc[i]), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_SYSTEM);
  if (r.nmax > 0) {
    double m = 0.0;
    for (int w = 0; w < 16; ++w) m = (red[w] > m || red[w] != red[w]) ? red[w] : m;
    __hip_atomic_store(&mb->dv[r.nd], (unsigned long long)__double_as_longlong(m), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_SYSTEM);
  }
  __hip_atomic_store(&mb->seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}
}  // namespace

kfbi_status kfbi_post_wait(kfbi_plan* pl, const PostReq& r, int* iout, double* dout) {
  if (r.ni > 8 || r.nd > 8 || (r.nmax > 0 && r.nd > 7)) {
    kfbi_set_error("post request too large");
    return KFBI_E_INVALID;
  }
  unsigned seq = 0;
  KCHK(kfbi_post_launch(pl, r, &seq));
  return kfbi_post_collect(pl, r, seq, iout, dout);
}

kfbi_status kfbi_post_launch(kfbi_plan* pl, const PostReq& r, unsigned* seq) {
  if (r.ni > 8 || r.nd > 8 || (r.nmax > 0 && r.nd > 7)) {
    kfbi_set_error("post request too large");
    return KFBI_E_INVALID;
  }
  *seq = ++pl->mseq == 0 ? ++pl->mseq : pl->mseq;
  hipLaunchKernelGGL(k_post, dim3(1), dim3(1024), 0, pl->stream, r, pl->mbox, *seq);
  HIPCHK(hipGetLastError());
  return KFBI_OK;
}

kfbi_status kfbi_post_collect(kfbi_plan* pl, const PostReq& r, unsigned seq, int* iout, double* dout) {
  const auto t0 = std::chrono::steady_clock::now();
  for (long s = 1;; ++s) {
    if (__atomic_load_n(&pl->mbox->seq, __ATOMIC_ACQUIRE) == seq) break;
    if ((s & 1023) == 0 && std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(2)) {
      HIPCHK(hipStreamSynchronize(pl->stream));
      if (__atomic_load_n(&pl->mbox->seq, __ATOMIC_ACQUIRE) != seq) {
        kfbi_set_error("device values were not posted");
        return KFBI_E_DEVICE;
      }
      break;
    }
  }
  for (int i = 0; i < r.ni; ++i) iout[i] = __atomic_load_n(&pl->mbox->iv[i], __ATOMIC_RELAXED);
  const int nd = r.nd + (r.nmax > 0 ? 1 : 0);
  for (int i = 0; i < nd; ++i) {
    const unsigned long long b = __atomic_load_n(&pl->mbox->dv[i], __ATOMIC_RELAXED);
    memcpy(&dout[i], &b, 8);
  }
  return KFBI_OK;
}

// ---------------------------------------------------------------- errors
void kfbi_set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

kfbi_status kfbi_hip_status(hipError_t e, const char* what) {
  kfbi_set_error("HIP error %d (%s) in %s", (int)e, hipGetErrorString(e), what);
  return e == hipErrorOutOfMemory ? KFBI_E_OOM : KFBI_E_DEVICE;
}

kfbi_status kfbi_flags_status(int f) {
  if (f & (FLAG_OVERLAP | FLAG_MARGIN)) {
    kfbi_set_error("invalid geometry:%s%s", f & FLAG_OVERLAP ? " interface interiors overlap" : "",
                   f & FLAG_MARGIN ? " interface too close to the box boundary" : "");
    return KFBI_E_INVALID;
  }
  if (f & (FLAG_UNRESOLVED_STENCIL | FLAG_UNRESOLVED_EXT | FLAG_UNRESOLVED_OWNER)) {
    kfbi_set_error("geometry not resolved by the grid:%s%s%s",
                   f & FLAG_UNRESOLVED_STENCIL ? " no collocation stencil" : "",
                   f & FLAG_UNRESOLVED_EXT ? " no density interpolation stencil" : "",
                   f & FLAG_UNRESOLVED_OWNER ? " no closest centre" : "");
    return KFBI_E_UNRESOLVED;
  }
  if (f & FLAG_SINGULAR) {
    kfbi_set_error("singular collocation matrix");
    return KFBI_E_SINGULAR;
  }
  if (f & FLAG_NONFINITE) {
    kfbi_set_error("non-finite data");
    return KFBI_E_NONFINITE;
  }
  kfbi_set_error("device flags 0x%x", f);
  return KFBI_E_DEVICE;
}

extern "C" const char* kfbi_last_error(void) { return g_err; }

// ---------------------------------------------------------------- plan
extern "C" kfbi_status kfbi_plan_create(const kfbi_problem* prob, void* stream, kfbi_plan** out) {
  std::shared_lock<std::shared_mutex> lock(kfbi_capture_mutex);
  return plan_create_impl(prob, (hipStream_t)stream, out);
}

void plan_box_solve(kfbi_plan* pl, const double* F, double* v) { box_solve_any(pl, F, v); }

kfbi_status plan_resetup(kfbi_plan* pl, const kfbi_problem* prob) {
  pl->prob = *prob;
  pl->g = make_grid(*prob);
  return run_setup(pl);
}

void plan_release(kfbi_plan* pl) {
  free_plan(pl);
  delete pl;
}

kfbi_status plan_create_impl(const kfbi_problem* prob, hipStream_t stream, kfbi_plan** out, bool is_aux) {
  if (!out) {
    kfbi_set_error("out is NULL");
    return KFBI_E_INVALID;
  }
  *out = nullptr;
  KCHK(check_problem(prob));
  kfbi_plan* pl = new (std::nothrow) kfbi_plan();
  if (!pl) {
    kfbi_set_error("host allocation failed");
    return KFBI_E_OOM;
  }
  memset((void*)pl, 0, sizeof(*pl));
  pl->relax_word = NAN;
  pl->is_aux = is_aux;
  pl->prob = *prob;
  pl->g = make_grid(*prob);
  pl->stream = (hipStream_t)stream;
  const GridDesc& g = pl->g;
  int p = g.p, d = g.d;
  pl->nC = kfbi_ncoef(d, p);
  {
    int offP[KFBI_MAXP][3], offD[KFBI_MAXD][2], offN[KFBI_MAXN][2];
    kfbi_pde_lattice(d, p, offP, &pl->nP);
    kfbi_dn_lattice(d - 1, p, offD, &pl->nD);
    kfbi_dn_lattice(d - 1, p - 1, offN, &pl->nN);
  }
  int64_t L = d == 2 ? g.n1 : (int64_t)g.n1 * g.n1;
  pl->n_seg = (int64_t)d * g.N * L;
  pl->n_lines = (int64_t)d * L;
  pl->ncell_axis = g.N / 2 + 1;
  pl->ncell = 1;
  for (int a = 0; a < d; ++a) pl->ncell *= pl->ncell_axis;
  kfbi_status st = alloc_fixed(pl);
  if (st == KFBI_OK) st = dst_init(pl);
  *out = pl;
  if (st != KFBI_OK) return st;
  return run_setup(pl);
}

extern "C" kfbi_status kfbi_plan_setup(kfbi_plan* pl, const kfbi_problem* prob) {
  std::shared_lock<std::shared_mutex> lock(kfbi_capture_mutex);
  if (!pl) {
    kfbi_set_error("plan is NULL");
    return KFBI_E_INVALID;
  }
  KCHK(check_problem(prob));
  if (prob->dim != pl->prob.dim || prob->order != pl->prob.order || prob->N != pl->prob.N ||
      prob->n_iface != pl->prob.n_iface || prob->lo != pl->prob.lo || prob->hi != pl->prob.hi ||
      prob->bie != pl->prob.bie) {
    kfbi_set_error("kfbi_plan_setup needs the same dim, order, N, n_iface, box and bie");
    return KFBI_E_INVALID;
  }
  pl->prob = *prob;
  pl->g = make_grid(*prob);
  return run_setup(pl);
}

extern "C" kfbi_status kfbi_plan_sizes(const kfbi_plan* pl, kfbi_sizes* out) {
  if (!pl || !out) {
    kfbi_set_error("NULL argument");
    return KFBI_E_INVALID;
  }
  out->n_nodes = pl->g.n_nodes;
  out->n_surf = pl->n_surf;
  out->n_dof = pl->n_dof;
  out->n_irregular = pl->n_irr;
  out->n_corr = pl->n_corr;
  out->n_pde = pl->nP;
  out->n_dir = pl->nD;
  out->n_neu = pl->nN;
  out->n_coef = pl->nC;
  out->h = pl->g.h;
  out->cond_max = pl->cond_max;
  return KFBI_OK;
}

extern "C" kfbi_status kfbi_plan_stream(const kfbi_plan* pl, void** stream) {
  if (!pl || !stream) {
    kfbi_set_error("NULL argument");
    return KFBI_E_INVALID;
  }
  *stream = (void*)pl->stream;
  return KFBI_OK;
}

extern "C" kfbi_status kfbi_plan_destroy(kfbi_plan* pl) {
  if (!pl) return KFBI_OK;
  std::shared_lock<std::shared_mutex> lock(kfbi_capture_mutex);
  if (pl->stream) (void)hipStreamSynchronize(pl->stream);
  else (void)hipDeviceSynchronize();
  free_plan(pl);
  delete pl;
  return KFBI_OK;
}

namespace {
struct PdeOffsets {
  int o[KFBI_MAXP * 3];
};

__global__ void k_pde_points(int64_t n_dof, int d, int nP, double h, const int* d2s, const double* spos,
                             PdeOffsets offs, double* out) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_dof * nP) return;
  int64_t c = t / nP;
  int j = (int)(t % nP);
  const double* P = spos + (int64_t)d2s[c] * d;
  for (int a = 0; a < d; ++a) out[t * d + a] = P[a] + (double)offs.o[j * 3 + a] * h;
}

__global__ void k_corr_table(int64_t n, const int* k, const int* node, const int* own, int* out) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  out[e * 3] = k[e];
  out[e * 3 + 1] = node[e];
  out[e * 3 + 2] = own[e];
}
__global__ void k_dof_pos(int64_t n, int d, const int* d2s, const double* spos, double* out) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * d) return;
  out[e] = spos[(int64_t)d2s[e / d] * d + e % d];
}
}  // namespace

extern "C" kfbi_status kfbi_plan_export(const kfbi_plan* pl_c, int which, void* dst, int64_t bytes) {
  KCHK(need_ready(pl_c));
  kfbi_plan* pl = const_cast<kfbi_plan*>(pl_c);
  const int d = pl->g.d;
  const void* src = nullptr;
  int64_t need = 0;
  switch (which) {
    case KFBI_EXPORT_REGION: src = pl->region; need = pl->g.n_nodes; break;
    case KFBI_EXPORT_SURF_POS: src = pl->s_pos; need = pl->n_surf * d * 8; break;
    case KFBI_EXPORT_SURF_NRM: src = pl->s_nrm; need = pl->n_surf * d * 8; break;
    case KFBI_EXPORT_SURF_META: src = pl->s_meta; need = pl->n_surf * 5 * 4; break;
    case KFBI_EXPORT_DOF_SURF: src = pl->d2s; need = pl->n_dof * 4; break;
    case KFBI_EXPORT_STENCIL_D: src = pl->stD; need = pl->n_dof * pl->nD * 4; break;
    case KFBI_EXPORT_STENCIL_N: src = pl->stN; need = pl->n_dof * pl->nN * 4; break;
    case KFBI_EXPORT_EXT_IDX: src = pl->ext_idx; need = pl->n_surf * pl->g.p * 4; break;
    case KFBI_EXPORT_EXT_W: src = pl->ext_w; need = pl->n_surf * pl->g.p * 8; break;
    case KFBI_EXPORT_IRREGULAR: src = pl->irr; need = pl->n_irr * 4; break;
    case KFBI_EXPORT_COND: src = pl->cond; need = pl->n_dof * 8; break;
    case KFBI_EXPORT_PDE_PTS: need = pl->n_dof * pl->nP * d * 8; break;
    case KFBI_EXPORT_CORR: need = pl->n_corr * 3 * 4; break;
    case KFBI_EXPORT_DOF_POS: need = pl->n_dof * d * 8; break;
    default:
      kfbi_set_error("unknown export table %d", which);
      return KFBI_E_INVALID;
  }
  if (!dst || bytes < need) {
    kfbi_set_error("export table %d needs %lld bytes (got %lld)", which, (long long)need, (long long)bytes);
    return KFBI_E_INVALID;
  }
  if (need == 0) return KFBI_OK;
  if (src) {
    HIPCHK(hipMemcpyAsync(dst, src, (size_t)need, hipMemcpyDeviceToDevice, pl->stream));
    return KFBI_OK;
  }
  if (which == KFBI_EXPORT_DOF_POS) {
    hipLaunchKernelGGL(k_dof_pos, dim3((unsigned)((pl->n_dof * d + 255) / 256)), dim3(256), 0, pl->stream,
                       pl->n_dof, d, pl->d2s, pl->s_pos, (double*)dst);
    HIPCHK(hipGetLastError());
    return KFBI_OK;
  }
  if (which == KFBI_EXPORT_CORR) {
    hipLaunchKernelGGL(k_corr_table, dim3((unsigned)((pl->n_corr + 255) / 256)), dim3(256), 0, pl->stream,
                       pl->n_corr, pl->ce_k, pl->ce_node, pl->ce_owner, (int*)dst);
    HIPCHK(hipGetLastError());
    return KFBI_OK;
  }
  int offP[KFBI_MAXP][3], nP;
  kfbi_pde_lattice(d, pl->g.p, offP, &nP);
  PdeOffsets po;
  memcpy(po.o, offP, sizeof(po.o));
  int64_t n = pl->n_dof * nP;
  hipLaunchKernelGGL(k_pde_points, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, pl->stream, pl->n_dof, d, nP,
                     pl->g.h, pl->d2s, pl->s_pos, po, (double*)dst);
  HIPCHK(hipGetLastError());
  return KFBI_OK;
}

// ---------------------------------------------------------------- operators
extern "C" kfbi_status kfbi_box_solve(kfbi_plan* pl, const double* F, double* v) {
  KCHK(need_ready(pl));
  if (!F || !v || F == v) {
    kfbi_set_error("box solve needs distinct F and v");
    return KFBI_E_INVALID;
  }
  box_solve_any(pl, F, v);
  op_boundary(pl, nullptr, v);
  HIPCHK(hipGetLastError());
  return KFBI_OK;
}

extern "C" kfbi_status kfbi_plan_set_box_solver(kfbi_plan* pl, int solver, double eps_in, int max_cycles) {
  KCHK(need_ready(pl));
  if (solver != KFBI_BOX_FFT && solver != KFBI_BOX_MG64 && solver != KFBI_BOX_MG32) {
    kfbi_set_error("unknown box solver %d", solver);
    return KFBI_E_INVALID;
  }
  if (!(eps_in > 0.0) || max_cycles < 1 || max_cycles > 64) {
    kfbi_set_error("box solver needs eps_in > 0 and 1 <= max_cycles <= 64");
    return KFBI_E_INVALID;
  }
  if (pl->g.bie == KFBI_BIE_TWO_DENSITY && solver != KFBI_BOX_FFT) {
    kfbi_set_error("the two-density form uses the FFT box solver");
    return KFBI_E_INVALID;
  }
  destroy_graphs(pl);
  std::shared_lock<std::shared_mutex> lock(kfbi_capture_mutex);
  return mg_configure(pl, solver, eps_in, max_cycles);
}

extern "C" kfbi_status kfbi_plan_set_box_relaxation(kfbi_plan* pl, double relax) {
  KCHK(need_ready(pl));
  if (!(relax >= 0.0) || !isfinite(relax)) {
    kfbi_set_error("relaxation factor must be finite and >= 0 (got %g)", relax);
    return KFBI_E_INVALID;
  }
  pl->mg_relax = relax;   // read on the device at every solve: the graphs stay valid
  return KFBI_OK;
}

extern "C" kfbi_status kfbi_plan_box_stats(kfbi_plan* pl, int32_t* cycles, double* rel_res) {
  KCHK(need_ready(pl));
  int c = 0;
  double r = 0.0;
  if (pl->box_solver != KFBI_BOX_FFT) {
    int h[2];
    double sc[2];
    HIPCHK(hipStreamSynchronize(pl->stream));
    HIPCHK(hipMemcpyAsync(h, pl->mg_ctl, sizeof(h), hipMemcpyDeviceToHost, pl->stream));
    HIPCHK(hipMemcpyAsync(sc, pl->mg_scal, sizeof(sc), hipMemcpyDeviceToHost, pl->stream));
    HIPCHK(hipStreamSynchronize(pl->stream));
    c = h[1];
    r = sc[1];
  }
  if (cycles) *cycles = c;
  if (rel_res) *rel_res = r;
  return KFBI_OK;
}

extern "C" kfbi_status kfbi_simple_solve(kfbi_plan* pl, const double* a, const double* b, const double* ftilde,
                                         const double* fhat, const double* gB, double* v, double* dn_in,
                                         double* dn_out) {
  KCHK(need_ready(pl));
  simple_solve_impl(pl, a, b, ftilde, fhat, gB, v ? v : pl->vsbuf, dn_in ? dn_in : pl->dn_in,
                    dn_out ? dn_out : pl->dn_out);
  HIPCHK(hipGetLastError());
  return KFBI_OK;
}

extern "C" kfbi_status kfbi_matvec(kfbi_plan* pl, const double* psi, double* Apsi) {
  KCHK(need_ready(pl));
  if (!psi || !Apsi || psi == Apsi) {
    kfbi_set_error("matvec needs distinct psi and Apsi");
    return KFBI_E_INVALID;
  }
  if (pl->g.bie == KFBI_BIE_TWO_DENSITY) return td_matvec(pl, psi, Apsi);
  matvec_impl(pl, psi, Apsi);
  HIPCHK(hipGetLastError());
  return KFBI_OK;
}

extern "C" kfbi_status kfbi_rhs(kfbi_plan* pl, const kfbi_data* data, double* b) {
  KCHK(need_ready(pl));
  if (!data || !b) {
    kfbi_set_error("NULL argument");
    return KFBI_E_INVALID;
  }
  if (pl->g.bie == KFBI_BIE_TWO_DENSITY) return td_rhs(pl, data, b);
  rhs_impl(pl, *data, b);
  HIPCHK(hipGetLastError());
  return KFBI_OK;
}

namespace {
// Steps 3-4 after gm_residual_start: launch captured iterations in batches,
// reading the control word back between batches.  The first batch goes
// out without a host wait (after convergence or a zero right-hand side
// every kernel of a captured iteration returns at once); later batches are
// predicted from the observed convergence rate.
struct GmresOut {
  int k;
  double est;
  bool conv;
  bool spec_ok;     // the work of `spec` ran on the final iterate
};

// Work enqueued behind the first batch of iterations on the guess that the
// batch converges: `before` ahead of the state post (its values ride on the
// post: the true residual), `after` behind it (the final solve).  If the
// batch did not converge the work is simply redone later.
struct GmresSpec {
  bool active = false;
  void (*before)(void*) = nullptr;
  void (*after)(void*) = nullptr;
  void* ctx = nullptr;
};

kfbi_status gmres_run(kfbi_plan* pl, double tol, int m, int first_batch, GmresOut* o,
                      const GmresSpec& spec = GmresSpec()) {
  o->spec_ok = false;
  hipStream_t st = pl->stream;
  // Multigrid iterations cost hundreds of microseconds each, and one
  // launched after convergence still costs its launches: their batches stay
  // short (a host round trip costs some tens of microseconds).
  const bool mgs = pl->box_solver != KFBI_BOX_FFT;
  const bool relaxed = mgs && pl->relax_word > 0.0;
  int launched = 0;
  int batch = first_batch;
  double nb = 0.0, res_prev = 0.0, res_host = 0.0;
  int k_prev = 0;
  bool first = true;
  bool stop = false;
  if (relaxed) {
    // |r_0| and |b| before the first batch: the caps of the relaxed
    // iterations follow from the residual estimate
    PostReq q{};
    q.ni = 4;
    for (int i = 0; i < 4; ++i) q.isrc[i] = pl->ctl + i;
    q.nd = 7;
    for (int i = 0; i < 7; ++i) q.dsrc[i] = pl->scal + i;
    unsigned seq = 0;
    KCHK(kfbi_post_launch(pl, q, &seq));
    int iv[6] = {0, 0, 0, 0, 0, 0};
    KCHK(kfbi_post_collect(pl, q, seq, iv, pl->h_dpinned));
    for (int i = 0; i < 4; ++i) pl->h_ctl[i] = iv[i];
    nb = pl->h_dpinned[1];
    res_prev = res_host = pl->h_dpinned[6];
    first = false;
    stop = pl->h_ctl[1] != 0;
  }
  while (!stop) {
    const int B = batch < m - launched ? batch : m - launched;
    if (mgs) {
      // relaxed: each iteration with its own correction cap
      const int c = relaxed ? relaxed_cap(pl, tol, nb, res_host) : 0;
      const int run_cap = pl->mg_run_cap;
      if (c > 0) pl->mg_run_cap = c;
      for (int b = 0; b < B; ++b) enqueue_mg_iteration(pl);
      pl->mg_run_cap = run_cap;
      HIPCHK(hipGetLastError());
    } else {
      // the graph of exactly B iterations if there is one, else the
      // largest captured graphs first (graph 0 always exists)
      int left = B;
      if (pl->graph_xe && B == pl->graph_xn) {
        HIPCHK(hipGraphLaunch(pl->graph_xe, st));
        left = 0;
      }
      for (int v = KFBI_NGRAPH - 1; v >= 0; --v)
        if (pl->graph_execs[v])
          for (; left >= (1 << v); left -= 1 << v) HIPCHK(hipGraphLaunch(pl->graph_execs[v], st));
    }
    launched += B;
    const bool sp = first && spec.active;
    {
      PostReq q{};
      q.ni = 4;
      for (int i = 0; i < 4; ++i) q.isrc[i] = pl->ctl + i;
      q.nd = 7;    // scal[4], scal[5]: the true residual's sums when speculating
      for (int i = 0; i < 7; ++i) q.dsrc[i] = pl->scal + i;
      if (sp) {
        spec.before(spec.ctx);
        if (pl->box_solver != KFBI_BOX_FFT) {
          q.ni = 6;
          q.isrc[4] = pl->mg_ctl + 2;
          q.isrc[5] = pl->mg_ctl + 3;
        }
      }
      unsigned seq = 0;
      KCHK(kfbi_post_launch(pl, q, &seq));
      if (sp) spec.after(spec.ctx);
      int iv[6] = {0, 0, 0, 0, 0, 0};
      KCHK(kfbi_post_collect(pl, q, seq, iv, pl->h_dpinned));
      for (int i = 0; i < 4; ++i) pl->h_ctl[i] = iv[i];
      if (sp && q.ni == 6) {
        pl->h_pinned[2] = iv[4];
        pl->h_pinned[3] = iv[5];
      }
    }
    if (first) {
      nb = pl->h_dpinned[1];
      res_prev = pl->h_dpinned[6];
      first = false;
    }
    if (sp && pl->h_ctl[1]) o->spec_ok = true;
    if (pl->h_ctl[1] || launched >= m) break;
    const int k = pl->h_ctl[2];
    const double res = pl->h_dpinned[0];
    res_host = res;
    const int bmax = mgs ? 4 : 16;
    batch = mgs ? 2 : 4;
    if (k > k_prev && res > 0.0 && res < res_prev && res_prev > 0.0) {
      double rate = pow(res / res_prev, 1.0 / (double)(k - k_prev));
      double need = log(tol * nb / res) / log(rate);
      batch = need < 1.0 ? 1 : (need > (double)bmax ? bmax : (int)ceil(need));
    }
    res_prev = res;
    k_prev = k;
  }
  o->k = pl->h_ctl[2];
  // a zero right-hand side gives 0; a NaN norm stays NaN (reported as non-finite)
  o->est = nb == 0.0 ? 0.0 : pl->h_dpinned[0] / nb;
  o->conv = pl->h_ctl[1] && (nb == 0.0 || pl->h_dpinned[0] <= tol * nb || pl->h_dpinned[2] != 0.0);
  return KFBI_OK;
}

// sqrt(|r|^2 / |b|^2): 0 for a zero right-hand side, NaN when either sum is
// not finite (so the solve reports KFBI_E_NONFINITE)
double rel_residual(double rr, double bb) {
  if (bb == 0.0) return 0.0;
  return sqrt(rr / bb);
}

// |b - A psi| / |b| with a fresh full-accuracy matvec
// with `then`, work enqueued after the residual's kernels and before the
// host waits for them
template <class Then>
kfbi_status true_residual(kfbi_plan* pl, const double* psi, double* tr, Then then) {
  matvec_impl(pl, psi, pl->work2);
  gm_true_residual(pl, pl->bvec, pl->work2, pl->scal + 4);
  PostReq q{};
  q.nd = 2;
  q.dsrc[0] = pl->scal + 4;
  q.dsrc[1] = pl->scal + 5;
  if (pl->box_solver != KFBI_BOX_FFT) {
    q.ni = 2;
    q.isrc[0] = pl->mg_ctl + 2;
    q.isrc[1] = pl->mg_ctl + 3;
  }
  unsigned seq = 0;
  KCHK(kfbi_post_launch(pl, q, &seq));
  then();
  KCHK(kfbi_post_collect(pl, q, seq, pl->h_pinned + 2, pl->h_dpinned + 4));
  *tr = rel_residual(pl->h_dpinned[4], pl->h_dpinned[5]);
  return KFBI_OK;
}

kfbi_status true_residual(kfbi_plan* pl, const double* psi, double* tr) {
  return true_residual(pl, psi, tr, [] {});
}

// the relaxation factor the captured iterations read (GMRES scal[7])
kfbi_status set_relax_word(kfbi_plan* pl, double r) {
  if (r == pl->relax_word) return KFBI_OK;    // unchanged on the device
  pl->relax_word = r;
  pl->h_dpinned[7] = r;
  HIPCHK(hipMemcpyAsync(pl->scal + 7, pl->h_dpinned + 7, sizeof(double), hipMemcpyHostToDevice, pl->stream));
  return KFBI_OK;
}

kfbi_status solve_steps(kfbi_plan* pl, const kfbi_data* data, const kfbi_opts* opts, double* psi, double* u_out,
                        kfbi_info* info, int m, double tol);

kfbi_status solve_steps_mg_eps(kfbi_plan* pl, const kfbi_data* data, const kfbi_opts* opts, double* psi,
                               double* u_out, kfbi_info* info, int m, double tol);

kfbi_status solve_body(kfbi_plan* pl, const kfbi_data* data, const kfbi_opts* opts, double* psi, double* u_out,
                       kfbi_info* info, int m, double tol) {
  // Multigrid box solves inside a solve run at most mg_cap_eff corrections:
  // the captured iterations enqueue every correction up to the cap and the
  // ones after convergence return at once, each still costing its launches.
  // The cap is the most corrections any box solve of the previous solve
  // needed plus 1 (the count hardly varies with the right-hand side); a
  // box solve to eps_in stopped by it above its tolerance raises it by 2
  // for the next solves.  Relaxed GMRES iterations run with caps of their
  // own, from the residual estimate (relaxed_cap).
  const bool mg = pl->box_solver != KFBI_BOX_FFT;
  if (mg) {
    KCHK(mg_store_reserve(pl));
    pl->mg_run_cap = pl->mg_cap_eff > 0 ? pl->mg_cap_eff : pl->mg_maxit;
    HIPCHK(hipMemsetAsync(pl->mg_ctl + 2, 0, 2 * sizeof(int), pl->stream));
  }
  kfbi_status s = solve_steps_mg_eps(pl, data, opts, psi, u_out, info, m, tol);
  if (mg) {
    if (s == KFBI_OK || s == KFBI_E_NOT_CONVERGED) {
      const int most = pl->h_pinned[2], hit = pl->h_pinned[3];
      const int run = pl->mg_run_cap > 0 ? pl->mg_run_cap : pl->mg_maxit;
      if (hit > 0)
        pl->mg_cap_eff = run + 2 < pl->mg_maxit ? run + 2 : pl->mg_maxit;
      else if (most > 0)
        pl->mg_cap_eff = most + 1 < pl->mg_maxit ? most + 1 : pl->mg_maxit;
    }
    pl->mg_run_cap = 0;
  }
  return s;
}

// status and info of a finished solve (k iterations, true residual tr)
kfbi_status solve_report(kfbi_plan* pl, kfbi_info* info, const GmresOut& o, int k, double tr, double tol, int m) {
  pl->last_iters = k;
  HIPCHK(hipGetLastError());
  kfbi_status s = o.conv ? KFBI_OK : KFBI_E_NOT_CONVERGED;
  if (!isfinite(tr) || !isfinite(o.est)) s = KFBI_E_NONFINITE;
  if (info) {
    info->iters = k;
    info->status = s;
    info->est_rel_res = o.est;
    info->true_rel_res = tr;
  }
  if (s == KFBI_E_NOT_CONVERGED) kfbi_set_error("GMRES did not reach tol %g in %d iterations", tol, m);
  if (s == KFBI_E_NONFINITE) kfbi_set_error("non-finite residual");
  return s;
}

// |b - A psi| / |b| with the multigrid box solvers.  psi = x0 + sum y_j v_j,
// so the box solution of A psi is U(x0) + sum y_j U(v_j) up to the box
// solves' tolerances: its box solve starts from that combination of the
// stored solutions and stops after at most 3 corrections; short of eps_in
// there, it continues from where it stopped with the full cap.  `then` is
// enqueued behind the residual's kernels, before the host waits (again
// after a continuation).  The box solution of A psi is left in vbuf.
template <class Then>
kfbi_status mg_true_residual(kfbi_plan* pl, const double* psi, int k, int use_x0, double* tr, Then then) {
  const bool guess = pl->ustore && k + 1 <= pl->ustore_slots;
  if (guess) mg_guess_from_store(pl, k, use_x0, pl->scal + 8, pl->vbuf);
  for (int pass = 0; pass < 2; ++pass) {
    const int run_cap = pl->mg_run_cap;
    if (pass == 0 && guess && (run_cap == 0 || run_cap > 3)) pl->mg_run_cap = 3;
    pl->mg_guess = guess;
    matvec_impl(pl, psi, pl->work2);
    pl->mg_guess = false;
    pl->mg_run_cap = run_cap;
    gm_true_residual(pl, pl->bvec, pl->work2, pl->scal + 4);
    PostReq q{};
    q.nd = 3;
    q.dsrc[0] = pl->scal + 4;
    q.dsrc[1] = pl->scal + 5;
    q.dsrc[2] = pl->mg_scal + 1;      // relative residual the box solve stopped at
    q.ni = 2;
    q.isrc[0] = pl->mg_ctl + 2;
    q.isrc[1] = pl->mg_ctl + 3;
    unsigned seq = 0;
    KCHK(kfbi_post_launch(pl, q, &seq));
    then();
    KCHK(kfbi_post_collect(pl, q, seq, pl->h_pinned + 2, pl->h_dpinned + 4));
    *tr = rel_residual(pl->h_dpinned[4], pl->h_dpinned[5]);
    if (!guess || pl->h_dpinned[6] <= pl->mg_eps) break;
  }
  return KFBI_OK;
}

// A multigrid solve of an interface problem from a given start takes its
// initial residual from one box solve instead of two: by linearity in the
// data and the density, r0 = b - A x0 = (g2 - J(w(g1, E x0, ftilde, fhat,
// gB))) / (beta_in + beta_out) (Alg. 1 steps 1-2 with the same w as step 4).
// b itself then sets only the scale |b| of the stopping test, which a box
// solve stopped after 3 corrections gives to about 1e-3.  The grid solution
// w(E x0, data) is slot 0 of the store, so the true residual's box solve
// starts from w(E psi, data) and leaves the final solution.  Off with
// KFBI_MERGED_START=0 in the environment.
bool merged_start(const kfbi_plan* pl, int use_x0) {
  if (!use_x0 || pl->box_solver == KFBI_BOX_FFT || pl->g.bie != KFBI_BIE_INTERFACE || !pl->ustore ||
      pl->ustore_slots < 2)
    return false;
  const char* e = getenv("KFBI_MERGED_START");
  return !(e && e[0] == '0');
}

// |b - A psi| / |b| of a merged start (psi = x0 + sum y_j v_j): the box
// solve of (data, E psi) starts from slot 0 + sum y_j slot(1 + j) and stops
// after at most 3 corrections, continuing with the full cap if short of
// eps; r = (g2 - J(w)) / (beta_in + beta_out) directly, passed to the
// residual kernel as b~ - (b~ - r).  w is left in u; b~ - r in work.
kfbi_status merged_true_residual(kfbi_plan* pl, const kfbi_data& data, const double* psi, int k, double* u,
                                 double* tr) {
  const bool guess = k + 1 <= pl->ustore_slots;
  if (guess) mg_guess_from_store(pl, k, 1, pl->scal + 8, u);
  for (int pass = 0; pass < 2; ++pass) {
    const int run_cap = pl->mg_run_cap;
    if (pass == 0 && guess && (run_cap == 0 || run_cap > 3)) pl->mg_run_cap = 3;
    pl->mg_guess = guess;
    final_impl(pl, data, psi, u);
    pl->mg_guess = false;
    pl->mg_run_cap = run_cap;
    op_bie_rhs(pl, data.g2, pl->dn_in, pl->dn_out, pl->work2);
    vec_diff(pl, pl->n_dof, pl->bvec, pl->work2, pl->work);
    gm_true_residual(pl, pl->bvec, pl->work, pl->scal + 4);
    PostReq q{};
    q.nd = 3;
    q.dsrc[0] = pl->scal + 4;
    q.dsrc[1] = pl->scal + 5;
    q.dsrc[2] = pl->mg_scal + 1;
    q.ni = 2;
    q.isrc[0] = pl->mg_ctl + 2;
    q.isrc[1] = pl->mg_ctl + 3;
    unsigned seq = 0;
    KCHK(kfbi_post_launch(pl, q, &seq));
    KCHK(kfbi_post_collect(pl, q, seq, pl->h_pinned + 2, pl->h_dpinned + 4));
    *tr = rel_residual(pl->h_dpinned[4], pl->h_dpinned[5]);
    if (!guess || pl->h_dpinned[6] <= pl->mg_eps) break;
  }
  return KFBI_OK;
}

kfbi_status solve_steps(kfbi_plan* pl, const kfbi_data* data, const kfbi_opts* opts, double* psi, double* u_out,
                        kfbi_info* info, int m, double tol);

// With a relaxed multigrid the box solves outside the GMRES iterations --
// the right-hand side, A x0, the true residual and the final solution --
// run to eps_out = min(eps_in, tol / 100): their errors enter b and the
// measured residual directly (with eps_in = tol / 10 the residual against
// a right-hand side and matvec to 1e-13 came out at 1.2-1.4 tol on the
// 1000:1 star), while the iterations' errors only perturb the Krylov
// space (relaxation).  The plan's eps_in is restored on return.
kfbi_status solve_steps_mg_eps(kfbi_plan* pl, const kfbi_data* data, const kfbi_opts* opts, double* psi,
                               double* u_out, kfbi_info* info, int m, double tol) {
  const double eps_in = pl->mg_eps;
  if (pl->box_solver != KFBI_BOX_FFT && pl->mg_relax > 0.0 && eps_in > 1e-2 * tol) pl->mg_eps_out = 1e-2 * tol;
  else pl->mg_eps_out = eps_in;
  const kfbi_status s = solve_steps(pl, data, opts, psi, u_out, info, m, tol);
  pl->mg_eps = eps_in;
  return s;
}

kfbi_status solve_steps(kfbi_plan* pl, const kfbi_data* data, const kfbi_opts* opts, double* psi, double* u_out,
                        kfbi_info* info, int m, double tol) {
  const bool mg = pl->box_solver != KFBI_BOX_FFT;
  const bool relax = pl->mg_relax > 0.0 && mg;
  const double eps_in = pl->mg_eps, eps_out = mg ? pl->mg_eps_out : eps_in;
  const int use_x0 = opts->start == KFBI_START_GIVEN ? 1 : 0;
  const bool merged = merged_start(pl, use_x0);
  // Step 1: right-hand side (its grid solution stays in vsbuf); of a merged
  // start only its scale, from zero (as a guess: a stop at the cap is no
  // sign of a short cap) in 3 corrections
  pl->mg_eps = eps_out;
  if (merged) {
    grid_zero(pl, pl->vsbuf);
    const int run_cap = pl->mg_run_cap;
    pl->mg_run_cap = 3;
    pl->mg_guess = true;
    rhs_impl(pl, *data, pl->bvec);
    pl->mg_guess = false;
    pl->mg_run_cap = run_cap;
  } else {
    rhs_impl(pl, *data, pl->bvec);
  }
  KCHK(set_relax_word(pl, relax ? pl->mg_relax : 0.0));
  // Step 2: initial residual and control word (multigrid: the box solution
  // of A x0, or of a merged start w(E x0, data), goes to the store's slot 0)
  if (merged) {
    final_impl(pl, *data, psi, pl->vsbuf);
    op_bie_rhs(pl, data->g2, pl->dn_in, pl->dn_out, pl->work2);     // r0
    vec_diff(pl, pl->n_dof, pl->bvec, pl->work2, pl->work);          // b~ - r0 in place of A x0
    mg_store_solution(pl, pl->vsbuf);
  } else if (use_x0) {
    matvec_impl(pl, psi, pl->work);
    if (mg) mg_store_solution(pl, pl->vbuf);
  }
  gm_residual_start(pl, pl->bvec, pl->work, use_x0, tol, m);
  pl->mg_eps = eps_in;
  KCHK(ensure_graph(pl));
  // final solve u = w(g1, E psi, ftilde, fhat, gB)
  double* u = u_out ? u_out : pl->vsbuf;
  auto final_solve = [&] { final_impl(pl, *data, psi, u); };
  // Steps 3-4.  FFT box solver: without relaxation and from a zero start,
  // on a graph key already solved with (a repeated problem, so the first
  // batch, sized to the previous iteration count, usually converges), the
  // update, the true residual and the final solve go out right behind the
  // first batch: a solve that converges within it waits on the host once;
  // otherwise they are redone after convergence.
  struct SpecCtx {
    kfbi_plan* pl;
    double* psi;
    decltype(final_solve)* fin;
  } sc{pl, psi, &final_solve};
  GmresSpec spec;
  spec.active = !mg && !use_x0 && pl->graph_uses > 1;
  spec.ctx = &sc;
  spec.before = [](void* c) {
    SpecCtx* x = (SpecCtx*)c;
    gm_update_device(x->pl, x->psi, 0);
    matvec_impl(x->pl, x->psi, x->pl->work2);
    gm_true_residual(x->pl, x->pl->bvec, x->pl->work2, x->pl->scal + 4);
  };
  spec.after = [](void* c) { (*((SpecCtx*)c)->fin)(); };
  GmresOut o;
  // the first batch: the previous solve's iteration count on this plan (at
  // least 4: an over-long batch costs a few microseconds, a short one a host
  // round trip), at most 4 with the multigrid box solvers
  int fb = pl->last_iters > 4 ? (pl->last_iters < 64 ? pl->last_iters : 64) : 4;
  if (mg && fb > 4) fb = 4;
  // a key solved with more than once (a repeated problem): its first batch,
  // when no power of two, as one graph instead of several (each graph
  // launch idles the GPU for a few microseconds)
  if (!mg && pl->graph_uses > 1 && (fb & (fb - 1)) != 0 && pl->graph_xn != fb) {
    // like every capture, exclusive of other threads' set-up and allocations
    std::unique_lock<std::shared_mutex> lock(kfbi_capture_mutex);
    if (pl->graph_xe) HIPCHK(hipStreamSynchronize(pl->stream));   // no launch of the old one in flight
    if (pl->graph_xe) (void)hipGraphExecDestroy(pl->graph_xe);
    if (pl->graph_x) (void)hipGraphDestroy(pl->graph_x);
    pl->graph_xe = nullptr;
    pl->graph_x = nullptr;
    pl->graph_xn = 0;
    KCHK(capture_iterations(pl, fb, &pl->graph_x, &pl->graph_xe));
    pl->graph_xn = fb;
  }
  KCHK(gmres_run(pl, tol, m, fb, &o, spec));
  if (o.spec_ok) {
    const double tr = rel_residual(pl->h_dpinned[4], pl->h_dpinned[5]);
    return solve_report(pl, info, o, o.k, tr, tol, m);
  }
  gm_update(pl, o.k, psi, use_x0);
  double tr = 0.0;
  if (!mg) {
    // psi is final here: the final solve is enqueued before the host waits
    // for the true residual
    KCHK(true_residual(pl, psi, &tr, final_solve));
    return solve_report(pl, info, o, o.k, tr, tol, m);
  }
  int k = o.k;
  if (merged) {
    pl->mg_eps = eps_out;
    KCHK(merged_true_residual(pl, *data, psi, o.k, u, &tr));
    // as below: continue from psi with full-accuracy box solves if the
    // relaxed estimate ran ahead of the true residual (its box solution
    // becomes slot 0, b~ - r(psi) is in work)
    if (relax && o.conv && tr > tol && k < m) {
      KCHK(set_relax_word(pl, 0.0));
      mg_store_solution(pl, u);
      gm_residual_start(pl, pl->bvec, pl->work, 1, tol, m - k);
      GmresOut o2;
      pl->mg_eps = eps_in;
      KCHK(gmres_run(pl, tol, m - k, 4, &o2));
      gm_update(pl, o2.k, psi, 1);
      pl->mg_eps = eps_out;
      KCHK(merged_true_residual(pl, *data, psi, o2.k, u, &tr));
      k += o2.k;
      o.est = o2.est;
      o.conv = o2.conv;
    }
    pl->mg_eps = eps_in;
    return solve_report(pl, info, o, k, tr, tol, m);
  }
  // Multigrid: the final solve's grid solution is, by linearity in the
  // data and the density, the step-1 solution (vsbuf) plus the box
  // solution of A psi (vbuf, left by the true residual); enqueued behind
  // the residual on the guess that no continuation follows.
  auto final_sum = [&] { mg_sum(pl, pl->vsbuf, pl->vbuf, u); };
  pl->mg_eps = eps_out;
  KCHK(mg_true_residual(pl, psi, o.k, use_x0, &tr, [] {}));
  // with a relaxed inner tolerance the GMRES estimate can run ahead of the
  // true residual: if it misses tol, continue from psi with full-accuracy
  // box solves until it meets it (A psi and its box solution are at hand)
  if (relax && o.conv && tr > tol && k < m) {
    KCHK(set_relax_word(pl, 0.0));
    mg_store_solution(pl, pl->vbuf);
    gm_residual_start(pl, pl->bvec, pl->work2, 1, tol, m - k);
    GmresOut o2;
    pl->mg_eps = eps_in;
    KCHK(gmres_run(pl, tol, m - k, 4, &o2));
    gm_update(pl, o2.k, psi, 1);
    pl->mg_eps = eps_out;
    KCHK(mg_true_residual(pl, psi, o2.k, 1, &tr, [] {}));
    k += o2.k;
    o.est = o2.est;
    o.conv = o2.conv;
  }
  final_sum();
  pl->mg_eps = eps_in;
  return solve_report(pl, info, o, k, tr, tol, m);
}
}  // namespace

// ---------------------------------------------------------------- solves of a group in lockstep
kfbi_status apply_solver(kfbi_plan* pl, const kfbi_opts& o);

namespace {
__global__ void k_group_open(int* const* ctls, int G, int* open) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  for (int p = threadIdx.x; p < G; p += blockDim.x)
    if (!ctls[p][1]) atomicAdd(&cnt, 1);
  __syncthreads();
  if (threadIdx.x == 0) *open = cnt;
}

// per problem: done, k, |r_k| estimate, |b|, breakdown flag, true residual sums
__global__ void k_group_state(int* const* ctls, double* const* scals, int G, double* out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= G) return;
  const int* c = ctls[p];
  const double* s = scals[p];
  double* o = out + 8 * (int64_t)p;
  o[0] = c[1];
  o[1] = c[2];
  o[2] = s[0];
  o[3] = s[1];
  o[4] = s[2];
  o[5] = s[4];
  o[6] = s[5];
  o[7] = 0.0;
}
}  // namespace

// Alg. 1 for G problems of one dimension (any grid sizes) with the FFT box
// solver, their GMRES iterations in lockstep: per iteration the
// interface-dependent kernels of every problem and one launch per box-solve
// pass for all the problems up to N = 256 (plus one per pass per larger
// size), captured once as a graph of four iterations; every kernel of a
// problem that has converged returns at once.  The right-hand sides, the
// updates, true residuals and final solves are those of kfbi_solve, so
// every problem's density and solution equal its own solve's bit for bit.
// All on `st`; the plans' own streams are restored at the end.
kfbi_status kfbi_solve_group(kfbi_plan* const* pls, int G, const kfbi_data* data, double* const* psi,
                             double* const* u, const kfbi_opts* opts, hipStream_t st, kfbi_info* infos) {
  const int m = opts->max_iter;
  const double tol = opts->tol > 0.0 ? opts->tol : 1e-10;
  const int use_x0 = opts->start == KFBI_START_GIVEN ? 1 : 0;
  if (G < 1 || m < 1 || m > KFBI_GMRES_MAX || opts->start == KFBI_START_LEARNED) {
    kfbi_set_error("group solve: G >= 1, 1 <= max_iter <= %d, no learned start", KFBI_GMRES_MAX);
    return KFBI_E_INVALID;
  }
  for (int p = 0; p < G; ++p) {
    KCHK(need_ready(pls[p]));
    if (opts->solver != KFBI_SOLVER_PLAN) KCHK(apply_solver(pls[p], *opts));
    if (pls[p]->box_solver != KFBI_BOX_FFT || pls[p]->g.d != pls[0]->g.d ||
        pls[p]->g.bie == KFBI_BIE_TWO_DENSITY) {
      kfbi_set_error("group solve: FFT box solver, one dimension, single-density plans");
      return KFBI_E_INVALID;
    }
    HIPCHK(hipStreamSynchronize(pls[p]->stream));
    {
      std::shared_lock<std::shared_mutex> lock(kfbi_capture_mutex);
      KCHK(ensure_gmres(pls[p], m));
    }
  }
  std::vector<hipStream_t> own(G);
  for (int p = 0; p < G; ++p) {
    own[p] = pls[p]->stream;
    pls[p]->stream = st;
  }
  kfbi_status status = KFBI_OK;
  DstBatch* db = nullptr;
  int** d_ctl = nullptr;
  double** d_scal = nullptr;
  int* d_open = nullptr;
  double* d_state = nullptr;
  int* h_open = nullptr;
  hipGraph_t gr = nullptr;
  hipGraphExec_t ex = nullptr;
  std::vector<double> state((size_t)8 * G);
  auto run = [&]() -> kfbi_status {
    // steps 1-2 of every problem
    for (int p = 0; p < G; ++p) {
      kfbi_plan* pl = pls[p];
      rhs_impl(pl, data[p], pl->bvec);
      KCHK(set_relax_word(pl, 0.0));
      if (use_x0) matvec_impl(pl, psi[p], pl->work);
      gm_residual_start(pl, pl->bvec, pl->work, use_x0, tol, m);
    }
    HIPCHK(hipGetLastError());
    kfbi_status s = KFBI_OK;
    db = dst_batch_create(pls, G, st, &s);
    KCHK(s);
    std::vector<int*> hc(G);
    std::vector<double*> hs(G);
    for (int p = 0; p < G; ++p) {
      hc[p] = pls[p]->ctl;
      hs[p] = pls[p]->scal;
    }
    if (hipMalloc((void**)&d_ctl, sizeof(int*) * G) != hipSuccess ||
        hipMalloc((void**)&d_scal, sizeof(double*) * G) != hipSuccess ||
        hipMalloc((void**)&d_open, sizeof(int)) != hipSuccess ||
        hipMalloc((void**)&d_state, sizeof(double) * 8 * G) != hipSuccess ||
        hipHostMalloc((void**)&h_open, sizeof(int), 0) != hipSuccess) {
      (void)hipGetLastError();
      kfbi_set_error("group solve: device allocation failed");
      return KFBI_E_OOM;
    }
    HIPCHK(hipMemcpyAsync(d_ctl, hc.data(), sizeof(int*) * G, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(d_scal, hs.data(), sizeof(double*) * G, hipMemcpyHostToDevice, st));
    // steps 3-4: four lockstep iterations and the count of open problems,
    // captured once
    {
      std::unique_lock<std::shared_mutex> lock(kfbi_capture_mutex);
      HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      for (int it = 0; it < 4; ++it) {
        for (int p = 0; p < G; ++p) {
          pls[p]->ctl_active = pls[p]->ctl;
          op_matvec_head(pls[p], nullptr);
          pls[p]->ctl_active = nullptr;
        }
        dst_batch_corrections(db, st);
        for (int p = 0; p < G; ++p) {
          pls[p]->ctl_active = pls[p]->ctl;
          op_matvec_tail(pls[p], nullptr, nullptr);
          gm_arnoldi(pls[p]);
          pls[p]->ctl_active = nullptr;
        }
      }
      hipLaunchKernelGGL(k_group_open, dim3(1), dim3(256), 0, st, d_ctl, G, d_open);
      const hipError_t e = hipStreamEndCapture(st, &gr);
      if (e != hipSuccess) return kfbi_hip_status(e, "hipStreamEndCapture");
      const hipError_t e2 = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
      if (e2 != hipSuccess) return kfbi_hip_status(e2, "hipGraphInstantiate");
    }
    for (int launched = 0; launched < m; launched += 4) {
      HIPCHK(hipGraphLaunch(ex, st));
      HIPCHK(hipMemcpyAsync(h_open, d_open, sizeof(int), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      if (*h_open == 0) break;
    }
    // update, true residual and final solve of every problem
    for (int p = 0; p < G; ++p) {
      kfbi_plan* pl = pls[p];
      gm_update_device(pl, psi[p], use_x0);
      matvec_impl(pl, psi[p], pl->work2);
      gm_true_residual(pl, pl->bvec, pl->work2, pl->scal + 4);
      final_impl(pl, data[p], psi[p], u[p]);
    }
    hipLaunchKernelGGL(k_group_state, dim3((G + 255) / 256), dim3(256), 0, st, d_ctl, d_scal, G, d_state);
    HIPCHK(hipMemcpyAsync(state.data(), d_state, sizeof(double) * 8 * G, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int p = 0; p < G; ++p) {
      const double* o = &state[(size_t)8 * p];
      GmresOut go;
      go.k = (int)o[1];
      const double nb = o[3];
      go.est = nb == 0.0 ? 0.0 : o[2] / nb;
      go.conv = o[0] != 0.0 && (nb == 0.0 || o[2] <= tol * nb || o[4] != 0.0);
      go.spec_ok = false;
      const double tr = rel_residual(o[5], o[6]);
      kfbi_info info{0, KFBI_OK, 0.0, 0.0};
      infos[p].status = solve_report(pls[p], &info, go, go.k, tr, tol, m);
      infos[p].iters = info.iters;
      infos[p].est_rel_res = info.est_rel_res;
      infos[p].true_rel_res = info.true_rel_res;
    }
    return KFBI_OK;
  };
  status = run();
  for (int p = 0; p < G; ++p) {
    pls[p]->ctl_active = nullptr;
    pls[p]->stream = own[p];
  }
  if (ex) (void)hipGraphExecDestroy(ex);
  if (gr) (void)hipGraphDestroy(gr);
  dst_batch_destroy(db);
  if (d_ctl) (void)hipFree(d_ctl);
  if (d_scal) (void)hipFree(d_scal);
  if (d_open) (void)hipFree(d_open);
  if (d_state) (void)hipFree(d_state);
  if (h_open) (void)hipHostFree(h_open);
  return status;
}

// the box solver the options ask for, set on the plan when it differs
kfbi_status apply_solver(kfbi_plan* pl, const kfbi_opts& o) {
  const int solver = o.solver - 1;
  const double eps = o.eps_in > 0.0 ? o.eps_in : 1e-12;
  const int cycles = o.max_cycles > 0 ? o.max_cycles : 40;
  if (solver != pl->box_solver || (solver != KFBI_BOX_FFT && (eps != pl->mg_eps || cycles != pl->mg_maxit)))
    KCHK(kfbi_plan_set_box_solver(pl, solver, eps, cycles));
  if (o.relax != pl->mg_relax) KCHK(kfbi_plan_set_box_relaxation(pl, o.relax));
  return KFBI_OK;
}

extern "C" kfbi_status kfbi_solve(kfbi_plan* pl, const kfbi_data* data, const kfbi_opts* opts_in, double* psi,
                                  double* u_out, kfbi_info* info) {
  KCHK(need_ready(pl));
  if (!data || !opts_in || !psi || !data->g2) {
    kfbi_set_error("NULL argument");
    return KFBI_E_INVALID;
  }
  kfbi_opts o = *opts_in;
  const kfbi_opts* opts = &o;
  if (o.start < KFBI_START_ZERO || o.start > KFBI_START_LEARNED || o.solver < KFBI_SOLVER_PLAN ||
      o.solver > KFBI_SOLVER_MG32 || (o.start == KFBI_START_LEARNED && !o.learned)) {
    kfbi_set_error("opts: start must be KFBI_START_* (learned needs opts->learned), solver KFBI_SOLVER_*");
    return KFBI_E_INVALID;
  }
  if (o.start == KFBI_START_LEARNED && pl->g.bie != KFBI_BIE_INTERFACE) {
    kfbi_set_error("a learned start is for interface problems");
    return KFBI_E_INVALID;
  }
  if (pl->g.bie == KFBI_BIE_TWO_DENSITY) {
    if (o.solver != KFBI_SOLVER_PLAN && o.solver != KFBI_SOLVER_FFT) {
      kfbi_set_error("the two-density form uses the FFT box solver");
      return KFBI_E_INVALID;
    }
    std::shared_lock<std::shared_mutex> lock(kfbi_capture_mutex);
    return td_solve(pl, data, &o, psi, u_out, info);
  }
  if (o.solver != KFBI_SOLVER_PLAN) KCHK(apply_solver(pl, o));
  if (o.start == KFBI_START_LEARNED) {
    // the predicted density, on the plan's stream ahead of the solve
    const kfbi_learned* L = o.learned;
    KCHK(kfbi_learned_start(pl, L->mlp, L->nb, L->geom, L->jumps, L->scale, psi));
    o.start = KFBI_START_GIVEN;
  }
  int m = opts->max_iter;
  if (m < 1 || m > KFBI_GMRES_MAX) {
    kfbi_set_error("max_iter must be in [1, %d]", KFBI_GMRES_MAX);
    return KFBI_E_INVALID;
  }
  double tol = opts->tol > 0.0 ? opts->tol : 1e-10;
  {
    std::shared_lock<std::shared_mutex> lock(kfbi_capture_mutex);
    KCHK(ensure_gmres(pl, m));
  }
  // graph capture needs a stream other than the default ones: a caller's
  // own stream is used as it is; for a default stream the solve runs on the
  // plan's private stream, ordered after and before the caller's by events
  hipStream_t user = pl->stream;
  if (user != nullptr && user != hipStreamLegacy && user != hipStreamPerThread)
    return solve_body(pl, data, opts, psi, u_out, info, m, tol);
  if (!pl->gstream) {
    HIPCHK(hipStreamCreateWithFlags(&pl->gstream, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&pl->ev_in, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&pl->ev_out, hipEventDisableTiming));
  }
  HIPCHK(hipEventRecord(pl->ev_in, user));
  HIPCHK(hipStreamWaitEvent(pl->gstream, pl->ev_in, 0));
  pl->stream = pl->gstream;
  kfbi_status s = solve_body(pl, data, opts, psi, u_out, info, m, tol);
  pl->stream = user;
  hipError_t e1 = hipEventRecord(pl->ev_out, pl->gstream);
  hipError_t e2 = hipStreamWaitEvent(user, pl->ev_out, 0);
  if (s == KFBI_OK && e1 != hipSuccess) return kfbi_hip_status(e1, "hipEventRecord");
  if (s == KFBI_OK && e2 != hipSuccess) return kfbi_hip_status(e2, "hipStreamWaitEvent");
  return s;
}

// ---------------------------------------------------------------- tracing
extern "C" kfbi_status kfbi_plan_profile(kfbi_plan* pl, int enable) {
  if (!pl) {
    kfbi_set_error("plan is NULL");
    return KFBI_E_INVALID;
  }
  if (pl->prof_ev) {
    HIPCHK(pl->stream ? hipStreamSynchronize(pl->stream) : hipDeviceSynchronize());
    for (hipEvent_t e : *pl->prof_ev) (void)hipEventDestroy(e);
    pl->prof_ev->clear();
  } else {
    pl->prof_ev = new (std::nothrow) std::vector<hipEvent_t>();
    if (!pl->prof_ev) {
      kfbi_set_error("host allocation failed");
      return KFBI_E_OOM;
    }
  }
  pl->prof_launches = 0;
  pl->prof_on = enable == 2 || enable == 3 ? enable : (enable ? 1 : 0);
  return KFBI_OK;
}

extern "C" kfbi_status kfbi_plan_timing(kfbi_plan* pl, int64_t* solves, int64_t* launches, double* ms) {
  if (!pl || !solves || !launches || !ms) {
    kfbi_set_error("NULL argument");
    return KFBI_E_INVALID;
  }
  *solves = 0;
  *launches = 0;
  *ms = 0.0;
  if (!pl->prof_ev) return KFBI_OK;
  HIPCHK(pl->stream ? hipStreamSynchronize(pl->stream) : hipDeviceSynchronize());
  double tot = 0.0;
  for (size_t i = 0; i + 1 < pl->prof_ev->size(); i += 2) {
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, (*pl->prof_ev)[i], (*pl->prof_ev)[i + 1]));
    tot += t;
  }
  *solves = (int64_t)(pl->prof_ev->size() / 2);
  *launches = pl->prof_launches;
  *ms = tot;
  return KFBI_OK;
}
