/* Manufactured-solution test data for the KFBI library (an input
 * generator for tests and benchmarks, built as libkfbi_gen.so; the solver
 * library does not use it).  Everything goes through the public C ABI of
 * kfbi.h: the plan's query points are exported, then the exact solutions
 * are evaluated there on the device.
 *
 *   KFBI_GEN_STAR2D   u_in = cos 2x e^y, u_out = x^2 - y^3 (2D)
 *   KFBI_GEN_TORUS3D  u_in = sin x sin y sin z, u_out = e^(x+y+z)/10 (3D)
 *
 * with fhat_s = Lap u_s - kappa u_s, g1 = [u], g2 = [beta d_n u] (beta_in
 * inside every interface), gB = u_out. */
#ifndef KFBI_GEN_H
#define KFBI_GEN_H

#include "../../include/kfbi.h"

#ifdef __cplusplus
extern "C" {
#endif

enum { KFBI_GEN_STAR2D = 1, KFBI_GEN_TORUS3D = 2 };

/* Data of the manufactured solution `kind` at a ready plan's query points,
 * ordered on `stream`, which must be the plan's stream, into caller device arrays
 * g1, g2 [n_surf], ftilde [n_dof][n_pde], fhat [n_iface+1][n_nodes],
 * gB [n_nodes]; prob is the problem the plan is set up for.  Uses a
 * workspace of the calling thread (grown on demand, kept until
 * kfbi_gen_release). */
kfbi_status kfbi_gen_plan_data(kfbi_plan* plan, const kfbi_problem* prob, int kind, void* stream, double* g1,
                               double* g2, double* ftilde, double* fhat, double* gB);

/* A kfbi_batch_data_fn source for a batch of n problems (copied) with
 * their kinds: kfbi_gen_batch_data with ctx = the kfbi_gen.  The data of a
 * problem live in the calling worker thread's workspace until its next
 * call.  With psi_all (device, may be NULL) the density of problem i goes
 * to psi_all + i * psi_stride (KFBI_E_INVALID if n_dof > psi_stride). */
typedef struct kfbi_gen kfbi_gen;
kfbi_status kfbi_gen_create(const kfbi_problem* probs, const int* kinds, int n, double* psi_all, int64_t psi_stride,
                            kfbi_gen** out);
kfbi_status kfbi_gen_batch_data(void* ctx, int problem, kfbi_plan* plan, void* stream, kfbi_data* data,
                                double** psi_out);
kfbi_status kfbi_gen_destroy(kfbi_gen* gen);
/* Free every thread's workspace (no generator call may be running). */
void kfbi_gen_release(void);

#ifdef __cplusplus
}
#endif

#endif
