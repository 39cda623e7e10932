// LCP layer: contacts, A = D^T M D products, BB-PGD / Mono-PQN / Bi-PQN, step.
#pragma once
#include "context.hpp"

namespace bipqn {

constexpr int kRmax = 32;   // quasi-Newton memory (pairs) held on the device

int lcp_find_contacts(pqn_ctx_impl& ctx, double delta);
void lcp_copy_contacts(pqn_ctx_impl& ctx, int n, int32_t* pairs, double* gaps);
void lcp_check_pairs(pqn_ctx_impl& ctx, int n, const int32_t* pairs);
void contact_scratch_setup(int device);
pqn_status lcp_find_contacts_noalloc(pqn_ctx_impl& ctx, double delta, int cap, int* n_out, int* pairs,
                                     double* gaps);
pqn_status lcp_apply_host(pqn_ctx_impl& ctx, int n, const int32_t* pairs, const double* x, double* Ax, int fidelity);
pqn_status lcp_solve_host(pqn_ctx_impl& ctx, int n, const int32_t* pairs, const double* b, double* x, int solver,
                          const pqn_lcp_opts* opts, pqn_lcp_stats* stats);
pqn_status lcp_solve_dev(pqn_ctx_impl& ctx, int n, const int32_t* pairs, const double* b, double* x, int solver,
                         const pqn_lcp_opts* opts, pqn_lcp_stats* stats);
pqn_status lcp_step(pqn_ctx_impl& ctx, double dt, double delta, int solver, const pqn_lcp_opts* opts,
                    pqn_step_stats* stats);

}  // namespace bipqn
