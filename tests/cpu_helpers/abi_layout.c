/* Prints size and field offsets of the structs of include/tmq.h, so that the
 * ctypes mirrors of the Python binding can be checked against the compiler's
 * layout on the host. */
#include <stddef.h>
#include <stdio.h>

#include "tmq.h"

#define F(S, f) printf("%s.%s %zu\n", #S, #f, offsetof(S, f))
#define Z(S) printf("%s %zu\n", #S, sizeof(S))

int main(void)
{
    Z(tmq_params);
    F(tmq_params, kappa); F(tmq_params, mu_tilde); F(tmq_params, theta);
    Z(tmq_nd_params);
    F(tmq_nd_params, kappa); F(tmq_nd_params, mubar_tilde); F(tmq_nd_params, epsbar_tilde);
    F(tmq_nd_params, theta);
    Z(tmq_solver_opts);
    F(tmq_solver_opts, tol); F(tmq_solver_opts, relative); F(tmq_solver_opts, max_iter);
    F(tmq_solver_opts, sloppy); F(tmq_solver_opts, sloppy_link); F(tmq_solver_opts, delta);
    F(tmq_solver_opts, mode);
    Z(tmq_solve_info);
    F(tmq_solve_info, status); F(tmq_solve_info, iters); F(tmq_solve_info, reliable_updates);
    F(tmq_solve_info, true_rel_residual); F(tmq_solve_info, seconds);
    Z(tmq_server_config);
    F(tmq_server_config, budget_bytes); F(tmq_server_config, max_batch);
    Z(tmq_server_stats);
    F(tmq_server_stats, submitted); F(tmq_server_stats, completed); F(tmq_server_stats, failed);
    F(tmq_server_stats, rejected); F(tmq_server_stats, queued); F(tmq_server_stats, running);
    F(tmq_server_stats, p50_s); F(tmq_server_stats, p99_s); F(tmq_server_stats, mean_s);
    F(tmq_server_stats, mean_wait_s); F(tmq_server_stats, solves_per_s); F(tmq_server_stats, elapsed_s);
    F(tmq_server_stats, budget_bytes); F(tmq_server_stats, bytes_in_use); F(tmq_server_stats, peak_bytes);
    F(tmq_server_stats, engines); F(tmq_server_stats, peak_running); F(tmq_server_stats, steps);
    return 0;
}
