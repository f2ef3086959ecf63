// Host launchers of the model / solve kernels and shared enums.
#pragma once
#include "device.hpp"
#include "host.hpp"

namespace inla {

enum { BORDER_CB = 0,   // border rows [C; b^T]  (Newton / prior / final passes)
       BORDER_CI = 1 }; // border rows [C; I]    (marginal variances)

__device__ __forceinline__ int round_up_dev(int v, int m) { return (v + m - 1) / m * m; }

// assembly (k_model.hip)
void launch_expcov_bordered(Ctx &ctx, const ThetaDesc *dtd, int B, int Np_max);
void launch_prior_assemble(Ctx &ctx, const ThetaDesc *dtd, int B, int np_max, double bytes);
// with_lik and m_max > 0: the per-observation terms of general design
// matrices are computed first
void launch_assemble(Ctx &ctx, const ThetaDesc *dtd, int B, int N_max, int with_lik, int want_xqx, int border,
                     double bytes, int prec, int m_max = 0);
void launch_kriging_build(Ctx &ctx, const ThetaDesc *dtd, int B, int kp_max, int prec);
void launch_objective_terms(Ctx &ctx, const ThetaDesc *dtd, int B, int np_max, double bytes);
void launch_kkt_residual(Ctx &ctx, const ThetaDesc *dtd, int B, int np_max, int kp_max, double bytes);

// solves and reductions (k_solve.hip)
void launch_kriging_solve(Ctx &ctx, const ThetaDesc *dtd, int B);
void launch_rhs(Ctx &ctx, const ThetaDesc *dtd, int B, int np_max, int from_z, int prec);
enum { V_X = 0, V_R = 1, V_XN = 2, V_Z = 3, V_U = 4 };   // vector selectors of the solves
// The triangular solves are sequences of np_max / 64 dependent launches; they
// take the host copy of the descriptors and run as one graph replay.
void launch_trsv_fwd(Ctx &ctx, const std::vector<ThetaDesc> &htd, int np_max, int src, int dst, double bytes, int prec);
void launch_trsv_bwd(Ctx &ctx, const std::vector<ThetaDesc> &htd, int np_max, int src, int dst, double bytes, int prec);
void launch_restart(Ctx &ctx, const ThetaDesc *dtd, int B, int np_max);
void launch_newton_accept(Ctx &ctx, const ThetaDesc *dtd, int B);
void launch_ir_correct(Ctx &ctx, const ThetaDesc *dtd, int B, int kp_max, int prec);
void launch_ir_update(Ctx &ctx, const ThetaDesc *dtd, int B);
void launch_finish(Ctx &ctx, const ThetaDesc *dtd, int B, int prec);
void launch_copy_in(Ctx &ctx, const ThetaDesc *dtd, int B, int np_max, int prec);
void launch_copy_out(Ctx &ctx, const ThetaDesc *dtd, int B, int n_max, int prec);
void launch_var_small_build(Ctx &ctx, const ThetaDesc *dtd, int B, int kp_max);
void launch_var_norms(Ctx &ctx, const ThetaDesc *dtd, int B, int np_max);

}  // namespace inla
