// Learned preconditioner (U-Net) -- placeholder until the network kernels land.
#include "rsv_internal.h"

rsv_status learned_create(rsv_matrix *A, const rsv_pc_params *, PcImpl **)
{
    return set_err(A->g->ctx, RSV_ERR_ARG, "learned preconditioner not available in this build");
}

extern "C" {
rsv_status rsv_net_create(rsv_ctx *c, const rsv_net_arch *, uint64_t, rsv_net **) { return set_err(c, RSV_ERR_ARG, "not available"); }
void rsv_net_destroy(rsv_net *) {}
int64_t rsv_net_num_params(const rsv_net *) { return 0; }
rsv_status rsv_net_get_params(rsv_net *, float *, int64_t) { return RSV_ERR_ARG; }
rsv_status rsv_net_set_params(rsv_net *, const float *, int64_t) { return RSV_ERR_ARG; }
rsv_status rsv_net_save(rsv_net *, const char *) { return RSV_ERR_ARG; }
rsv_status rsv_net_load(rsv_net *, const char *) { return RSV_ERR_ARG; }
rsv_status rsv_net_forward(rsv_net *, rsv_grid *, const double *, const float *, double *) { return RSV_ERR_ARG; }
rsv_status rsv_net_train_step(rsv_net *, rsv_grid *, int32_t, const double *, const double *, const float *, float, float *) { return RSV_ERR_ARG; }
rsv_status rsv_net_loss_grad(rsv_net *, rsv_grid *, int32_t, const double *, const double *, const float *, float *, float *) { return RSV_ERR_ARG; }
}
