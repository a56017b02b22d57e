// Learned coarse-grid correction (network set-up, training, inference).
#pragma once

#include "context.hpp"

namespace mfmg {

int net_n_params(int nq);
bool net_supported(int k);
void net_setup(Context& ctx, const LevelDofs& L0);
void net_init_params(Context& ctx, uint64_t seed);
float net_loss_grad(Context& ctx, int rows, const float* X, const float* T, float* grad, hipStream_t s);
void net_train(Context& ctx, const mfmg_net_train_desc& d, float* history, hipStream_t s);
void net_coarse_solve(Context& ctx, int dtype, void* x, const void* b, hipStream_t s);
// y = the network's prediction for the coarse right-hand side b (no check)
void net_predict(Context& ctx, int dtype, void* y, const void* b, hipStream_t s);

}  // namespace mfmg
