// Learned initial guess: gauge-covariant parallel-transport convolution network (FP32).
#pragma once
#include "engine.hpp"

namespace dl {

constexpr int kNetLayers = 3;
constexpr int kNetWidth[kNetLayers + 1] = {4, 16, 16, 4};  // colour-triplet channels per layer boundary

int net_num_weights();       // complex weights over all layers, each [9 hops][C_out][C_in]
long net_weight_offset(int layer);

// Device activations of one forward/backward pass over `items` fields.
struct NetActs {
  int items = 0;
  long nc = 0;
  DBuf<float2> a0, z1, a1, z2, a2;   // input / pre-activations / activations
  DBuf<float2> g16a, g16b, g4, y, r; // gradients and loss work
  DBuf<double> part;                 // reduction partials
  DBuf<double> s, inv_s, bn2;        // per-item input scale s (RMS site norm over the support), 1/s, ||b||^2
  DBuf<float> gsc;                   // per-item gradient scale of the loss
  void ensure(const Lattice& lat, int nitems);
};

}  // namespace dl

struct dl_net {
  dl_ctx* ctx = nullptr;
  dl::DBuf<float2> W;      // weights (FP32 complex), layers concatenated
  dl::DBuf<float2> G;      // gradient of the last loss_grad call
  dl::DBuf<float2> Wt;     // adjoint weights of the backward pass
  dl::DBuf<float> m, v;    // Adam moments (per real component)
  long step = 0;           // Adam steps taken
  dl::DBuf<unsigned> frag16; // BF16 matrix-core operands of the 16 -> 16 layer (built per inference)
  dl::NetActs acts;
  const dl_eig* proj = nullptr;  // training loss over the error left after this Galerkin projection
};

namespace dl {

// Y64 (tiled FP64, nitems fields at stride lat.nc) = net(B) for tiled FP64 B; bf16: the 16 -> 16
// layer's channel mixing with BF16 operands on the matrix cores (FP32 accumulation).
void net_apply(dl_net* net, dl_op* op, int nitems, const double2* B, double2* Y64, bool bf16 = false);
// Mean over items of ||M (net(b) - x)||^2 / ||b||^2; with grad, net->G holds its real gradient.
// With net->proj set (eigenvectors Y of op's M^dag M, H = Y^H M^dag M Y), the error d = net(b) - x
// is first replaced by what the D-CG start leaves of it, d' = d - Y H^-1 Y^H M^dag M d.
double net_loss_grad(dl_net* net, dl_op* op, int nitems, const double2* B, const double2* X, bool grad);
// One Adam step on net->W from net->G (bias-corrected, beta1 0.9, beta2 0.999, eps 1e-8).
void net_adam_step(dl_net* net, float lr);
void net_reset_adam(dl_net* net);

}  // namespace dl
