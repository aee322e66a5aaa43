// Internal types shared by the host plan builder and the gfx950 kernels.
#pragma once
#include <stdint.h>

namespace ddp {

constexpr int kMaxOut = 3;        // network outputs (u, v, p for Navier-Stokes)
constexpr int kMaxDepth = 8;      // hidden layers
constexpr int kMaxWidth = 112;    // hidden width
constexpr int kWaves = 4;         // waves per workgroup
constexpr int kTilePts = 16 * kWaves;  // points per tile: 16 per wave
constexpr int kRedParams = 256;  // parameters (threads) per block of the gradient reduction
constexpr int kLossTerms = 4;     // MSE_u, MSE_F, MSE_uavg, MSE_flux|MSE_R

// point classes of a work item; KIND_AUX = points with known values of the
// second network (the conductivity K of the inverse diffusion problem)
enum Kind { KIND_RES = 0, KIND_DATA = 1, KIND_IFACE = 2, KIND_AUX = 3 };
enum Pde { PDE_POISSON = 0, PDE_BURGERS = 1, PDE_NS = 2, PDE_INV = 3 };
enum Method { METHOD_CPINN = 0, METHOD_XPINN = 1 };
// hidden-layer activation Phi (Sec. 3; chosen per subdomain in Table 4)
enum Act { ACT_TANH = 0, ACT_SIN = 1, ACT_COS = 2 };

// One network: widths 2 -> w (x depth) -> d_out.
//
// Besides the canonical parameters (per layer W[out][in] then b[out]) every
// network has a zero-padded "kernel layout" copy, rewritten by the Adam kernel
// after each update, with WP = wclass, WS = WP + 4 (LDS row stride):
//   [WP][4]            layer 1: (W1[m][0], W1[m][1], b1[m], 0)
//   per hidden layer k = 2..D:
//     [WP][WS]         W^k            [WP][WS]  W^k transposed    [WP]  b^k
//   [d_out][WP]        output W^L     [4]       b^L
//   [kMaxDepth]        effective slopes c_k = n a^k of hidden layers 1..D
//                      (adaptive networks only; otherwise 1 is used)
// Gradient partial rows use the same order without the transposes and
// without the row padding:  [WP][4], per hidden layer [WP][WP] + [WP],
// [d_out][WP] + [4], [kMaxDepth] (dJ/dc_k).  Canonical parameters of an
// adaptive network end with its D slopes a^1..a^D.
//
// A subdomain owns one network, or two for the inverse diffusion problem (the
// solution u, then the conductivity K at the next index).  Networks are the
// unit of parameters, gradient rows, reduction and Adam; subdomains the unit
// of loss terms.
struct NetDesc {
  int sd;           // owning subdomain
  int pair;         // index of the K-network trained with this u-network, else -1
  int width;        // hidden width w
  int depth;        // hidden layers D
  int d_out;        // outputs
  int wclass;       // padded width class (multiple of 16)
  int64_t poff;     // offset of the canonical parameters in the flat buffer
                    // (a subdomain's networks are adjacent: [u | K])
  int n_params;
  int64_t koff;     // offset of the kernel-layout copy
  int ksize;        // floats of the kernel-layout copy
  int gsize;        // floats of one gradient partial row
  float loss_w[4];  // W_u, W_F, W_I, W_flux | W_IF
  float lr;
  int act;          // Act
  int adaptive;     // 1: trainable slopes a^k (canonical parameters after the layers)
  float slope_n;    // the scale n of the slopes (c_k = n a^k)
};

// kernel-layout and partial-row offsets (floats) of a network
struct Layout {
  int WP, WS, D, DO;
  __host__ __device__ Layout(int wp, int d, int dout) : WP(wp), WS(wp + 4), D(d), DO(dout) {}
  __host__ __device__ int k_hidden(int k) const { return 4 * WP + (k - 2) * (2 * WP * WS + WP); }
  __host__ __device__ int k_w(int k) const { return k_hidden(k); }
  __host__ __device__ int k_wt(int k) const { return k_hidden(k) + WP * WS; }
  __host__ __device__ int k_b(int k) const { return k_hidden(k) + 2 * WP * WS; }
  __host__ __device__ int k_out() const { return k_hidden(D + 1); }
  __host__ __device__ int k_bout() const { return k_out() + DO * WP; }
  __host__ __device__ int k_slope() const { return k_bout() + 4; }
  __host__ __device__ int k_size() const { return k_slope() + kMaxDepth; }
  __host__ __device__ int g_w(int k) const { return 4 * WP + (k - 2) * (WP * WP + WP); }
  __host__ __device__ int g_b(int k) const { return g_w(k) + WP * WP; }
  __host__ __device__ int g_out() const { return g_w(D + 1); }
  __host__ __device__ int g_bout() const { return g_out() + DO * WP; }
  __host__ __device__ int g_slope() const { return g_bout() + 4; }
  __host__ __device__ int g_size() const { return g_slope() + kMaxDepth; }
};

// One work item: a contiguous range of one point set evaluated by one network.
struct Item {
  int q;            // network (the u-network for a paired item)
  int kind;         // Kind
  int begin;        // first point in the kind's packed array
  int count;        // number of points
  int iface;        // interface index (KIND_IFACE) else -1
  int side;         // 0: q is interface side a, 1: side b
  int lrow;         // loss partial row
  float inv_n;      // 1 / size of the point set whose mean this item feeds
  int64_t prow;     // gradient partial row offset (floats); a paired item's
                    // row holds the u-network's part, then the K-network's
};

struct IfaceDesc {
  int a, b;         // subdomains
  int a_net, b_net; // their (u-)networks
  int begin, count; // range in the packed interface point array
  float nx, ny;
  int method;       // interface condition: METHOD_CPINN flux matching or METHOD_XPINN residual continuity
};

// Arguments of the per-point kernels.
struct KArgs {
  const float* kparams;   // kernel-layout parameter copies
  const NetDesc* nets;
  const Item* items;
  int n_items;
  const IfaceDesc* ifaces;
  const float* res_xy;    // 2 per point
  const float* res_f;     // n_eq per point
  const float* dat_xy;
  const float* dat_g;     // d_out per point
  const float* if_xy;
  const float* aux_xy;    // KIND_AUX points
  const float* aux_g;     // 1 per point
  float* partial;         // gradient partial rows
  float* loss_part;       // kLossTerms per loss row
  float* scratch;         // per-workgroup activation stash
  int64_t scratch_slot;   // floats per workgroup slot
  int* counter;           // work counter of this launch (zero at launch)
  int* tstate;            // [0] completed Adam steps, [1] pending increment
  int n_eq;
  float coef0;
  int prologue;           // 1: block 0 settles the Adam step counter
};

// Arguments of the reduction / Adam kernel.
struct RArgs {
  float* params;
  float* kparams;
  float* adam_m;
  float* adam_v;
  const float* partial;
  const float* loss_part;
  const NetDesc* nets;
  const int64_t* net_poff;    // n_nets + 1 prefix of parameter offsets
  const int* net_row_ptr;     // n_nets + 1: CSR over networks of the partial rows
  const int64_t* row_prow;    // per CSR row: offset of that network's part of a row
  const int* sd_net;          // n_sd + 1: first network of each subdomain
  const int* sd_loss_ptr;     // n_sd + 1: CSR over subdomains of the loss rows
  const int* loss_rows;       // per CSR entry: loss row
  int net_begin, net_end;     // networks reduced (and updated) by this launch
  const int* net_blk;         // n_nets + 1: first reduction block of each network (kRedParams a block)
  const int* blk_net;         // per reduction block: its network
  int sd_begin, sd_end;       // subdomains whose loss terms this launch sums
  float* grad_out;            // gradient output or nullptr
  float* loss_out;            // n_sd x 5 or nullptr
  int* flags;                 // [0] non-finite loss seen
  int* tstate;
  int do_adam;
  int* counter_reset;         // work counters to re-arm for the next train launches
  int n_counter_reset;
};

}  // namespace ddp
