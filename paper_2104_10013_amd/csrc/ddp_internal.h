// Internal types shared by the host plan builder and the gfx950 kernels.
#pragma once
#include <stdint.h>

namespace ddp {

constexpr int kMaxOut = 3;        // network outputs (u, v, p for Navier-Stokes)
constexpr int kMaxDepth = 8;      // hidden layers
constexpr int kMaxWidth = 112;    // hidden width
constexpr int kWaves = 4;         // waves per workgroup
constexpr int kTilePts = 16 * kWaves;  // points per tile: 16 per wave
constexpr int kLossTerms = 4;     // MSE_u, MSE_F, MSE_uavg, MSE_flux|MSE_R

enum Kind { KIND_RES = 0, KIND_DATA = 1, KIND_IFACE = 2 };
enum Pde { PDE_POISSON = 0, PDE_BURGERS = 1, PDE_NS = 2 };
enum Method { METHOD_CPINN = 0, METHOD_XPINN = 1 };

// One network: widths 2 -> w (x depth) -> d_out.
struct NetDesc {
  int width;        // hidden width w
  int depth;        // hidden layers D
  int d_out;        // outputs
  int wclass;       // padded width class (multiple of 16)
  int64_t poff;     // offset of this network's parameters in the flat buffer
  int n_params;
  float loss_w[4];  // W_u, W_F, W_I, W_flux | W_IF
  float lr;
};

// One work item: a contiguous range of one point set evaluated by one network.
struct Item {
  int q;            // subdomain / network
  int kind;         // Kind
  int begin;        // first point in the kind's packed array
  int count;        // number of points
  int iface;        // interface index (KIND_IFACE) else -1
  int side;         // 0: q is interface side a, 1: side b
  int lrow;         // loss partial row
  float inv_n;      // 1 / size of the point set whose mean this item feeds
  int64_t prow;     // gradient partial row offset (floats)
};

struct IfaceDesc {
  int a, b;
  int begin, count; // range in the packed interface point array
  float nx, ny;
};

// Arguments of the per-point kernels.
struct KArgs {
  const float* params;
  const NetDesc* nets;
  const Item* items;
  int n_items;
  const IfaceDesc* ifaces;
  const float* res_xy;    // 2 per point
  const float* res_f;     // n_eq per point
  const float* dat_xy;
  const float* dat_g;     // d_out per point
  const float* if_xy;
  float* if_val;          // per interface point: 2 sides x n_val
  float* partial;         // gradient partial rows
  float* loss_part;       // kLossTerms per loss row
  float* scratch;         // per-workgroup activation stash
  int64_t scratch_slot;   // floats per workgroup slot
  int* counter;           // work counter of this launch
  int* counters_all;      // all work counters (reset by the prologue)
  int n_counters;
  int* tstate;            // [0] completed Adam steps, [1] pending increment
  int method;
  int n_eq;
  int n_val;              // values per interface point and side
  float coef0;
  int prologue;           // 1: this launch settles t and resets counters
};

// Arguments of the reduction / Adam kernel.
struct RArgs {
  float* params;
  float* adam_m;
  float* adam_v;
  const float* partial;
  const float* loss_part;
  const NetDesc* nets;
  const int64_t* sd_poff;     // n_sd + 1 prefix of parameter offsets
  const int* sd_rows;         // CSR over subdomains of item indices
  const int* sd_row_ptr;      // n_sd + 1
  const int64_t* row_prow;    // per item: gradient partial offset
  const int* row_lrow;        // per item: loss row
  int n_sd;
  int q_begin, q_end;         // subdomain range handled by this launch
  float* grad_out;            // gradient output or nullptr
  float* loss_out;            // n_sd x 5 or nullptr
  int* flags;                 // [0] non-finite loss seen
  int* tstate;
  int do_adam;
};

}  // namespace ddp
