// gfx950 kernels of one cPINN / XPINN training step.
//
// Each workgroup (4 waves) evaluates one network on a tile of 64 points,
// 16 points per wave.  The network value and its input derivatives are carried
// forward as four "streams" per (neuron, point): value, d/dz0, d/dz1 and the
// second-order sum over the set S the operator needs (S = {x, y} for the
// Laplacian, S = {x} for Burgers' u_xx).  For a hidden layer
//     a = W h + b,  a_i = W h_i,  a_S = W h_S          (Sec. 3 recurrence)
// and through tanh, with t = tanh a, s1 = sech^2 a, s2 = -2 t s1:
//     h = t,  h_i = s1 a_i,  h_S = s1 a_S + s2 sum_{i in S} a_i^2.
// The four streams of 16 points are the columns of one FP32 MFMA contraction
// per layer (v_mfma_f32_16x16x4_f32, weights from LDS); the output layout of
// one layer is the B operand of the next with the K index permuted, so the
// tanh rule stays lane-local.  Pre-activation streams are stashed per
// workgroup in global memory for the reverse pass.
//
// The reverse (adjoint) pass differentiates the subdomain loss of
// Eq. cPINNLoss / Eq. XPINNLoss with respect to the subdomain's own
// parameters: seeds at the output from the PDE residual, data and interface
// terms, the adjoint of the tanh rule (s3 = -2 s1 (1 - 3 t^2))
//     abar_S = s1 g_S
//     abar_i = s1 g_i + 2 s2 a_i g_S            (i in S; s1 g_i otherwise)
//     abar   = s1 g + s2 sum_i a_i g_i + (s2 a_S + s3 sum_{i in S} a_i^2) g_S
// then g_prev = W^T abar (MFMA) and dW = sum over points and streams of
// abar h_prev^T (MFMA over LDS-staged tiles).  Every work item writes its own
// gradient partial row; a second kernel sums the rows of each subdomain in a
// fixed order (deterministic, no float atomics) and applies Adam.

#include <hip/hip_runtime.h>

#include <algorithm>

#include "act_math.h"
#include "ddp_internal.h"
#include "kernels.h"

namespace ddp {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int TP = kTilePts;      // points per tile
constexpr int TPS = kTilePts + 4; // LDS row stride of staged tiles (floats)
constexpr int TPS2 = 2 * kTilePts + 4; // row stride of two streams staged side by side

// Widths whose reverse pass stages two streams at once for dW (one pair of
// barriers per two streams): the doubled staging tiles fit the LDS budget
// of the widest class up to 48.
constexpr bool pair_staged(int wp) { return wp <= 48; }
constexpr int NT = 64 * kWaves;   // threads per workgroup

// One 16-byte-per-lane store into the activation stash, followed by wait
// states before anything may overwrite its data registers.  The compiler
// treats a buffer store with an SGPR offset as free of the store-data
// overwrite hazard and will reuse the data VGPRs in the next instruction; with
// two waves per SIMD such stores were seen to write the later value now and
// then (values read back from the stash came back wrong for a few points),
// and the padding below removes that.
__device__ __forceinline__ void stash_put(f4 v, __amdgpu_buffer_rsrc_t rs, int voff, int soff) {
  __builtin_amdgcn_raw_buffer_store_b128(v, rs, voff, soff, 0);
  __builtin_amdgcn_sched_barrier(0);
  asm volatile("s_nop 4");
  __builtin_amdgcn_sched_barrier(0);
}

// Per-item copy of the thread index the compiler cannot treat as loop
// invariant: keeps per-lane address arithmetic of every width class from being
// hoisted out of the persistent item loop (where it would pin registers).
__device__ __forceinline__ int item_tid() {
  int t = (int)threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// Asynchronous copy of n4 float4 (16-byte aligned at both ends) from global
// memory straight into LDS (gfx950 LDS DMA, no registers): wave `wave`
// copies the 1 KB blocks wave, wave + kWaves, ...; lane l of a block moves
// its 16 bytes to block base + 16 l.  A wave's copies are counted by its
// vector-memory counter; the compiler waits on it only before that wave's own
// LDS reads, so the barrier that hands the buffer to the other waves must be
// preceded by dma_landed() in every wave.
__device__ __forceinline__ void dma_to_lds(float* dst, const float* src, int n4, int wave, int lane) {
  for (int b = wave; b * 64 < n4; b += kWaves) {
    const int c = b * 64 + lane;
    if (c < n4)
      __builtin_amdgcn_global_load_lds(src + 4 * c, (__attribute__((address_space(3))) void*)(dst + 256 * b), 16, 0,
                                       0);
  }
}

// Wait until every vector-memory operation of this wave has completed
// (s_waitcnt vmcnt(0), the other counters left alone), so its LDS DMA copies
// have landed; gfx950 does not wait for them at a barrier by itself.
__device__ __forceinline__ void dma_landed() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Sum over the 16 lanes of each row (the 16 points of one lane group) with
// DPP moves: pairs, quads, half rows, rows.  Every lane of the row receives
// the same (bitwise) sum.
__device__ __forceinline__ float dpp_add(float v, int ctrl) {
  switch (ctrl) {   // the control must be a constant
    case 0xB1: return v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xf, 0xf, false));
    case 0x4E: return v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xf, 0xf, false));
    case 0x141: return v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xf, 0xf, false));
    default: return v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x140, 0xf, 0xf, false));
  }
}
__device__ __forceinline__ float row_sum16(float v) {
  v = dpp_add(v, 0xB1);    // quad_perm [1, 0, 3, 2]
  v = dpp_add(v, 0x4E);    // quad_perm [2, 3, 0, 1]
  v = dpp_add(v, 0x141);   // row_half_mirror
  return dpp_add(v, 0x140);   // row_mirror
}

__device__ __forceinline__ f4 mma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// tanh(a) and sech^2(a) from e = exp(-2|a|):  t = sign(a)(1-e)/(1+e),
// s1 = 4e/(1+e)^2 (no cancellation for large |a|).
__device__ __forceinline__ void tanh_s1(float a, float& t, float& s1) {
  const float e = __expf(-2.f * fabsf(a));
  const float r = __builtin_amdgcn_rcpf(1.f + e);
  t = copysignf((1.f - e) * r, a);
  s1 = 4.f * e * r * r;
}

// Sums over the TP points of LDS-staged rows (16-byte aligned), partially unrolled.
__device__ __forceinline__ float row_sum(const float* a) {
  float acc = 0.f;
#pragma unroll 2
  for (int p = 0; p < TP; p += 4) {
    const f4 x = *reinterpret_cast<const f4*>(a + p);
    acc += (x[0] + x[1]) + (x[2] + x[3]);
  }
  return acc;
}
template <bool S2>
__device__ __forceinline__ void tanh_rule(float a, float ax, float ay, float al, float& h, float& hx,
                                          float& hy, float& hl) {
  float t, s1;
  tanh_s1(a, t, s1);
  const float s2 = -2.f * t * s1;
  h = t;
  hx = s1 * ax;
  hy = s1 * ay;
  const float q = S2 ? fmaf(ax, ax, ay * ay) : ax * ax;
  hl = fmaf(s1, al, s2 * q);
}

template <bool S2>
__device__ __forceinline__ void tanh_adj(float a, float ax, float ay, float al, float g, float gx,
                                         float gy, float gl, float& ab, float& abx, float& aby,
                                         float& abl) {
  float t, s1;
  tanh_s1(a, t, s1);
  const float s2 = -2.f * t * s1;
  const float s3 = -2.f * s1 * (1.f - 3.f * t * t);
  const float q = S2 ? fmaf(ax, ax, ay * ay) : ax * ax;
  abl = s1 * gl;
  abx = fmaf(s1, gx, 2.f * s2 * ax * gl);
  aby = S2 ? fmaf(s1, gy, 2.f * s2 * ay * gl) : s1 * gy;
  ab = fmaf(s1, g, fmaf(s2, fmaf(ax, gx, ay * gy), fmaf(s2, al, s3 * q) * gl));
}

// sin_cos (act_math.h): Cody-Waite reduction and the Cephes single-precision
// polynomials, register-light where pre-activations are small.

// General activation (Sec. 3): h = Phi(c a) with the effective slope c = n a^k
// of the layer and Phi in {tanh, sin, cos}.  The Taylor streams of y = c a are
// c times those of a, so the rule is the unit-slope one on the scaled streams:
// h = Phi(y), d_i h = Phi'(y) d_i y, Delta_S h = Phi'(y) Delta_S y +
// Phi''(y) sum_{i in S} (d_i y)^2.
__device__ __forceinline__ void act_derivs(int act, float y, float& f0, float& f1, float& f2, float& f3) {
  if (act == ACT_TANH) {
    float t, s1;
    tanh_s1(y, t, s1);
    f0 = t;
    f1 = s1;
    f2 = -2.f * t * s1;
    f3 = -2.f * s1 * (1.f - 3.f * t * t);
  } else {
    float sn, cs;
    sin_cos(y, sn, cs);
    f0 = act == ACT_SIN ? sn : cs;
    f1 = act == ACT_SIN ? cs : -sn;
    f2 = -f0;
    f3 = -f1;
  }
}

template <bool S2>
__device__ __forceinline__ void act_rule(int act, float c, float a, float ax, float ay, float al, float& h,
                                         float& hx, float& hy, float& hl) {
  const float y = c * a, yx = c * ax, yy = c * ay, yl = c * al;
  float f0, f1, f2, f3;
  act_derivs(act, y, f0, f1, f2, f3);
  h = f0;
  hx = f1 * yx;
  hy = f1 * yy;
  const float q = S2 ? fmaf(yx, yx, yy * yy) : yx * yx;
  hl = fmaf(f1, yl, f2 * q);
}

// Adjoint of act_rule: from the adjoints g of (h, d_i h, Delta_S h) the
// adjoints of the unscaled streams a (c times those of the scaled streams y),
// and dc += the derivative of the layer's share of J with respect to c, i.e.
// the adjoints of y dotted with the streams of a.
template <bool S2>
__device__ __forceinline__ void act_adj(int act, float c, float a, float ax, float ay, float al, float g, float gx,
                                        float gy, float gl, float& ab, float& abx, float& aby, float& abl,
                                        float& dc) {
  const float y = c * a, yx = c * ax, yy = c * ay, yl = c * al;
  float f0, f1, f2, f3;
  act_derivs(act, y, f0, f1, f2, f3);
  const float q = S2 ? fmaf(yx, yx, yy * yy) : yx * yx;
  const float bl = f1 * gl;
  const float bx = fmaf(f1, gx, 2.f * f2 * yx * gl);
  const float by = S2 ? fmaf(f1, gy, 2.f * f2 * yy * gl) : f1 * gy;
  const float b = fmaf(f1, g, fmaf(f2, fmaf(yx, gx, yy * gy), fmaf(f2, yl, f3 * q) * gl));
  dc = fmaf(b, a, fmaf(bx, ax, fmaf(by, ay, fmaf(bl, al, dc))));
  ab = c * b;
  abx = c * bx;
  aby = c * by;
  abl = c * bl;
}

// ---------------------------------------------------------------------------
// Operators.  u[c][s]: output c, stream s = (value, d/dz0, d/dz1, second order).

template <int PDE> struct Op;

// -Lap u = f   (F = -u_S - f; flux f = -grad u)
template <> struct Op<PDE_POISSON> {
  static constexpr int DO = 1, NEQ = 1;
  static constexpr bool S2 = true;
  __device__ static void residual(const float (&u)[DO][4], const float* f, float coef, float (&F)[NEQ]) {
    F[0] = -u[0][3] - f[0];
  }
  __device__ static void residual_adj(const float (&u)[DO][4], const float (&c)[NEQ], float coef,
                                      float (&ub)[DO][4]) {
    ub[0][3] -= c[0];
  }
  __device__ static void flux(const float (&u)[DO][4], float nx, float ny, float coef, float (&fl)[NEQ]) {
    fl[0] = -(nx * u[0][1] + ny * u[0][2]);
  }
  __device__ static void flux_adj(const float (&u)[DO][4], float nx, float ny, float coef, const float (&c)[NEQ],
                                  float (&ub)[DO][4]) {
    ub[0][1] -= c[0] * nx;
    ub[0][2] -= c[0] * ny;
  }
};

// u_t + u u_x - nu u_xx = f, inputs (x, t); space-time flux (u^2/2 - nu u_x, u)
template <> struct Op<PDE_BURGERS> {
  static constexpr int DO = 1, NEQ = 1;
  static constexpr bool S2 = false;
  __device__ static void residual(const float (&u)[DO][4], const float* f, float nu, float (&F)[NEQ]) {
    F[0] = u[0][2] + u[0][0] * u[0][1] - nu * u[0][3] - f[0];
  }
  __device__ static void residual_adj(const float (&u)[DO][4], const float (&c)[NEQ], float nu,
                                      float (&ub)[DO][4]) {
    ub[0][2] += c[0];
    ub[0][0] += c[0] * u[0][1];
    ub[0][1] += c[0] * u[0][0];
    ub[0][3] -= nu * c[0];
  }
  __device__ static void flux(const float (&u)[DO][4], float nx, float ny, float nu, float (&fl)[NEQ]) {
    fl[0] = nx * (0.5f * u[0][0] * u[0][0] - nu * u[0][1]) + ny * u[0][0];
  }
  __device__ static void flux_adj(const float (&u)[DO][4], float nx, float ny, float nu, const float (&c)[NEQ],
                                  float (&ub)[DO][4]) {
    ub[0][0] += c[0] * (nx * u[0][0] + ny);
    ub[0][1] -= c[0] * nx * nu;
  }
};

// steady incompressible Navier-Stokes, outputs (u, v, p), coef = Re; the
// conservative fluxes of Table 1 (x-momentum, y-momentum, mass) dotted with n:
//   (u^2 + p - u_x/Re, uv - u_y/Re), (uv - v_x/Re, v^2 + p - v_y/Re), (u, v)
template <> struct Op<PDE_NS> {
  static constexpr int DO = 3, NEQ = 3;
  static constexpr bool S2 = true;
  __device__ static void residual(const float (&u)[DO][4], const float* f, float re, float (&F)[NEQ]) {
    const float ir = 1.f / re;
    F[0] = u[0][0] * u[0][1] + u[1][0] * u[0][2] + u[2][1] - ir * u[0][3] - f[0];
    F[1] = u[0][0] * u[1][1] + u[1][0] * u[1][2] + u[2][2] - ir * u[1][3] - f[1];
    F[2] = u[0][1] + u[1][2] - f[2];
  }
  __device__ static void residual_adj(const float (&u)[DO][4], const float (&c)[NEQ], float re,
                                      float (&ub)[DO][4]) {
    const float ir = 1.f / re;
    ub[0][0] += c[0] * u[0][1] + c[1] * u[1][1];
    ub[0][1] += c[0] * u[0][0] + c[2];
    ub[0][2] += c[0] * u[1][0];
    ub[0][3] -= c[0] * ir;
    ub[1][0] += c[0] * u[0][2] + c[1] * u[1][2];
    ub[1][1] += c[1] * u[0][0];
    ub[1][2] += c[1] * u[1][0] + c[2];
    ub[1][3] -= c[1] * ir;
    ub[2][1] += c[0];
    ub[2][2] += c[1];
  }
  __device__ static void flux(const float (&u)[DO][4], float nx, float ny, float re, float (&fl)[NEQ]) {
    const float ir = 1.f / re;
    const float U = u[0][0], V = u[1][0], P = u[2][0];
    // the viscous parts are -(n . grad u)/Re and -(n . grad v)/Re
    const float un = fmaf(nx, u[0][1], ny * u[0][2]), vn = fmaf(nx, u[1][1], ny * u[1][2]);
    fl[0] = fmaf(nx, fmaf(U, U, P), fmaf(ny, U * V, -ir * un));
    fl[1] = fmaf(nx, U * V, fmaf(ny, fmaf(V, V, P), -ir * vn));
    fl[2] = fmaf(nx, U, ny * V);
  }
  __device__ static void flux_adj(const float (&u)[DO][4], float nx, float ny, float re, const float (&c)[NEQ],
                                  float (&ub)[DO][4]) {
    const float ir = 1.f / re;
    const float U = u[0][0], V = u[1][0];
    ub[0][0] += c[0] * (2.f * nx * U + ny * V) + c[1] * nx * V + c[2] * nx;
    ub[1][0] += c[0] * ny * U + c[1] * (nx * U + 2.f * ny * V) + c[2] * ny;
    ub[2][0] += c[0] * nx + c[1] * ny;
    ub[0][1] -= c[0] * ir * nx;
    ub[0][2] -= c[0] * ir * ny;
    ub[1][1] -= c[1] * ir * nx;
    ub[1][2] -= c[1] * ir * ny;
  }
};

// inverse diffusion div(K grad u) = f: both networks carry the (x, y)
// Laplacian stream set; the operator couples the u-network's streams with
// the K-network's and is evaluated in the paired epilogue of Tile, not here
template <> struct Op<PDE_INV> : Op<PDE_POISSON> {};

// epilogue modes of a train tile
enum {
  EPI_OWN = 0,    // the item's own loss terms and output seeds
  EPI_INV_U = 1,  // u-network of a paired inverse item: loss, u seeds, and the K seeds into LDS
  EPI_SEED = 2    // K-network of a paired inverse item: output seeds read from LDS, no loss
};
// parts of a train tile
enum {
  PH_ALL = 0,  // forward, loss / seeds, reverse pass
  PH_FWD = 1,  // forward only (stashed), output streams (value, d/dz0, d/dz1) to LDS
  PH_BWD = 2   // reverse pass only, from the stash of an earlier PH_FWD of the same tile
};
// values_tile modes
enum {
  VAL_OWN = 0,     // interface values of the item's method (u, then flux.n or L(u))
  VAL_STREAMS = 1, // output streams (value, d/dz0, d/dz1) of a one-output network
  VAL_INV_NB = 2   // inverse problem, neighbour u-network: (u, K, L(u, K)) with K from LDS
};

// ---------------------------------------------------------------------------
// Tile processor for one padded width class WP.
//
// Lane layout (one wave = 16 points): lane = 16 g + pc holds point pc and,
// for output block mb and register i, neuron 16 mb + 4 g + i.  This is the
// C/D layout of v_mfma_f32_16x16x4_f32, and with the K index of the next
// contraction permuted the same way it is also its B-operand layout.

// one stream of the tanh rule (used when staging h^{k-1} for dW)
template <bool S2>
__device__ __forceinline__ float act_stream(int s, float a, float ax, float ay, float al) {
  float t, s1;
  tanh_s1(a, t, s1);
  if (s == 0) return t;
  if (s == 1) return s1 * ax;
  if (s == 2) return s1 * ay;
  const float q = S2 ? fmaf(ax, ax, ay * ay) : ax * ax;
  return fmaf(s1, al, -2.f * t * s1 * q);
}

// one stream of the general activation rule (slope c, activation act)
template <bool S2>
__device__ __forceinline__ float act_stream_ga(int s, int act, float c, float a, float ax, float ay, float al) {
  const float y = c * a, yx = c * ax, yy = c * ay, yl = c * al;
  float f0, f1, f2, f3;
  act_derivs(act, y, f0, f1, f2, f3);
  if (s == 0) return f0;
  if (s == 1) return f1 * yx;
  if (s == 2) return f1 * yy;
  const float q = S2 ? fmaf(yx, yx, yy * yy) : yx * yx;
  return fmaf(f1, yl, f2 * q);
}

template <int WP, int PDE>
struct Tile {
  static constexpr int MB = WP / 16;
  static constexpr int DO = Op<PDE>::DO;
  static constexpr int NEQ = Op<PDE>::NEQ;
  static constexpr bool S2 = Op<PDE>::S2;
  static constexpr int WS = WP + 4;                         // row stride of staged weights
  static constexpr int NBT = MB * MB;                       // 16x16 blocks of dW
  static constexpr int NB = (NBT + kWaves - 1) / kWaves;    // dW blocks per wave
  static constexpr int KL = (DO * WP + NT - 1) / NT;        // output-layer slots per thread
  static constexpr int STASH_LAYER = kWaves * 4 * MB * 1024;  // bytes of one layer's stash

  typedef f4 Streams[4][MB];

  // layer 1: a = W^1 z + b^1, a_0 = W^1[:,0], a_1 = W^1[:,1], a_S = 0
  __device__ static void layer1(const float* K, float x, float y, int g, Streams& A) {
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const f4 c = *reinterpret_cast<const f4*>(K + (16 * mb + 4 * g + i) * 4);
        A[0][mb][i] = fmaf(c[0], x, fmaf(c[1], y, c[2]));
        A[1][mb][i] = c[0];
        A[2][mb][i] = c[1];
        A[3][mb][i] = 0.f;
      }
    }
  }

  // GA: a network with another activation than tanh or with trainable
  // slopes (activation act, effective slope c of the layer); else plain tanh
  template <bool GA>
  __device__ static void activate(const Streams& A, Streams& H, int act, float c) {
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float h, hx, hy, hl;
        if constexpr (GA) act_rule<S2>(act, c, A[0][mb][i], A[1][mb][i], A[2][mb][i], A[3][mb][i], h, hx, hy, hl);
        else tanh_rule<S2>(A[0][mb][i], A[1][mb][i], A[2][mb][i], A[3][mb][i], h, hx, hy, hl);
        H[0][mb][i] = h;
        H[1][mb][i] = hx;
        H[2][mb][i] = hy;
        H[3][mb][i] = hl;
      }
    }
  }

  // copy a zero-padded [WP][WS] matrix from the kernel layout into LDS
  __device__ static void stage(float* sW, const float* src, int tid) {
    constexpr int N4 = WP * WS / 4;
    const f4* s4 = reinterpret_cast<const f4*>(src);
    f4* d4 = reinterpret_cast<f4*>(sW);
    for (int idx = tid; idx < N4; idx += NT) d4[idx] = s4[idx];
  }

  // Forward weights alternate between two LDS buffers, sW and the tile buffers
  // sA/sH (free during the forward, WP x WS + WP <= 2 WP x TPS floats), so
  // that layer k + 1's weights stream in while layer k computes; the last
  // hidden layer D always uses sW (the output layer's adjoint stages in sA/sH
  // right after it).
  __device__ static float* wbuf(float* sW, int D, int k) {
    return ((D - k) & 1) ? sW + WP * WS + WP : sW;
  }
  __device__ static void fetch_wb(float* dst, const float* K, const Layout& L, int k, int wave, int lane) {
    dma_to_lds(dst, K + L.k_w(k), WP * WS / 4, wave, lane);
    dma_to_lds(dst + WP * WS, K + L.k_b(k), WP / 4, wave, lane);
  }
  __device__ static void fetch_wt(float* sW, const float* K, const Layout& L, int k, int wave, int lane) {
    dma_to_lds(sW, K + L.k_wt(k), WP * WS / 4, wave, lane);
  }

  // A forward layer's weights and bias go to LDS as [WP][WS] then [WP]: the
  // hidden layer then reads its bias from LDS between its stash stores, and a
  // global load there would have to wait for those stores to drain (one
  // in-order counter covers vector loads and stores).
  static constexpr int NWB4 = (WP * WS + WP) / 4;            // float4 of weights + bias
  __device__ static void stage_wb(float* sW, const float* srcW, const float* srcB, int tid) {
    constexpr int N4 = WP * WS / 4;
    f4* d4 = reinterpret_cast<f4*>(sW);
    for (int idx = tid; idx < NWB4; idx += NT)
      d4[idx] = idx < N4 ? reinterpret_cast<const f4*>(srcW)[idx] : reinterpret_cast<const f4*>(srcB)[idx - N4];
  }

  // One hidden layer, output block by output block: a^k_mb = W^k h^{k-1}
  // (+ b^k on the value stream) for all four streams, stash a^k_mb, and the
  // tanh rule into the new activations Hn (H stays intact as the B operand).
  // rq: MFMA steps of the last 16-neuron input block that hold real neurons
  // (neuron_pos puts neurons 4i..4i+3 of a block in step i); the rest of that
  // block is zero padding and is skipped.
  __device__ static int real_steps(int width) { return (width - (WP - 16) + 3) >> 2; }

  template <bool STASH, bool GA>
  __device__ static void hidden_layer(const float* sW, const float* bias, int g, int pc, int rq, const Streams& H,
                                      Streams& Hn, __amdgpu_buffer_rsrc_t rs, int layer, int wave, int lane, int act,
                                      float c) {
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      f4 acc[4];
      acc[0] = *reinterpret_cast<const f4*>(bias + 16 * mb + 4 * g);
      acc[1] = f4{0.f, 0.f, 0.f, 0.f};
      acc[2] = f4{0.f, 0.f, 0.f, 0.f};
      acc[3] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kb = 0; kb < MB; ++kb) {
        const f4 wv = *reinterpret_cast<const f4*>(&sW[(16 * mb + pc) * WS + 16 * kb + 4 * g]);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          if (kb == MB - 1 && i >= rq) continue;
#pragma unroll
          for (int s = 0; s < 4; ++s) acc[s] = mma(wv[i], H[s][kb][i], acc[s]);
        }
      }
      if constexpr (STASH) {
#pragma unroll
        for (int st = 0; st < 4; ++st)
          stash_put(acc[st], rs, lane * 16, stash_off(0, layer, wave, st, mb));
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float h, hx, hy, hl;
        if constexpr (GA) act_rule<S2>(act, c, acc[0][i], acc[1][i], acc[2][i], acc[3][i], h, hx, hy, hl);
        else tanh_rule<S2>(acc[0][i], acc[1][i], acc[2][i], acc[3][i], h, hx, hy, hl);
        Hn[0][mb][i] = h;
        Hn[1][mb][i] = hx;
        Hn[2][mb][i] = hy;
        Hn[3][mb][i] = hl;
      }
    }
  }

  // g^{k-1}_s = W^{kT} abar^k_s for two streams at once (sW holds W^T): each
  // weight read from LDS feeds two independent MFMA chains
  // (rq as in hidden_layer: padded output neurons of layer k contribute nothing)
  __device__ static void hidden_bwd_pair(const float* sWT, int g, int pc, int rq, const f4 (&A0)[MB],
                                         const f4 (&A1)[MB], f4 (&G0)[MB], f4 (&G1)[MB]) {
#pragma unroll
    for (int jb = 0; jb < MB; ++jb) {
      G0[jb] = f4{0.f, 0.f, 0.f, 0.f};
      G1[jb] = f4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int jb = 0; jb < MB; ++jb) {
        const f4 wv = *reinterpret_cast<const f4*>(&sWT[(16 * jb + pc) * WS + 16 * mb + 4 * g]);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          if (mb == MB - 1 && i >= rq) continue;
          G0[jb] = mma(wv[i], A0[mb][i], G0[jb]);
          G1[jb] = mma(wv[i], A1[mb][i], G1[jb]);
        }
      }
    }
  }

  // Activation stash of the workgroup's slot, [region][layer][wave][stream][mblock][lane]
  // float4, addressed through a buffer resource: region 0 holds the
  // pre-activation streams a^k (k = 2..D), region 1 the post-activation
  // streams h^k (k = 1..D-1) the reverse pass needs for dW^{k+1}.
  static constexpr int STASH_REGION = (kMaxDepth - 1) * STASH_LAYER;
  __device__ static int stash_off(int region, int layer, int wave, int s, int mb) {
    return region * STASH_REGION + layer * STASH_LAYER + ((wave * 4 + s) * MB + mb) * 1024;
  }
  __device__ static void stash_store(__amdgpu_buffer_rsrc_t rs, int region, int layer, int wave, int lane,
                                     const Streams& A) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
        stash_put(A[s][mb], rs, lane * 16, stash_off(region, layer, wave, s, mb));
  }
  // Stash loads read at device scope (SC1): a slot is rewritten by the same
  // wave on every tile, and the per-CU vector L1 must not serve a copy from
  // before the rewrite.
  static constexpr int kStashLoadPolicy = 16;
  __device__ static void stash_load(__amdgpu_buffer_rsrc_t rs, int region, int layer, int wave, int lane,
                                    Streams& A) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
        A[s][mb] = __builtin_amdgcn_raw_buffer_load_b128(rs, lane * 16, stash_off(region, layer, wave, s, mb), kStashLoadPolicy);
  }
  __device__ static void stash_load_stream(__amdgpu_buffer_rsrc_t rs, int region, int layer, int wave, int lane,
                                           int s, f4 (&As)[MB]) {
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
      As[mb] = __builtin_amdgcn_raw_buffer_load_b128(rs, lane * 16, stash_off(region, layer, wave, s, mb), kStashLoadPolicy);
  }

  // output layer u = W^L h + b^L for DO outputs; every lane group ends with
  // the full sums for its point (bitwise identical across groups)
  __device__ static void out_fwd(const float* WL, const float* bL, int g, const Streams& H, float (&u)[DO][4]) {
#pragma unroll
    for (int c = 0; c < DO; ++c) {
      float acc[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        const f4 wv = *reinterpret_cast<const f4*>(WL + c * WP + 16 * mb + 4 * g);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int s = 0; s < 4; ++s) acc[s] = fmaf(wv[i], H[s][mb][i], acc[s]);
      }
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        float v = acc[s];
        v += __shfl_xor(v, 16);
        v += __shfl_xor(v, 32);
        u[c][s] = s == 0 ? v + bL[c] : v;
      }
    }
  }

  // values this network contributes on an interface: u (DO) then the normal
  // flux (cPINN) or the operator value L_x(u) without forcing (XPINN)
  __device__ static void own_values(int method, const float (&u)[DO][4], float nx, float ny, float coef,
                                    float (&ov)[DO + NEQ]) {
#pragma unroll
    for (int c = 0; c < DO; ++c) ov[c] = u[c][0];
    if (method == METHOD_XPINN) {
      const float zero[NEQ] = {};
      float F[NEQ];
      Op<PDE>::residual(u, zero, coef, F);
#pragma unroll
      for (int e = 0; e < NEQ; ++e) ov[DO + e] = F[e];
    } else {
      float fl[NEQ];
      Op<PDE>::flux(u, nx, ny, coef, fl);
#pragma unroll
      for (int e = 0; e < NEQ; ++e) ov[DO + e] = fl[e];
    }
  }

  // loss contributions and output seeds of one point (the derivative of the
  // item's share of J_q with respect to the output streams)
  //
  // EPI_INV_U: inv holds the K-network's streams (K, K_x, K_y) per tile point
  // and nb the neighbour's (u, K, L) on interfaces; F = L - f with
  // L = K Lap u + K_x u_x + K_y u_y (Eq. heq expanded), and kb receives the
  // seeds of (K, K_x, K_y).  EPI_SEED: the seeds come from inv + 3 TP.
  template <int MODE>
  __device__ __forceinline__ static void epilogue(const KArgs& ka, const Item& it, const NetDesc& nd, int pt, int tp, bool valid,
                                  const float* nb, const float* inv, const float (&u)[DO][4], float (&ub)[DO][4],
                                  float (&loss)[kLossTerms], float (&kb)[3]) {
#pragma unroll
    for (int c = 0; c < DO; ++c)
#pragma unroll
      for (int s = 0; s < 4; ++s) ub[c][s] = 0.f;
#pragma unroll
    for (int t = 0; t < kLossTerms; ++t) loss[t] = 0.f;
    kb[0] = kb[1] = kb[2] = 0.f;
    if (!valid) return;
    const float inv_n = it.inv_n;
    const int gp = it.begin + pt;
    if constexpr (MODE == EPI_SEED) {
#pragma unroll
      for (int s = 0; s < 3; ++s) ub[0][s] = inv[3 * TP + 3 * tp + s];
      return;
    } else if constexpr (MODE == EPI_INV_U) {
      const float K = inv[3 * tp], Kx = inv[3 * tp + 1], Ky = inv[3 * tp + 2];
      const float L = fmaf(K, u[0][3], fmaf(Kx, u[0][1], Ky * u[0][2]));
      float c;
      if (it.kind == KIND_RES) {
        const float F = L - ka.res_f[gp];
        loss[1] += F * F;
        c = 2.f * nd.loss_w[1] * F * inv_n;
      } else {
        const float dT = u[0][0] - nb[0], dK = K - nb[1], dL = L - nb[2];
        loss[2] += 0.25f * (dT * dT + dK * dK);
        ub[0][0] += 0.5f * nd.loss_w[2] * dT * inv_n;
        kb[0] += 0.5f * nd.loss_w[2] * dK * inv_n;
        loss[3] += dL * dL;
        c = 2.f * nd.loss_w[3] * dL * inv_n;
      }
      ub[0][1] += c * Kx;
      ub[0][2] += c * Ky;
      ub[0][3] += c * K;
      kb[0] += c * u[0][3];
      kb[1] += c * u[0][1];
      kb[2] += c * u[0][2];
      return;
    }
    if (it.kind == KIND_RES) {
      float F[NEQ];
      Op<PDE>::residual(u, ka.res_f + (int64_t)gp * ka.n_eq, ka.coef0, F);
      float c[NEQ];
#pragma unroll
      for (int e = 0; e < NEQ; ++e) {
        loss[1] += F[e] * F[e];
        c[e] = 2.f * nd.loss_w[1] * F[e] * inv_n;
      }
      Op<PDE>::residual_adj(u, c, ka.coef0, ub);
    } else if (it.kind == KIND_DATA || it.kind == KIND_AUX) {
      const float* tg = it.kind == KIND_DATA ? ka.dat_g : ka.aux_g;
#pragma unroll
      for (int c = 0; c < DO; ++c) {
        const float d = u[c][0] - tg[(int64_t)gp * DO + c];
        loss[0] += d * d;
        ub[c][0] += 2.f * nd.loss_w[0] * d * inv_n;
      }
    } else if constexpr (PDE != PDE_INV) {
      const IfaceDesc ifd = ka.ifaces[it.iface];
      float ov[DO + NEQ];
      own_values(ifd.method, u, ifd.nx, ifd.ny, ka.coef0, ov);
#pragma unroll
      for (int c = 0; c < DO; ++c) {
        const float d = ov[c] - nb[c];
        loss[2] += 0.25f * d * d;
        ub[c][0] += 0.5f * nd.loss_w[2] * d * inv_n;
      }
      // the fourth term: residual continuity (XPINN) or flux matching (cPINN),
      // each equation's squared jump summed
      float c[NEQ];
#pragma unroll
      for (int e = 0; e < NEQ; ++e) {
        const float d = ov[DO + e] - nb[DO + e];
        loss[3] += d * d;
        c[e] = 2.f * nd.loss_w[3] * d * inv_n;
      }
      if (ifd.method == METHOD_XPINN) Op<PDE>::residual_adj(u, c, ka.coef0, ub);
      else Op<PDE>::flux_adj(u, ifd.nx, ifd.ny, ka.coef0, c, ub);
    }
  }

  // gradient / loss partial rows: written by the first tile of an item,
  // accumulated by the following ones (read at device scope, as for the stash)
  __device__ static void accum(float* dst, float v, bool first) {
    if (first) *dst = v;
    else *dst = __hip_atomic_load(dst, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + v;
  }
  // the value a partial-row entry holds before this tile (0 on an item's first
  // tile): loaded early into the accumulator, so the tile's sums add onto it
  // and the entry is then simply stored
  __device__ static float prior(const float* src, bool first) {
    return first ? 0.f : __hip_atomic_load(src, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }

  // ------------------------------------------------------------------------
  // forward only, one tile starting at point t0 of the item, results written by
  // the first lane group of each point to dst (stride 3, or DO + NEQ for
  // VAL_OWN):
  //  VAL_OWN      the values this network contributes on an interface (u, then
  //               flux.n or L_x(u)) for the other side's loss -- the exchange of
  //               Algorithm 1 as an on-chip read;
  //  VAL_STREAMS  the output streams (value, d/dz0, d/dz1) of a one-output
  //               network (the K-network of the inverse problem);
  //  VAL_INV_NB   (u, K, L(u, K)) of a neighbour's u-network, with its K streams
  //               read from kin.
  // effective slope c_k = n a^k of hidden layer k (1 unless adaptive)
  __device__ static float slope(const NetDesc& nd, const float* K, const Layout& L, int k) {
    return nd.adaptive ? K[L.k_slope() + k - 1] : 1.f;
  }

  // GA: the general activation rule (any activation, trainable slopes);
  // for a tanh network without slopes it gives the plain rule's values
  template <int VMODE, bool GA>
  __device__ __forceinline__ static void values_tile(const KArgs& ka, const Item& it, const NetDesc& nd, float* lds,
                                                     float* dst, const float* kin, int t0) {
    float* sW = lds;
    const int tid = item_tid();
    const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int g = lane >> 4, pc = lane & 15;
    const int tp = wave * 16 + pc;
    const Layout L(WP, nd.depth, DO);
    const float* K = ka.kparams + nd.koff;
    const float* xyv = it.kind == KIND_IFACE ? ka.if_xy : ka.res_xy;
    const bool valid = t0 + tp < it.count;
    const int gp = it.begin + t0 + tp;
    const float x = valid ? xyv[2 * (int64_t)gp] : 0.f;
    const float y = valid ? xyv[2 * (int64_t)gp + 1] : 0.f;
    Streams H;
    {
      Streams A;
      layer1(K, x, y, g, A);
      activate<GA>(A, H, nd.act, slope(nd, K, L, 1));
    }
    const __amdgpu_buffer_rsrc_t none = __builtin_amdgcn_make_buffer_rsrc(lds, 0, 0, 0x00020000);  // unused
    for (int k = 2; k <= nd.depth; ++k) {
      __syncthreads();
      stage_wb(sW, K + L.k_w(k), K + L.k_b(k), tid);
      __syncthreads();
      Streams Hn;
      hidden_layer<false, GA>(sW, sW + WP * WS, g, pc, real_steps(nd.width), H, Hn, none, 0, wave, lane, nd.act,
                              slope(nd, K, L, k));
#pragma unroll
      for (int st = 0; st < 4; ++st)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) H[st][mb] = Hn[st][mb];
    }
    float u[DO][4];
    out_fwd(K + L.k_out(), K + L.k_bout(), g, H, u);
    if (g != 0) return;
    if constexpr (VMODE == VAL_OWN) {
      const IfaceDesc ifd = ka.ifaces[it.iface];
      float ov[DO + NEQ];
      own_values(ifd.method, u, ifd.nx, ifd.ny, ka.coef0, ov);
#pragma unroll
      for (int v = 0; v < DO + NEQ; ++v) dst[tp * (DO + NEQ) + v] = ov[v];
    } else if constexpr (VMODE == VAL_STREAMS) {
#pragma unroll
      for (int s = 0; s < 3; ++s) dst[3 * tp + s] = u[0][s];
    } else {
      const float Kv = kin[3 * tp], Kx = kin[3 * tp + 1], Ky = kin[3 * tp + 2];
      dst[3 * tp] = u[0][0];
      dst[3 * tp + 1] = Kv;
      dst[3 * tp + 2] = fmaf(Kv, u[0][3], fmaf(Kx, u[0][1], Ky * u[0][2]));
    }
  }

  // ------------------------------------------------------------------------
  // forward, loss, adjoint and parameter-gradient partials of one item
  //
  // PREFETCH_A: load a^{k-1} during layer k of the reverse pass (and a^D while
  // the output layer runs) instead of at the top of each reverse layer.
  // Tiles starting at t_lo .. t_hi - 1 (step TP) of the item; roff is the
  // offset of this network's part in the item's gradient row; MODE selects the
  // epilogue (sInv: the LDS exchange area of the inverse problem); PHASE the
  // parts run.  slot is this network's stash (slot_floats long).
  // Sum of dc over the wave's lanes into sSl[wave] (a fixed butterfly).
  __device__ static void slope_wave_sum(float dc, float* sSl, int lane, int wave) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) dc += __shfl_xor(dc, m);
    if (lane == 0) sSl[wave] = dc;
  }

  template <bool PREFETCH_A, int MODE, int PHASE, bool GA, bool RH>
  __device__ __forceinline__ static void run_train(const KArgs& ka, const Item& it, const NetDesc& nd, float* lds,
                                   float* slot, int64_t slot_floats, const float* sNb, float* sInv, int t_lo,
                                   int t_hi, int roff) {
    constexpr bool kPair = pair_staged(WP);
    float* sW = lds;
    float* sA = sW + WP * WS + WP;   // after the staged weights and bias
    float* sH = sA + WP * TPS;
    // two streams side by side ([neuron][stream][point], rows of TPS2 floats)
    // over the same space and beyond it
    float* sH2 = sA + WP * TPS2;
    float* sRed = sA + 2 * WP * (kPair ? TPS2 : TPS);   // [kWaves][kLossTerms]
    float* sSl = sRed + kWaves * kLossTerms;   // [kWaves] slope-gradient sums
    const int D = nd.depth;
    const Layout L(WP, D, DO);
    const float* K = ka.kparams + nd.koff;
    float* R = ka.partial + it.prow + roff;
    const float* xy = it.kind == KIND_RES    ? ka.res_xy
                      : it.kind == KIND_DATA ? ka.dat_xy
                      : it.kind == KIND_AUX  ? ka.aux_xy
                                             : ka.if_xy;
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(slot, 0, (int)(slot_floats * sizeof(float)), 0x00020000);

    for (int t0 = t_lo; t0 < t_hi; t0 += TP) {
      // lane indices re-derived per tile (see item_tid)
      int tid = item_tid();
      int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
      int g = lane >> 4, pc = lane & 15;
      int tp = wave * 16 + pc;
      const bool first = t0 == 0;
      const int pt = t0 + tp;
      const bool valid = pt < it.count;
      const int gp = it.begin + pt;
      const float x = valid ? xy[2 * (int64_t)gp] : 0.f;
      const float y = valid ? xy[2 * (int64_t)gp + 1] : 0.f;
      __syncthreads();  // previous tile done with LDS
      // the first hidden layer's weights stream in during layer 1
      if (PHASE != PH_BWD && D >= 2) fetch_wb(wbuf(sW, D, 2), K, L, 2, wave, lane);

      // ---- forward: Taylor streams through every layer, stash a^k (in PH_BWD
      // only h^D is rebuilt, from the stashed a^D, or from layer 1 if D = 1)
      Streams H;
      {
        Streams A;
        if (PHASE == PH_BWD && D >= 2) stash_load(rs, 0, D - 2, wave, lane, A);
        else layer1(K, x, y, g, A);
        activate<GA>(A, H, nd.act, slope(nd, K, L, PHASE == PH_BWD && D >= 2 ? D : 1));
      }
      for (int k = 2; k <= (PHASE == PH_BWD ? 1 : D); ++k) {
        tid = item_tid();
        lane = tid & 63;
        wave = __builtin_amdgcn_readfirstlane(tid >> 6);
        g = lane >> 4;
        pc = lane & 15;
        tp = wave * 16 + pc;
        // W^k is in LDS (every wave's share landed) and every wave is done
        // with layer k - 1's buffer, which now receives W^{k+1}
        dma_landed();
        __syncthreads();
        if (k < D) fetch_wb(wbuf(sW, D, k + 1), K, L, k + 1, wave, lane);
        if constexpr (!RH) stash_store(rs, 1, k - 2, wave, lane, H);   // h^{k-1}
        Streams Hn;
        float* wb = wbuf(sW, D, k);
        hidden_layer<true, GA>(wb, wb + WP * WS, g, pc, real_steps(nd.width), H, Hn, rs, k - 2, wave, lane,
                               nd.act, slope(nd, K, L, k));   // stashes a^k
#pragma unroll
        for (int st = 0; st < 4; ++st)
#pragma unroll
          for (int mb = 0; mb < MB; ++mb) H[st][mb] = Hn[st][mb];
      }
      float u[DO][4];
      if constexpr (PHASE == PH_BWD) {
#pragma unroll
        for (int c = 0; c < DO; ++c) u[c][0] = u[c][1] = u[c][2] = u[c][3] = 0.f;   // seeds come from LDS
      } else {
        out_fwd(K + L.k_out(), K + L.k_bout(), g, H, u);
      }
      if constexpr (PHASE == PH_FWD) {
        if (g == 0) {
#pragma unroll
          for (int s = 0; s < 3; ++s) sInv[3 * tp + s] = u[0][s];
        }
        continue;
      }

      // ---- loss terms and output seeds
      float ub[DO][4], loss[kLossTerms], kb[3];
      epilogue<MODE>(ka, it, nd, pt, tp, valid, sNb + tp * (PDE == PDE_INV ? 3 : DO + NEQ), sInv, u, ub, loss, kb);
#pragma unroll
      for (int t = 0; t < kLossTerms; ++t) {
        float v = g == 0 ? loss[t] : 0.f;
        v += __shfl_xor(v, 1);
        v += __shfl_xor(v, 2);
        v += __shfl_xor(v, 4);
        v += __shfl_xor(v, 8);
        if (lane == 0) sRed[wave * kLossTerms + t] = v;
      }
      if constexpr (MODE == EPI_INV_U) {
        if (g == 0) {
#pragma unroll
          for (int s = 0; s < 3; ++s) sInv[3 * TP + 3 * tp + s] = kb[s];
        }
      }

      // ---- output layer adjoint: g^D = W^{LT} ubar; dW^L, db^L
      // dW^L[c][n] = sum over points and streams of ubar_c h^D_n and db^L[c] =
      // sum over points of ubar_c (value stream): each lane's point term, summed
      // over the wave's 16 points by row_sum16 and over the waves through LDS
      // (sA is free: the last forward layer used sW)
      {
        float* sOut = sA;                      // [kWaves][DO][WP], then [kWaves][DO] bias sums
        float* sOutB = sA + kWaves * DO * WP;
#pragma unroll
        for (int c = 0; c < DO; ++c) {
#pragma unroll
          for (int mb = 0; mb < MB; ++mb) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              float v = ub[c][0] * H[0][mb][i];
#pragma unroll
              for (int st = 1; st < 4; ++st) v = fmaf(ub[c][st], H[st][mb][i], v);
              v = row_sum16(v);
              if (pc == 0) sOut[(wave * DO + c) * WP + 16 * mb + 4 * g + i] = v;
            }
          }
          const float vb = row_sum16(ub[c][0]);
          if (lane == 0) sOutB[wave * DO + c] = vb;
        }
      }
      Streams G;
      {
        const float* WL = K + L.k_out();
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
          f4 wl[DO];
#pragma unroll
          for (int c = 0; c < DO; ++c) wl[c] = *reinterpret_cast<const f4*>(WL + c * WP + 16 * mb + 4 * g);
#pragma unroll
          for (int i = 0; i < 4; ++i) {
#pragma unroll
            for (int s = 0; s < 4; ++s) {
              float acc = 0.f;
#pragma unroll
              for (int c = 0; c < DO; ++c) acc = fmaf(wl[c][i], ub[c][s], acc);
              G[s][mb][i] = acc;
            }
          }
        }
      }
      // a^D for the first reverse layer, loaded while the output layer runs
      // (where registers allow; else at the top of each reverse layer)
      Streams Ak;
      if ((PREFETCH_A || RH) && D >= 2) stash_load(rs, 0, D - 2, wave, lane, Ak);
      __syncthreads();
      // every wave is past the last forward layer: W^{D T} streams into sW
      if (D >= 2) fetch_wt(sW, K, L, D, wave, lane);
#pragma unroll
      for (int r = 0; r < KL; ++r) {
        const int t = tid + r * NT;
        if (t < DO * WP) {
          float v = prior(R + L.g_out() + t, first);
#pragma unroll
          for (int wv = 0; wv < kWaves; ++wv) v += sA[wv * DO * WP + t];
          R[L.g_out() + t] = v;
        }
      }
      if (tid < DO) {
        float v = prior(R + L.g_bout() + tid, first);
#pragma unroll
        for (int wv = 0; wv < kWaves; ++wv) v += sA[kWaves * DO * WP + wv * DO + tid];
        R[L.g_bout() + tid] = v;
      }
      if (MODE != EPI_SEED && tid < kLossTerms) {   // the u pass holds a paired item's loss
        float v = 0.f;
        for (int wv = 0; wv < kWaves; ++wv) v += sRed[wv * kLossTerms + tid];
        accum(ka.loss_part + (int64_t)it.lrow * kLossTerms + tid, v * it.inv_n, first);
      }

      // ---- hidden layers, top down.  G holds g^k on entry to layer k; it is
      // turned into abar^k in place, and stream by stream each abar^k_s is
      // replaced by g^{k-1}_s once it has been staged for dW^k, so the reverse
      // pass holds one layer of streams plus one stream in flight.
      for (int k = D; k >= 2; --k) {
        // and again per layer, so address arithmetic is not pinned across layers
        tid = item_tid();
        lane = tid & 63;
        wave = __builtin_amdgcn_readfirstlane(tid >> 6);
        g = lane >> 4;
        pc = lane & 15;
        tp = wave * 16 + pc;
        // dW^k / db^k accumulators start from the partial row
        float* Rw = R + L.g_w(k);
        f4 dacc[NB];
#pragma unroll
        for (int r = 0; r < NB; ++r) {
          const int b = wave + r * kWaves;
          if (b < NBT) {
            const int mb = b / MB, jb = b - (b / MB) * MB;
#pragma unroll
            for (int i = 0; i < 4; ++i) dacc[r][i] = prior(Rw + (16 * mb + 4 * g + i) * WP + 16 * jb + pc, first);
          } else {
            dacc[r] = f4{0.f, 0.f, 0.f, 0.f};
          }
        }
        float dbias = tid < WP ? prior(R + L.g_b(k) + tid, first) : 0.f;
        // abar^k from the stashed a^k (loaded ahead) and the incoming g^k (in place
        // of g^k); with a general activation also the layer's slope gradient
        {
          if (!PREFETCH_A && !RH) stash_load(rs, 0, k - 2, wave, lane, Ak);
          const float ck = GA ? slope(nd, K, L, k) : 1.f;
          float dc = 0.f;
#pragma unroll
          for (int mb = 0; mb < MB; ++mb) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              float a0, a1, a2, a3;
              if constexpr (GA)
                act_adj<S2>(nd.act, ck, Ak[0][mb][i], Ak[1][mb][i], Ak[2][mb][i], Ak[3][mb][i], G[0][mb][i],
                            G[1][mb][i], G[2][mb][i], G[3][mb][i], a0, a1, a2, a3, dc);
              else
                tanh_adj<S2>(Ak[0][mb][i], Ak[1][mb][i], Ak[2][mb][i], Ak[3][mb][i], G[0][mb][i], G[1][mb][i],
                             G[2][mb][i], G[3][mb][i], a0, a1, a2, a3);
              G[0][mb][i] = a0;
              G[1][mb][i] = a1;
              G[2][mb][i] = a2;
              G[3][mb][i] = a3;
            }
          }
          if constexpr (GA) slope_wave_sum(dc, sSl, lane, wave);
        }
        // recompute policy: a^{k-1} now (the stash for k - 1 >= 2, layer 1
        // from the point itself), h^{k-1} rebuilt from it stream by stream below
        if constexpr (RH) {
          if (k > 2) stash_load(rs, 0, k - 3, wave, lane, Ak);
          else layer1(K, x, y, g, Ak);
        }
        Streams& Ab = G;
        dma_landed();
        __syncthreads();   // W^{kT} is in sW (fetched during the previous stage)
        if constexpr (GA) {
          if (nd.adaptive && tid == 0) accum(R + L.g_slope() + k - 1, (sSl[0] + sSl[1]) + (sSl[2] + sSl[3]), first);
        }
        // per stream: g^{k-1}_s = W^{kT} abar^k_s, then the stream's share of
        // dW^k = sum_{points, streams} abar^k h^{k-1 T}; db^k = sum_points abar^k_0.
        // The barrier that frees sA/sH from the previous stream's dW comes after
        // the W^T abar products, which only read sW: a wave that finished its
        // dW blocks early goes on with them.
        // streams in pairs (0, 1), (2, 3): g^{k-1} of both = W^{kT} abar^k
        // (one weight read per two MFMAs), then per stream its share of dW^k
        // wider classes load h^{k-1} per stream: in the inverse problem's
        // kernels and the one-wave classes one stream ahead (stream s + 1 while
        // stream s runs its dW and, after stream 1, the next pair's W^T abar);
        // elsewhere right before use, where the register budget is tighter
        // (measured: ahead is 1.7-2.7 % faster there, 1.3-1.8 % slower here)
        constexpr bool kEarlyH = WP <= 64;
        constexpr bool kNextH = !RH && !kEarlyH && (PDE == PDE_INV || WP >= 96);
        f4 Hnext[MB];
        if constexpr (kNextH) stash_load_stream(rs, 1, k - 2, wave, lane, 0, Hnext);
#pragma unroll
        for (int sp = 0; sp < 2; ++sp) {
          // h^{k-1} of both streams (stored in the forward), loaded ahead of the
          // pair's MFMAs so that their latency hides behind them (where the
          // registers allow: classes up to 64; wider ones one stream ahead)
          f4 Hp[2][MB];
          if constexpr (!RH && kEarlyH) {
#pragma unroll
            for (int hh = 0; hh < 2; ++hh) stash_load_stream(rs, 1, k - 2, wave, lane, 2 * sp + hh, Hp[hh]);
          }
          f4 Gp[2][MB];
          hidden_bwd_pair(sW, g, pc, real_steps(nd.width), Ab[2 * sp], Ab[2 * sp + 1], Gp[0], Gp[1]);
          if constexpr (kPair) {
            // both streams of the pair staged at once: dW^k over 2 x 64
            // (stream, point) terms per barrier pair
            f4 Hs2[2][MB];
#pragma unroll
            for (int hh = 0; hh < 2; ++hh) {
              const int s = 2 * sp + hh;
              if constexpr (RH) {
                const float cp = GA ? slope(nd, K, L, k - 1) : 1.f;
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                  for (int i = 0; i < 4; ++i) {
                    if constexpr (GA)
                      Hs2[hh][mb][i] =
                          act_stream_ga<S2>(s, nd.act, cp, Ak[0][mb][i], Ak[1][mb][i], Ak[2][mb][i], Ak[3][mb][i]);
                    else
                      Hs2[hh][mb][i] = act_stream<S2>(s, Ak[0][mb][i], Ak[1][mb][i], Ak[2][mb][i], Ak[3][mb][i]);
                  }
              } else {
#pragma unroll
                for (int mb = 0; mb < MB; ++mb) Hs2[hh][mb] = Hp[hh][mb];
              }
            }
            if (sp > 0) __syncthreads();
#pragma unroll
            for (int hh = 0; hh < 2; ++hh)
#pragma unroll
              for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                  sA[(16 * mb + 4 * g + i) * TPS2 + hh * TP + tp] = Ab[2 * sp + hh][mb][i];
                  sH2[(16 * mb + 4 * g + i) * TPS2 + hh * TP + tp] = Hs2[hh][mb][i];
                }
#pragma unroll
            for (int hh = 0; hh < 2; ++hh)
#pragma unroll
              for (int mb = 0; mb < MB; ++mb) G[2 * sp + hh][mb] = Gp[hh][mb];
            if (PREFETCH_A && !RH && sp == 1 && k > 2) stash_load(rs, 0, k - 3, wave, lane, Ak);
            __syncthreads();
            if (sp == 1 && k > 2) fetch_wt(sW, K, L, k - 1, wave, lane);
#pragma unroll
            for (int r = 0; r < NB; ++r) {
              __builtin_amdgcn_sched_barrier(0);
              const int b = wave + r * kWaves;
              if (b < NBT) {
                const int mb = b / MB, jb = b - (b / MB) * MB;
#pragma unroll
                for (int gq = 0; gq < 2 * TP / 16; ++gq) {
                  const f4 av = *reinterpret_cast<const f4*>(&sA[(16 * mb + pc) * TPS2 + 16 * gq + 4 * g]);
                  const f4 hv = *reinterpret_cast<const f4*>(&sH2[(16 * jb + pc) * TPS2 + 16 * gq + 4 * g]);
#pragma unroll
                  for (int i = 0; i < 4; ++i) dacc[r] = mma(av[i], hv[i], dacc[r]);
                }
              }
            }
            // db^k from stream 0 (the first half of each row)
            if (sp == 0 && tid < WP) dbias += row_sum(sA + tid * TPS2);
            continue;
          }
#pragma unroll
          for (int hh = 0; hh < 2; ++hh) {
            const int s = 2 * sp + hh;
            f4 Hs[MB];
            if constexpr (RH) {   // h^{k-1}_s = the activation rule on a^{k-1}
              const float cp = GA ? slope(nd, K, L, k - 1) : 1.f;
#pragma unroll
              for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                  if constexpr (GA)
                    Hs[mb][i] =
                        act_stream_ga<S2>(s, nd.act, cp, Ak[0][mb][i], Ak[1][mb][i], Ak[2][mb][i], Ak[3][mb][i]);
                  else
                    Hs[mb][i] = act_stream<S2>(s, Ak[0][mb][i], Ak[1][mb][i], Ak[2][mb][i], Ak[3][mb][i]);
                }
            } else if constexpr (kEarlyH) {
#pragma unroll
              for (int mb = 0; mb < MB; ++mb) Hs[mb] = Hp[hh][mb];
            } else if constexpr (kNextH) {
#pragma unroll
              for (int mb = 0; mb < MB; ++mb) Hs[mb] = Hnext[mb];   // h^{k-1}_s (stored in the forward)
            } else {
              stash_load_stream(rs, 1, k - 2, wave, lane, s, Hs);   // h^{k-1}_s (stored in the forward)
            }
            if (s > 0) __syncthreads();
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                sA[(16 * mb + 4 * g + i) * TPS + tp] = Ab[s][mb][i];
                sH[(16 * mb + 4 * g + i) * TPS + tp] = Hs[mb][i];
              }
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) G[s][mb] = Gp[hh][mb];   // g^{k-1}_s replaces abar^k_s
            // a^{k-1} for the next reverse layer, loaded during the last dW^k stream
            if (PREFETCH_A && !RH && s == 3 && k > 2) stash_load(rs, 0, k - 3, wave, lane, Ak);
            if constexpr (kNextH) {
              if (s < 3) stash_load_stream(rs, 1, k - 2, wave, lane, s + 1, Hnext);
            }
            __syncthreads();
            // every wave is done with W^{kT}: W^{(k-1)T} streams in during the last dW^k
            if (s == 3 && k > 2) fetch_wt(sW, K, L, k - 1, wave, lane);
#pragma unroll
            for (int r = 0; r < NB; ++r) {
              __builtin_amdgcn_sched_barrier(0);
              const int b = wave + r * kWaves;
              if (b < NBT) {
                const int mb = b / MB, jb = b - (b / MB) * MB;
#pragma unroll
                for (int gq = 0; gq < TP / 16; ++gq) {
                  const f4 av = *reinterpret_cast<const f4*>(&sA[(16 * mb + pc) * TPS + 16 * gq + 4 * g]);
                  const f4 hv = *reinterpret_cast<const f4*>(&sH[(16 * jb + pc) * TPS + 16 * gq + 4 * g]);
#pragma unroll
                  for (int i = 0; i < 4; ++i) dacc[r] = mma(av[i], hv[i], dacc[r]);
                }
              }
            }
            if (s == 0 && tid < WP) dbias += row_sum(sA + tid * TPS);
          }
        }
#pragma unroll
        for (int r = 0; r < NB; ++r) {
          const int b = wave + r * kWaves;
          if (b < NBT) {
            const int mb = b / MB, jb = b - (b / MB) * MB;
#pragma unroll
            for (int i = 0; i < 4; ++i) Rw[(16 * mb + 4 * g + i) * WP + 16 * jb + pc] = dacc[r][i];
          }
        }
        if (tid < WP) R[L.g_b(k) + tid] = dbias;
      }

      // ---- layer 1: abar^1 from a^1 and g^1; dW^1[n] = sum over points of
      // (abar^1_n z + d abar^1_n) and db^1[n] = sum of abar^1_n: each lane's
      // point terms, summed over the wave's 16 points by row_sum16 and over
      // the waves through LDS
      {
        float p0 = 0.f, p1 = 0.f, p2 = 0.f;
        if (tid < WP) {
          p0 = prior(R + 4 * tid, first);
          p1 = prior(R + 4 * tid + 1, first);
          p2 = prior(R + 4 * tid + 2, first);
        }
        Streams A1;
        layer1(K, x, y, g, A1);
        const float c1 = GA ? slope(nd, K, L, 1) : 1.f;
        float dc = 0.f;
        float* sOut = sA;   // [kWaves][3][WP]
        __syncthreads();    // every wave is done with sA (the last dW, or the output layer's sums)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            float a0, a1, a2, a3;
            if constexpr (GA)
              act_adj<S2>(nd.act, c1, A1[0][mb][i], A1[1][mb][i], A1[2][mb][i], A1[3][mb][i], G[0][mb][i],
                          G[1][mb][i], G[2][mb][i], G[3][mb][i], a0, a1, a2, a3, dc);
            else
              tanh_adj<S2>(A1[0][mb][i], A1[1][mb][i], A1[2][mb][i], A1[3][mb][i], G[0][mb][i], G[1][mb][i],
                           G[2][mb][i], G[3][mb][i], a0, a1, a2, a3);
            const float r0 = row_sum16(fmaf(a0, x, a1));
            const float r1 = row_sum16(fmaf(a0, y, a2));
            const float r2 = row_sum16(a0);
            if (pc == 0) {
              const int n = 16 * mb + 4 * g + i;
              sOut[(wave * 3 + 0) * WP + n] = r0;
              sOut[(wave * 3 + 1) * WP + n] = r1;
              sOut[(wave * 3 + 2) * WP + n] = r2;
            }
          }
        }
        if constexpr (GA) slope_wave_sum(dc, sSl, lane, wave);
        __syncthreads();
        if constexpr (GA) {
          if (nd.adaptive && tid == 0) accum(R + L.g_slope(), (sSl[0] + sSl[1]) + (sSl[2] + sSl[3]), first);
        }
        if (tid < WP) {
          float dw0 = p0, dw1 = p1, db = p2;
#pragma unroll
          for (int wv = 0; wv < kWaves; ++wv) {
            dw0 += sOut[(wv * 3 + 0) * WP + tid];
            dw1 += sOut[(wv * 3 + 1) * WP + tid];
            db += sOut[(wv * 3 + 2) * WP + tid];
          }
          R[4 * tid] = dw0;
          R[4 * tid + 1] = dw1;
          R[4 * tid + 2] = db;
          if (first) R[4 * tid + 3] = 0.f;
        }
      }
    }
  }

  // entry from a kernel built for classes up to WPMAX: the a^k prefetch costs
  // registers, so it is used for classes up to 48 in kernels that run two
  // waves per SIMD anyway because of a wider class
  // (GA as in values_tile)
  template <int WPMAX, int MODE, int PHASE, bool GA, bool RH>
  __device__ __forceinline__ static void train(const KArgs& ka, const Item& it, const NetDesc& nd, float* lds, float* slot,
                               int64_t slot_floats, const float* sNb, float* sInv, int t_lo, int t_hi, int roff) {
    run_train<(WP <= 48 && WPMAX >= 48), MODE, PHASE, GA, RH>(ka, it, nd, lds, slot, slot_floats, sNb, sInv, t_lo,
                                                               t_hi, roff);
  }
};

// LDS floats of a train kernel for classes up to WP: the tile buffers of
// Tile<WP> (sW, sA, sH, sRed, sSl), then the neighbour values sNb (6 per
// point), then for the inverse problem 9 per point: the own K streams, the K
// seeds, the neighbour's K streams.
template <int WP>
constexpr int tile_need_floats() {
  return WP * (WP + 4) + WP + 2 * WP * (pair_staged(WP) ? TPS2 : TPS) + kWaves * kLossTerms + kWaves;
}
template <int WP, int PDE>
constexpr int lds_tile_floats() {
  // the largest need of the classes up to WP (a pair-staged narrow class
  // can need more than a wider one)
  int n = 0;
  if (WP >= 16) n = tile_need_floats<16>();
  if (WP >= 32) n = n > tile_need_floats<32>() ? n : tile_need_floats<32>();
  if (WP >= 48) n = n > tile_need_floats<48>() ? n : tile_need_floats<48>();
  if (WP >= 64) n = n > tile_need_floats<64>() ? n : tile_need_floats<64>();
  if (WP >= 80) n = n > tile_need_floats<80>() ? n : tile_need_floats<80>();
  if (WP >= 96) n = n > tile_need_floats<96>() ? n : tile_need_floats<96>();
  if (WP >= 112) n = n > tile_need_floats<112>() ? n : tile_need_floats<112>();
  return n;
}
template <int WP, int PDE>
constexpr int lds_train_floats() {
  return lds_tile_floats<WP, PDE>() + 6 * TP + (PDE == PDE_INV ? 9 * TP : 0);
}

// bytes of dynamic LDS the train kernel is launched with: the tile buffers and
// one 16-byte slot for the work-item broadcast
template <int WP, int PDE>
constexpr int lds_train_bytes() {
  return lds_train_floats<WP, PDE>() * 4 + 16;
}

// Run one item: for an interface item first evaluate the neighbour's network
// on the same tile (its width class may differ), then the item's own network.
// A paired item of the inverse problem goes tile by tile: the neighbour's K-
// and u-networks (interfaces), the own K-network's streams, the u-network's
// train pass (loss, u seeds, K seeds), then the K-network's train pass.
template <int WPMAX, int PDE, bool GA, bool RH>
__device__ __forceinline__ void dispatch(const KArgs& ka, const Item& it, const NetDesc& nd, float* lds,
                                         float* slot) {
  float* sNb = lds + lds_tile_floats<WPMAX, PDE>();
  float* sInv = sNb + 6 * TP;
#define DDP_CASE(WPV, ...)                                    \
  case WPV:                                                   \
    if constexpr (WPV <= WPMAX) Tile<WPV, PDE>::__VA_ARGS__;  \
    break;
#define DDP_SWITCH(CLS, ...)     \
  switch (CLS) {                 \
    DDP_CASE(16, __VA_ARGS__)    \
    DDP_CASE(32, __VA_ARGS__)    \
    DDP_CASE(48, __VA_ARGS__)    \
    DDP_CASE(64, __VA_ARGS__)    \
    DDP_CASE(80, __VA_ARGS__)    \
    DDP_CASE(96, __VA_ARGS__)    \
    DDP_CASE(112, __VA_ARGS__)   \
    default: break;              \
  }
  if constexpr (PDE == PDE_INV) {
    if (nd.pair >= 0 && (it.kind == KIND_RES || it.kind == KIND_IFACE)) {
      const NetDesc ndk = ka.nets[nd.pair];
      NetDesc nbu = nd, nbk = ndk;
      if (it.kind == KIND_IFACE) {
        const IfaceDesc ifd = ka.ifaces[it.iface];
        nbu = ka.nets[it.side == 0 ? ifd.b_net : ifd.a_net];
        nbk = ka.nets[nbu.pair];
      }
      // each network of the pair stashes into its own half of the slot: the
      // K-network's forward (its streams to LDS) comes first, its reverse pass
      // after the u-network's whole tile
      const int64_t half = ka.scratch_slot / 2;
      for (int t0 = 0; t0 < it.count; t0 += TP) {
        __syncthreads();
        if (it.kind == KIND_IFACE) {
          DDP_SWITCH(nbk.wclass,
                     template values_tile<VAL_STREAMS, GA>(ka, it, nbk, lds, sInv + 6 * TP, nullptr, t0))
          __syncthreads();
          DDP_SWITCH(nbu.wclass, template values_tile<VAL_INV_NB, GA>(ka, it, nbu, lds, sNb, sInv + 6 * TP, t0))
          __syncthreads();
        }
        DDP_SWITCH(ndk.wclass, template train<WPMAX, EPI_SEED, PH_FWD, GA, RH>(ka, it, ndk, lds, slot + half, half,
                                                                            sNb, sInv, t0, t0 + 1, nd.gsize))
        DDP_SWITCH(nd.wclass,
                   template train<WPMAX, EPI_INV_U, PH_ALL, GA, RH>(ka, it, nd, lds, slot, half, sNb, sInv, t0, t0 + 1, 0))
        DDP_SWITCH(ndk.wclass, template train<WPMAX, EPI_SEED, PH_BWD, GA, RH>(ka, it, ndk, lds, slot + half, half,
                                                                            sNb, sInv, t0, t0 + 1, nd.gsize))
      }
      return;
    }
  } else if (it.kind == KIND_IFACE) {
    const IfaceDesc ifd = ka.ifaces[it.iface];
    const NetDesc ndn = ka.nets[it.side == 0 ? ifd.b_net : ifd.a_net];
    __syncthreads();
    DDP_SWITCH(ndn.wclass, template values_tile<VAL_OWN, GA>(ka, it, ndn, lds, sNb, nullptr, 0))
    __syncthreads();
  }
  DDP_SWITCH(nd.wclass, template train<WPMAX, EPI_OWN, PH_ALL, GA, RH>(ka, it, nd, lds, slot,
                                                       PDE == PDE_INV ? ka.scratch_slot / 2 : ka.scratch_slot, sNb,
                                                       sInv, 0, it.count, 0))
#undef DDP_SWITCH
#undef DDP_CASE
}

// Persistent kernel: workgroups pull items (in descending cost order) from a
// device counter until the list is drained.
// Widths up to 80 fit two waves per SIMD (<= 256 registers); wider classes
// run one wave per SIMD.
template <int WPMAX>
constexpr int min_waves_per_eu() {
  return WPMAX <= 80 ? 2 : 1;
}

// GA: kernels with the general activation rule, launched for problems where a
// network uses another activation than tanh or trainable slopes (built for
// the class groups up to 80 and up to 112 only)
template <int WPMAX, int PDE, bool GA, bool RH>
__global__ __launch_bounds__(NT, min_waves_per_eu<WPMAX>()) void k_train(KArgs ka) {
  // one 16-byte aligned dynamic LDS block: the tile buffers, then the slot
  // that broadcasts the next work item (no static LDS, so the float4
  // accesses of the tile buffers stay 16-byte aligned)
  extern __shared__ __attribute__((aligned(16))) float lds[];
  int& s_item = *reinterpret_cast<int*>(lds + lds_train_floats<WPMAX, PDE>());
  float* slot = ka.scratch + (int64_t)blockIdx.x * ka.scratch_slot;
  if (ka.prologue && blockIdx.x == 0 && threadIdx.x == 0) {
    // settle the Adam step counter of the previous update (k_reduce reads it)
    ka.tstate[0] += ka.tstate[1];
    ka.tstate[1] = 0;
  }
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(ka.counter, 1);
    __syncthreads();
    const int idx = s_item;
    __syncthreads();
    if (idx >= ka.n_items) break;
    const Item it = ka.items[idx];
    const NetDesc nd = ka.nets[it.q];
    dispatch<WPMAX, PDE, GA, RH>(ka, it, nd, lds, slot);
  }
}

// Position of hidden neuron n in the kernel layout and the gradient rows: the
// index inside each 16-neuron block is transposed as a 4x4 grid (4a + b ->
// 4b + a).  Register i of lane group g then holds neuron 16 mb + 4 i + g, so
// the MFMA step i of a contraction over a block covers four consecutive
// neurons, and in a padded last block the steps past the real neurons can be
// skipped.  The map is its own inverse.
__host__ __device__ __forceinline__ int neuron_pos(int n) { return (n & ~15) | ((n & 3) << 2) | ((n >> 2) & 3); }

// Position of canonical parameter li of a network in its gradient partial row
// (g) and in its kernel-layout copy (k1, and k2 for the transposed copy of a
// hidden weight, else -1).  sc: the kernel copy holds sc times the parameter
// and the partial rows hold the gradient divided by sc (n for a slope a^k,
// whose kernel copy is c_k = n a^k; 1 otherwise).
__device__ __forceinline__ void param_map(const NetDesc& nd, int li, int& g, int& k1, int& k2, float& sc) {
  const int w = nd.width, WP = nd.wclass, D = nd.depth, DO = nd.d_out;
  const Layout L(WP, D, DO);
  k2 = -1;
  sc = 1.f;
  if (li < 2 * w) {                 // W^1[m][c]
    const int m = li >> 1, c = li & 1;
    g = k1 = neuron_pos(m) * 4 + c;
    return;
  }
  if (li < 3 * w) {                 // b^1[m]
    g = k1 = neuron_pos(li - 2 * w) * 4 + 2;
    return;
  }
  int r = li - 3 * w;
  const int per = w * w + w;
  const int h = r / per;
  if (h < D - 1) {                  // hidden layer k = h + 2
    const int k = h + 2;
    const int rr = r - h * per;
    if (rr < w * w) {
      const int m = neuron_pos(rr / w), j = neuron_pos(rr - (rr / w) * w);
      g = L.g_w(k) + m * WP + j;
      k1 = L.k_w(k) + m * L.WS + j;
      k2 = L.k_wt(k) + j * L.WS + m;
    } else {
      const int m = neuron_pos(rr - w * w);
      g = L.g_b(k) + m;
      k1 = L.k_b(k) + m;
    }
    return;
  }
  r -= (D - 1) * per;               // output layer
  if (r < DO * w) {
    const int c = r / w, j = neuron_pos(r - (r / w) * w);
    g = L.g_out() + c * WP + j;
    k1 = L.k_out() + c * WP + j;
  } else if (r < DO * w + DO) {
    const int c = r - DO * w;
    g = L.g_bout() + c;
    k1 = L.k_bout() + c;
  } else {                          // slope a^k of hidden layer k = 1..D
    const int k = r - DO * w - DO;
    g = L.g_slope() + k;
    k1 = L.k_slope() + k;
    sc = nd.slope_n;
  }
}

// network holding flat parameter i, searching upward from network n
__device__ __forceinline__ int find_net(const int64_t* net_poff, int n, int64_t i) {
  while (net_poff[n + 1] <= i) ++n;
  return n;
}

// The train kernels of each operator are compiled in a translation unit of
// their own (DDP_TRAIN_PDE set to the operator), so the build runs them in
// parallel; the unit without it holds the other kernels and the launchers.
#ifndef DDP_TRAIN_PDE

// Sum each network's gradient partial rows in a fixed order, then write the
// gradient and/or apply Adam (Kingma-Ba, bias corrected) and refresh the
// kernel-layout copy; the waves of block 0 also sum each subdomain's loss
// rows and flag non-finite losses.
//
// A block owns kRedParams consecutive parameters of one network, a thread one
// parameter; it keeps kRedLanes independent partial sums over the rows (row r
// goes to sum r mod kRedLanes), combined by a fixed tree: the loads of a batch
// are independent, and the order does not depend on timing.
constexpr int kRedLanes = 16;

__global__ __launch_bounds__(kRedParams) void k_reduce(RArgs ra) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // the block's network, its row list and the row offsets are uniform
  // across the block (scalar loads)
  const int bidx = ra.net_blk[ra.net_begin] + (int)blockIdx.x;
  if (bidx < ra.net_blk[ra.net_end]) {
    const int q = ra.blk_net[bidx];
    const int64_t i = ra.net_poff[q] + (int64_t)(bidx - ra.net_blk[q]) * kRedParams + threadIdx.x;
    const NetDesc nd = ra.nets[q];
    const int r0 = ra.net_row_ptr[q], n = ra.net_row_ptr[q + 1] - r0;
    const int64_t* pr = ra.row_prow + r0;
    if (i < ra.net_poff[q + 1]) {
      int gi, k1, k2;
      float sc;
      param_map(nd, (int)(i - ra.net_poff[q]), gi, k1, k2, sc);
      const float* P = ra.partial + gi;
      float a[kRedLanes];
#pragma unroll
      for (int j = 0; j < kRedLanes; ++j) a[j] = 0.f;
      int r = 0;
      for (; r + kRedLanes <= n; r += kRedLanes) {
#pragma unroll
        for (int j = 0; j < kRedLanes; ++j) a[j] += P[pr[r + j]];
      }
#pragma unroll
      for (int j = 0; j < kRedLanes; ++j)
        if (r + j < n) a[j] += P[pr[r + j]];
#pragma unroll
      for (int w = kRedLanes / 2; w >= 1; w /= 2)
#pragma unroll
        for (int j = 0; j < w; ++j) a[j] += a[j + w];
      const float s = sc * a[0];
      if (ra.grad_out) ra.grad_out[i] = s;
      if (ra.do_adam) {
        const float tstep = (float)(ra.tstate[0] + 1);
        const float bc1 = 1.f - powf(b1, tstep);
        const float bc2 = 1.f - powf(b2, tstep);
        const float m = b1 * ra.adam_m[i] + (1.f - b1) * s;
        const float v = b2 * ra.adam_v[i] + (1.f - b2) * s * s;
        ra.adam_m[i] = m;
        ra.adam_v[i] = v;
        const float mh = m / bc1;
        const float vh = v / bc2;
        const float th = ra.params[i] - nd.lr * mh / (sqrtf(vh) + eps);
        ra.params[i] = th;
        float* K = ra.kparams + nd.koff;
        K[k1] = sc * th;
        if (k2 >= 0) K[k2] = th;
      }
    }
  }
  if (blockIdx.x == 0) {
    // one wave per subdomain: lane l sums rows l, l + 64, ...; then a fixed
    // butterfly across the wave
    for (int q = ra.sd_begin + wave; q < ra.sd_end; q += (int)(blockDim.x >> 6)) {
      float t[kLossTerms] = {0.f, 0.f, 0.f, 0.f};
      for (int r = ra.sd_loss_ptr[q] + lane; r < ra.sd_loss_ptr[q + 1]; r += 64) {
        const float* lp = ra.loss_part + (int64_t)ra.loss_rows[r] * kLossTerms;
        for (int k = 0; k < kLossTerms; ++k) t[k] += lp[k];
      }
      for (int k = 0; k < kLossTerms; ++k)
        for (int m = 32; m >= 1; m >>= 1) t[k] += __shfl_xor(t[k], m);
      if (lane == 0) {
        const NetDesc nd = ra.nets[ra.sd_net[q]];
        float J = 0.f;
        for (int k = 0; k < kLossTerms; ++k) J += nd.loss_w[k] * t[k];
        if (ra.loss_out) {
          ra.loss_out[q * 5] = J;
          for (int k = 0; k < kLossTerms; ++k) ra.loss_out[q * 5 + 1 + k] = t[k];
        }
        if (!isfinite(J)) ra.flags[0] = 1;
      }
    }
    if (ra.do_adam && threadIdx.x == 0) ra.tstate[1] = 1;
    // the train kernel of this step has finished: re-arm its work counter
    if (ra.counter_reset && (int)threadIdx.x < ra.n_counter_reset) ra.counter_reset[threadIdx.x] = 0;
  }
}

__global__ void k_reset_counter(int* c) { *c = 0; }

// Rewrite the kernel-layout copy of networks [n_begin, n_end) from their
// canonical parameters (after the caller sets them).
__global__ __launch_bounds__(256) void k_pack(const float* params, float* kparams, const NetDesc* nets,
                                              const int64_t* net_poff, int n_begin, int n_end) {
  const int64_t p0 = net_poff[n_begin], p1 = net_poff[n_end];
  for (int64_t i = p0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < p1;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int q = find_net(net_poff, n_begin, i);
    const NetDesc nd = nets[q];
    int gi, k1, k2;
    float sc;
    param_map(nd, (int)(i - net_poff[q]), gi, k1, k2, sc);
    float* K = kparams + nd.koff;
    K[k1] = sc * params[i];
    if (k2 >= 0) K[k2] = params[i];
  }
}

// Stitched solution (Eq. FSol): average of the owning subdomains' outputs;
// the columns are the outputs of a subdomain's networks in order (u, or u
// then K for the inverse problem).  One thread per point.
__global__ __launch_bounds__(256) void k_eval(const float* params, const NetDesc* nets, const int* sd_net, int n_sd,
                                              int n, const float* xy, const int* owner, float* out, int n_cols) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float acc[kMaxOut] = {0.f, 0.f, 0.f};
  int cnt = 0;
  float h[kMaxWidth], h2[kMaxWidth];
  const float x = xy[2 * i], y = xy[2 * i + 1];
  for (int o = 0; o < 4; ++o) {
    const int q = owner[4 * i + o];
    if (q < 0 || q >= n_sd) continue;
    ++cnt;
    int col = 0;
    for (int net = sd_net[q]; net < sd_net[q + 1]; ++net) {
      const NetDesc nd = nets[net];
      const float* P = params + nd.poff;
      const int w = nd.width;
      // slopes follow the output layer in the canonical layout
      const float* Sl = P + 3 * w + (int64_t)(nd.depth - 1) * (w * w + w) + nd.d_out * w + nd.d_out;
      // sin and cos as in training (sin_cos); tanh from the library
      auto phi = [&](float a, int k) {
        const float yv = nd.adaptive ? nd.slope_n * Sl[k - 1] * a : a;
        if (nd.act == ACT_TANH) return tanhf(yv);
        float sn, cs;
        sin_cos(yv, sn, cs);
        return nd.act == ACT_SIN ? sn : cs;
      };
      for (int m = 0; m < w; ++m) h[m] = phi(fmaf(P[2 * m], x, fmaf(P[2 * m + 1], y, P[2 * w + m])), 1);
      int64_t off = 3 * w;
      for (int k = 2; k <= nd.depth; ++k) {
        for (int m = 0; m < w; ++m) {
          float a = P[off + w * w + m];
          for (int j = 0; j < w; ++j) a = fmaf(P[off + m * w + j], h[j], a);
          h2[m] = phi(a, k);
        }
        for (int m = 0; m < w; ++m) h[m] = h2[m];
        off += w * w + w;
      }
      for (int c = 0; c < nd.d_out && col < n_cols; ++c, ++col) {
        float a = P[off + nd.d_out * w + c];
        for (int j = 0; j < w; ++j) a = fmaf(P[off + c * w + j], h[j], a);
        acc[col] += a;
      }
    }
  }
  for (int c = 0; c < n_cols; ++c) out[(int64_t)i * n_cols + c] = cnt ? acc[c] / cnt : 0.f;
}

#endif  // DDP_TRAIN_PDE

// ---------------------------------------------------------------------------
// host-side launchers

static int wclass_index(int wpmax) {
  switch (wpmax) {
    case 16: return 0;
    case 32: return 1;
    case 48: return 2;
    case 64: return 3;
    case 80: return 4;
    case 96: return 5;
    case 112: return 6;
  }
  return -1;
}

// Train kernels per operator and activation policy RH (0: the forward
// stashes a^k and h^k; 1: it stashes a^k only and the reverse pass rebuilds
// h^{k-1} from a^{k-1}), and the LDS bytes per class (policy-independent).
template <int PDE, int RH>
struct KTable {
  static const void* train[7];
  static const void* train_ga[2];   // general activation: class groups up to 80, up to 112
};
template <int PDE>
struct KLds {
  static int lds[7];
};
// (a unit built with DDP_TRAIN_GA defines the general-activation row of its
// operator and policy, one without it the plain row, and with policy 0 also
// the LDS sizes)
#ifndef DDP_TRAIN_RH
#define DDP_TRAIN_RH 0
#endif
#ifdef DDP_TRAIN_GA
#define DDP_ROW(PDE, RH)                                                                                          \
  template <> const void* KTable<PDE, RH>::train_ga[2] = {(const void*)k_train<80, PDE, true, RH>,                \
                                                          (const void*)k_train<112, PDE, true, RH>};
#else
#define DDP_ROW(PDE, RH)                                                                                          \
  template <> const void* KTable<PDE, RH>::train[7] = {                                                           \
      (const void*)k_train<16, PDE, false, RH>, (const void*)k_train<32, PDE, false, RH>,                         \
      (const void*)k_train<48, PDE, false, RH>, (const void*)k_train<64, PDE, false, RH>,                         \
      (const void*)k_train<80, PDE, false, RH>, (const void*)k_train<96, PDE, false, RH>,                         \
      (const void*)k_train<112, PDE, false, RH>};
#endif
#ifdef DDP_TRAIN_PDE
DDP_ROW(DDP_TRAIN_PDE, (DDP_TRAIN_RH != 0))
#if !defined(DDP_TRAIN_GA) && DDP_TRAIN_RH == 0
template <> int KLds<DDP_TRAIN_PDE>::lds[7] = {
    lds_train_bytes<16, DDP_TRAIN_PDE>(), lds_train_bytes<32, DDP_TRAIN_PDE>(), lds_train_bytes<48, DDP_TRAIN_PDE>(),
    lds_train_bytes<64, DDP_TRAIN_PDE>(), lds_train_bytes<80, DDP_TRAIN_PDE>(), lds_train_bytes<96, DDP_TRAIN_PDE>(),
    lds_train_bytes<112, DDP_TRAIN_PDE>()};
#endif
#undef DDP_ROW
#else
#undef DDP_ROW
// the tables are defined in the operators' own translation units
#define DDP_DECL(PDE)                                                  \
  template <> const void* KTable<PDE, false>::train[7];                \
  template <> const void* KTable<PDE, true>::train[7];                 \
  template <> const void* KTable<PDE, false>::train_ga[2];             \
  template <> const void* KTable<PDE, true>::train_ga[2];              \
  template <> int KLds<PDE>::lds[7];
DDP_DECL(PDE_POISSON)
DDP_DECL(PDE_BURGERS)
DDP_DECL(PDE_NS)
DDP_DECL(PDE_INV)
#undef DDP_DECL

template <int RH>
static const void* pick_rh(int pde, int c, bool ga, int g) {
  switch (pde) {
    case PDE_POISSON: return ga ? KTable<PDE_POISSON, RH>::train_ga[g] : KTable<PDE_POISSON, RH>::train[c];
    case PDE_BURGERS: return ga ? KTable<PDE_BURGERS, RH>::train_ga[g] : KTable<PDE_BURGERS, RH>::train[c];
    case PDE_NS: return ga ? KTable<PDE_NS, RH>::train_ga[g] : KTable<PDE_NS, RH>::train[c];
    case PDE_INV: return ga ? KTable<PDE_INV, RH>::train_ga[g] : KTable<PDE_INV, RH>::train[c];
  }
  return nullptr;
}

static const void* pick(int pde, int wpmax, bool ga, bool rh) {
  const int c = wclass_index(wpmax);
  if (c < 0) return nullptr;
  int g = 0;
  if (ga) {   // general-activation kernels exist for the groups up to 80 and up to 112
    if (wpmax != 80 && wpmax != 112) return nullptr;
    g = wpmax == 80 ? 0 : 1;
  }
  return rh ? pick_rh<true>(pde, c, ga, g) : pick_rh<false>(pde, c, ga, g);
}

size_t lds_bytes(int pde, int wpmax) {
  const int c = wclass_index(wpmax);
  if (c < 0) return 0;
  int f = 0;
  switch (pde) {
    case PDE_POISSON: f = KLds<PDE_POISSON>::lds[c]; break;
    case PDE_BURGERS: f = KLds<PDE_BURGERS>::lds[c]; break;
    case PDE_NS: f = KLds<PDE_NS>::lds[c]; break;
    case PDE_INV: f = KLds<PDE_INV>::lds[c]; break;
  }
  return (size_t)f;
}

int64_t scratch_slot_floats(int pde, int wpmax, bool rh) {
  // two regions (a^k and h^k) of kMaxDepth - 1 layers, or the a^k region
  // alone under the recompute policy; the inverse problem keeps one such
  // stash per network of a pair
  const int64_t one = (int64_t)(rh ? 1 : 2) * (kMaxDepth - 1) * kWaves * 4 * (wpmax / 16) * 64 * 4;
  return pde == PDE_INV ? 2 * one : one;
}

int kernel_wpmax(int wpmax, bool ga) { return ga ? (wpmax <= 80 ? 80 : 112) : wpmax; }

hipError_t launch_train(int pde, int wpmax, bool ga, bool rh, const KArgs& ka, int grid, hipStream_t st) {
  const void* fn = pick(pde, wpmax, ga, rh);
  if (!fn) return hipErrorInvalidValue;
  KArgs a = ka;
  void* args[] = {&a};
  return hipLaunchKernel(fn, dim3(grid), dim3(NT), args, lds_bytes(pde, wpmax), st);
}

hipError_t train_occupancy(int pde, int wpmax, bool ga, bool rh, int* blocks_per_cu) {
  const void* fn = pick(pde, wpmax, ga, rh);
  if (!fn) return hipErrorInvalidValue;
  const size_t lds = lds_bytes(pde, wpmax);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, fn, NT, lds);
}

hipError_t launch_reset_counter(int* c, hipStream_t st) {
  hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, st, c);
  return hipGetLastError();
}

hipError_t launch_reduce(const RArgs& ra, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce, dim3(grid), dim3(kRedParams), 0, st, ra);
  return hipGetLastError();
}

hipError_t launch_pack(const float* params, float* kparams, const NetDesc* nets, const int64_t* net_poff,
                       int n_begin, int n_end, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int grid = (int)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_pack, dim3(grid), dim3(256), 0, st, params, kparams, nets, net_poff, n_begin, n_end);
  return hipGetLastError();
}

hipError_t launch_eval(const float* params, const NetDesc* nets, const int* sd_net, int n_sd, int n, const float* xy,
                       const int* owner, float* out, int n_cols, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_eval, dim3((n + 255) / 256), dim3(256), 0, st, params, nets, sd_net, n_sd, n, xy, owner, out,
                     n_cols);
  return hipGetLastError();
}

#endif  // DDP_TRAIN_PDE
}  // namespace ddp
