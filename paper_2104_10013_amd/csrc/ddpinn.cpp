// libddpinn: host side of the C ABI declared in include/ddpinn.h.
//
// Builds the packed plan (per-network descriptors, point arrays, interface
// table, work items in descending-cost order, gradient partial rows), owns
// the device buffers, launches the kernels of kernels.hip, and captures the
// fused step as a HIP graph.
#include "../../include/ddpinn.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "ddp_internal.h"
#include "kernels.h"

using namespace ddp;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIP_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(DDP_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));          \
  } while (0)

struct HostSd {
  std::vector<int> widths;
  std::vector<int> aux_widths;  // K-network (inverse problem), else empty
  float loss_w[4];
  float lr;
  std::vector<float> res_xy, res_f, dat_xy, dat_g, aux_xy, aux_g;
  int n_res = 0, n_dat = 0, n_aux = 0;
  int act = DDP_ACT_TANH;   // activation of the subdomain's networks
  int adaptive = 0;         // 1: trainable slopes, one per hidden layer of each network
  float slope_n = 10.f;
};

struct HostIf {
  int a, b, n;
  std::vector<float> xy;
  float nx, ny;
  int method = -1;   // interface condition; -1: the problem's method
};

template <class T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
};

bool all_finite(const float* v, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

int width_class(int w) { return ((w + 15) / 16) * 16; }

}  // namespace

struct ddp_problem {
  int method = 0, pde = 0;
  double coef[4] = {0, 0, 0, 0};
  int n_eq = 1, d_out = 1;
  std::vector<HostSd> sds;
  std::vector<HostIf> ifs;
  int64_t chunk_points = 1024;  // upper bound of points per work item
  int blocks_per_cu = 0;         // 0: from the occupancy query
  int items_per_slot = 4;        // work items per resident workgroup the plan aims for
  int recompute = 0;             // activation policy: 1 stash a^k and rebuild h^k in the reverse pass, 0 stash both
  int concurrent = 0;            // fused step with several train launches: 1 = they run side by side
  int tail_pct = 0;              // percent of each subdomain's residual points in one-tile items

  // plan
  bool planned = false, finalized = false;
  bool plan_ok = false;          // install_plan completed: work list, rows, stash and graph are in place
  int fused = 1;
  int wpmax = 16;                // width group of the (plain path's) train kernel
  bool ga = false;               // some network needs the general activation rule
  std::vector<NetDesc> nets;     // a subdomain's networks are adjacent: u [, K]
  std::vector<int> sd_net;       // n_sd + 1: first network of each subdomain
  std::vector<int64_t> sd_poff;  // n_sd + 1: parameter offsets of subdomains
  std::vector<int64_t> net_poff; // n_nets + 1: parameter offsets of networks
  std::vector<int> net_blk, blk_net;  // reduction blocks: CSR over networks, and each block's network
  int64_t kparam_floats = 0;
  int plan_slots = 512;          // workgroups the plan balances for
  std::vector<Item> titems;      // train items (fused: descending cost per launch; plain: grouped by q)
  // fused path: one persistent launch per kernel class the items need (items
  // whose networks are all at most 80 wide run in a kernel that fits two
  // waves per SIMD; items with a wider network in the widest class's kernel)
  struct Launch {
    int wpmax = 16;          // widest class of the launch's items
    int begin = 0, count = 0;
    int occupancy = 1;       // resident workgroups per CU of that kernel
    int n_slots = 1;
    int64_t slot_floats = 0;
    int64_t scratch_off = 0;  // first float of the launch's stash slots in the scratch buffer
  };
  std::vector<Launch> launches;
  std::vector<int> t_begin;      // per q ranges (plain path), n_sd + 1
  std::vector<IfaceDesc> ifaces;
  // gradient rows: CSR over networks (item index and offset of the network's
  // part); loss rows: CSR over subdomains
  std::vector<int> net_row_ptr, net_row_item, sd_loss_ptr, loss_rows;
  std::vector<int64_t> row_prow;
  int64_t partial_floats = 0;
  std::vector<float> h_res_xy, h_res_f, h_dat_xy, h_dat_g, h_if_xy, h_aux_xy, h_aux_g;

  // device
  int device = 0;
  hipStream_t stream = nullptr;      // caller's stream
  hipStream_t cap_stream = nullptr;  // private stream used for graph capture
  hipStream_t side_stream = nullptr; // second stream of concurrent train launches
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  int n_slots = 0;
  int64_t slot_floats = 0;
  float *d_params = nullptr, *d_m = nullptr, *d_v = nullptr, *d_kparams = nullptr;
  int *d_tstate = nullptr, *d_flags = nullptr, *d_counters = nullptr;
  int n_counters = 0;
  NetDesc* d_nets = nullptr;
  Item* d_titems = nullptr;
  IfaceDesc* d_ifaces = nullptr;
  float *d_res_xy = nullptr, *d_res_f = nullptr, *d_dat_xy = nullptr, *d_dat_g = nullptr;
  float *d_if_xy = nullptr, *d_aux_xy = nullptr, *d_aux_g = nullptr;
  float *d_partial = nullptr, *d_loss_part = nullptr, *d_scratch = nullptr, *d_loss = nullptr;
  int64_t* d_net_poff = nullptr;
  int *d_net_blk = nullptr, *d_blk_net = nullptr;
  int* d_sd_net = nullptr;
  int *d_net_row_ptr = nullptr, *d_sd_loss_ptr = nullptr, *d_loss_rows = nullptr;
  int64_t* d_row_prow = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  std::vector<void*> allocations;       // static buffers
  std::vector<void*> plan_allocations;  // buffers that depend on the work plan
  int n_cu = 0, occupancy = 0;
};

namespace {

template <class T>
int dev_alloc(ddp_problem* p, T** out, size_t count) {
  *out = nullptr;
  if (count == 0) count = 1;
  void* ptr = nullptr;
  hipError_t e = hipMalloc(&ptr, count * sizeof(T));
  if (e != hipSuccess) return fail(DDP_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  p->allocations.push_back(ptr);
  *out = static_cast<T*>(ptr);
  return DDP_OK;
}

template <class T>
int plan_alloc(ddp_problem* p, T** out, size_t count) {
  int rc = dev_alloc(p, out, count);
  if (rc) return rc;
  p->allocations.pop_back();
  p->plan_allocations.push_back(*out);
  return DDP_OK;
}

template <class T>
int plan_upload(ddp_problem* p, T** out, const std::vector<T>& v) {
  int rc = plan_alloc(p, out, v.size());
  if (rc) return rc;
  if (!v.empty()) HIP_TRY(hipMemcpy(*out, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return DDP_OK;
}

template <class T>
int dev_upload(ddp_problem* p, T** out, const std::vector<T>& v) {
  int rc = dev_alloc(p, out, v.size());
  if (rc) return rc;
  if (!v.empty()) HIP_TRY(hipMemcpy(*out, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return DDP_OK;
}

int copy_in(const float* src, size_t n, int on_device, std::vector<float>& dst) {
  dst.resize(n);
  if (n == 0) return DDP_OK;
  if (!src) return fail(DDP_EINVAL, "null input pointer");
  if (on_device) {
    HIP_TRY(hipMemcpy(dst.data(), src, n * sizeof(float), hipMemcpyDeviceToHost));
  } else {
    std::memcpy(dst.data(), src, n * sizeof(float));
  }
  return DDP_OK;
}

int64_t net_param_count(const std::vector<int>& wd, int adaptive) {
  int64_t n = 0;
  for (size_t k = 1; k < wd.size(); ++k) n += (int64_t)wd[k] * wd[k - 1] + wd[k];
  return n + (adaptive ? (int64_t)wd.size() - 2 : 0);
}

double item_cost(const NetDesc& nd, int count) {
  // MFMA work of one item: streams x padded hidden products, forward + backward
  const double wp = nd.wclass;
  return (double)count * (1.0 + (nd.depth - 1) * wp * wp * 24.0 + 40.0 * wp);
}

// work of an item of network q: a paired inverse item also trains the K-network
// and evaluates it once more for its streams (a forward is a third of a train)
double item_cost(const std::vector<NetDesc>& nets, const Item& it) {
  double c = item_cost(nets[it.q], it.count);
  if (nets[it.q].pair >= 0 && (it.kind == KIND_RES || it.kind == KIND_IFACE))
    c += item_cost(nets[nets[it.q].pair], it.count) * (4.0 / 3.0);
  return c;
}

int build_plan(ddp_problem* p) {
  const int n_sd = (int)p->sds.size();
  if (n_sd == 0) return fail(DDP_EINVAL, "no subdomains");
  for (const HostIf& f : p->ifs)
    if (f.a >= n_sd || f.b >= n_sd) return fail(DDP_EINVAL, "interface names an unknown subdomain");
  const int64_t chunk_max = std::max<int64_t>(kTilePts, (p->chunk_points + kTilePts - 1) / kTilePts * kTilePts);

  // networks (u, then K for the inverse problem) and parameter offsets
  p->nets.clear();
  p->sd_net.assign(n_sd + 1, 0);
  p->sd_poff.assign(n_sd + 1, 0);
  p->net_poff.assign(1, 0);
  p->kparam_floats = 0;
  p->wpmax = 16;
  p->ga = false;
  for (int q = 0; q < n_sd; ++q) {
    const HostSd& s = p->sds[q];
    p->sd_net[q] = (int)p->nets.size();
    for (int which = 0; which < (s.aux_widths.empty() ? 1 : 2); ++which) {
      const std::vector<int>& wd = which == 0 ? s.widths : s.aux_widths;
      NetDesc nd{};
      nd.sd = q;
      nd.pair = (which == 0 && !s.aux_widths.empty()) ? (int)p->nets.size() + 1 : -1;
      nd.width = wd[1];
      nd.depth = (int)wd.size() - 2;
      nd.d_out = wd.back();
      nd.wclass = width_class(nd.width);
      nd.poff = p->net_poff.back();
      nd.n_params = (int)net_param_count(wd, s.adaptive);
      const Layout L(nd.wclass, nd.depth, nd.d_out);
      nd.koff = p->kparam_floats;
      nd.ksize = L.k_size();
      nd.gsize = L.g_size();
      p->kparam_floats += nd.ksize;
      for (int k = 0; k < 4; ++k) nd.loss_w[k] = s.loss_w[k];
      nd.lr = s.lr;
      nd.act = s.act;
      nd.adaptive = s.adaptive;
      nd.slope_n = s.slope_n;
      p->net_poff.push_back(nd.poff + nd.n_params);
      p->wpmax = std::max(p->wpmax, nd.wclass);
      if (nd.act != ACT_TANH || nd.adaptive) p->ga = true;
      p->nets.push_back(nd);
    }
    p->sd_poff[q + 1] = p->net_poff.back();
  }
  p->sd_net[n_sd] = (int)p->nets.size();
  p->wpmax = kernel_wpmax(p->wpmax, p->ga);
  // the reduction's blocks: kRedParams consecutive parameters of one network each
  p->net_blk.assign(1, 0);
  p->blk_net.clear();
  for (int q = 0; q < (int)p->nets.size(); ++q) {
    const int nb = (int)((p->net_poff[q + 1] - p->net_poff[q] + kRedParams - 1) / kRedParams);
    for (int b = 0; b < nb; ++b) p->blk_net.push_back(q);
    p->net_blk.push_back(p->net_blk.back() + nb);
  }

  // packed point arrays
  p->h_res_xy.clear();
  p->h_res_f.clear();
  p->h_dat_xy.clear();
  p->h_dat_g.clear();
  p->h_if_xy.clear();
  p->h_aux_xy.clear();
  p->h_aux_g.clear();
  std::vector<int> res_begin(n_sd), dat_begin(n_sd), aux_begin(n_sd);
  for (int q = 0; q < n_sd; ++q) {
    const HostSd& s = p->sds[q];
    res_begin[q] = (int)(p->h_res_xy.size() / 2);
    p->h_res_xy.insert(p->h_res_xy.end(), s.res_xy.begin(), s.res_xy.end());
    p->h_res_f.insert(p->h_res_f.end(), s.res_f.begin(), s.res_f.end());
    dat_begin[q] = (int)(p->h_dat_xy.size() / 2);
    p->h_dat_xy.insert(p->h_dat_xy.end(), s.dat_xy.begin(), s.dat_xy.end());
    p->h_dat_g.insert(p->h_dat_g.end(), s.dat_g.begin(), s.dat_g.end());
    aux_begin[q] = (int)(p->h_aux_xy.size() / 2);
    p->h_aux_xy.insert(p->h_aux_xy.end(), s.aux_xy.begin(), s.aux_xy.end());
    p->h_aux_g.insert(p->h_aux_g.end(), s.aux_g.begin(), s.aux_g.end());
  }
  p->ifaces.clear();
  for (const HostIf& f : p->ifs) {
    IfaceDesc d;
    d.a = f.a;
    d.b = f.b;
    d.a_net = p->sd_net[f.a];
    d.b_net = p->sd_net[f.b];
    d.begin = (int)(p->h_if_xy.size() / 2);
    d.count = f.n;
    d.nx = f.nx;
    d.ny = f.ny;
    d.method = f.method >= 0 ? f.method : p->method;
    p->h_if_xy.insert(p->h_if_xy.end(), f.xy.begin(), f.xy.end());
    p->ifaces.push_back(d);
  }

  // Work items per subdomain: residual, data and interface-side chunks (and
  // K-data chunks of the inverse problem, where residual and interface items
  // train both networks).  The chunk length of each subdomain is chosen so
  // items carry similar work (about 1/items_per_slot of an even share per
  // workgroup), between one 64-point tile and chunk_max points: cheap networks
  // get long items, expensive ones short.
  auto point_cost = [&](int q) {
    Item one{};
    one.q = p->sd_net[q];
    one.kind = KIND_RES;
    one.count = 1;
    return item_cost(p->nets, one);
  };
  double total_cost = 0.0;
  for (int q = 0; q < n_sd; ++q) {
    const HostSd& s = p->sds[q];
    int n_pts = s.n_res + s.n_dat + s.n_aux;
    for (const HostIf& f : p->ifs)
      if (f.a == q || f.b == q) n_pts += f.n;
    total_cost += point_cost(q) * n_pts;
  }
  const double target = total_cost / ((double)std::max(1, p->items_per_slot) * std::max(1, p->plan_slots));
  std::vector<int64_t> chunk_q(n_sd);
  for (int q = 0; q < n_sd; ++q) {
    int64_t c = (int64_t)(target / point_cost(q));
    c = (c + kTilePts - 1) / kTilePts * kTilePts;
    chunk_q[q] = std::min(chunk_max, std::max<int64_t>(kTilePts, c));
  }
  std::vector<std::vector<Item>> per_q(n_sd);
  auto add_chunks = [&](int q, int net, int kind, int begin, int count, int iface, int side, float inv_n) {
    // interface items are one tile: the neighbour's network is evaluated on
    // the same tile first
    // With a tail share, the last tail_pct percent of a subdomain's residual
    // points go into one-tile items, which the cost-ordered queue hands out
    // last: workgroups that finish their long items early share the end.
    const int64_t chunk = kind == KIND_IFACE ? kTilePts : chunk_q[q];
    int64_t tail = 0;
    if (kind == KIND_RES && p->fused && p->tail_pct > 0)
      tail = std::min<int64_t>(count, ((int64_t)count * p->tail_pct / 100 + kTilePts - 1) / kTilePts * kTilePts);
    const int64_t bulk = count - tail;
    for (int64_t c0 = 0; c0 < count;) {
      const int64_t len = c0 < bulk ? std::min<int64_t>(chunk, bulk - c0) : std::min<int64_t>(kTilePts, count - c0);
      Item it{};
      it.q = net;
      it.kind = kind;
      it.begin = begin + (int)c0;
      it.count = (int)len;
      it.iface = iface;
      it.side = side;
      it.inv_n = inv_n;
      per_q[q].push_back(it);
      c0 += len;
    }
  };
  for (int q = 0; q < n_sd; ++q) {
    const HostSd& s = p->sds[q];
    const int u = p->sd_net[q];
    if (s.n_res > 0) add_chunks(q, u, KIND_RES, res_begin[q], s.n_res, -1, 0, 1.f / (float)s.n_res);
    if (s.n_dat > 0) add_chunks(q, u, KIND_DATA, dat_begin[q], s.n_dat, -1, 0, 1.f / (float)s.n_dat);
    if (s.n_aux > 0) add_chunks(q, u + 1, KIND_AUX, aux_begin[q], s.n_aux, -1, 0, 1.f / (float)s.n_aux);
  }
  for (int e = 0; e < (int)p->ifaces.size(); ++e) {
    const IfaceDesc& d = p->ifaces[e];
    if (d.count <= 0) continue;
    add_chunks(d.a, d.a_net, KIND_IFACE, d.begin, d.count, e, 0, 1.f / (float)d.count);
    add_chunks(d.b, d.b_net, KIND_IFACE, d.begin, d.count, e, 1, 1.f / (float)d.count);
  }

  // train items: fused = one list in descending cost (largest first, a
  // greedy longest-processing-time order for the dynamic queue); plain =
  // grouped by subdomain so each launch takes one contiguous range
  auto by_cost = [&](const Item& x, const Item& y) { return item_cost(p->nets, x) > item_cost(p->nets, y); };
  p->titems.clear();
  p->t_begin.assign(n_sd + 1, 0);
  for (int q = 0; q < n_sd; ++q) {
    p->t_begin[q] = (int)p->titems.size();
    std::vector<Item> v = per_q[q];
    std::stable_sort(v.begin(), v.end(), by_cost);
    p->titems.insert(p->titems.end(), v.begin(), v.end());
  }
  p->t_begin[n_sd] = (int)p->titems.size();
  // widest class an item's kernel must handle: its networks, its pair, and on
  // an interface the neighbour's networks
  auto need = [&](const Item& it) {
    const NetDesc& n = p->nets[it.q];
    int c = n.wclass;
    const bool pair = n.pair >= 0 && (it.kind == KIND_RES || it.kind == KIND_IFACE);
    if (pair) c = std::max(c, p->nets[n.pair].wclass);
    if (it.kind == KIND_IFACE) {
      const IfaceDesc& d = p->ifaces[it.iface];
      const int nb = it.side == 0 ? d.b_net : d.a_net;
      c = std::max(c, p->nets[nb].wclass);
      if (p->nets[nb].pair >= 0) c = std::max(c, p->nets[p->nets[nb].pair].wclass);
    }
    return c;
  };
  p->launches.clear();
  if (p->fused) {
    std::vector<Item> narrow, wide;
    int w_narrow = 16, w_wide = 16;
    for (const Item& it : p->titems) {
      const int c = need(it);
      if (c <= 80) {
        narrow.push_back(it);
        w_narrow = std::max(w_narrow, c);
      } else {
        wide.push_back(it);
        w_wide = std::max(w_wide, c);
      }
    }
    std::stable_sort(narrow.begin(), narrow.end(), by_cost);
    std::stable_sort(wide.begin(), wide.end(), by_cost);
    p->titems.clear();
    for (auto* grp : {&narrow, &wide}) {
      if (grp->empty()) continue;
      ddp_problem::Launch l;
      l.wpmax = kernel_wpmax(grp == &narrow ? w_narrow : w_wide, p->ga);
      l.begin = (int)p->titems.size();
      l.count = (int)grp->size();
      p->titems.insert(p->titems.end(), grp->begin(), grp->end());
      p->launches.push_back(l);
    }
  }
  // partial rows and loss rows follow item order; a paired item's row holds
  // the u-network's part, then the K-network's
  auto paired = [&](const Item& it) {
    return p->nets[it.q].pair >= 0 && (it.kind == KIND_RES || it.kind == KIND_IFACE);
  };
  int64_t off = 0;
  for (int i = 0; i < (int)p->titems.size(); ++i) {
    Item& it = p->titems[i];
    it.lrow = i;
    it.prow = off;
    off += p->nets[it.q].gsize + (paired(it) ? p->nets[p->nets[it.q].pair].gsize : 0);
  }
  p->partial_floats = off;
  // gradient row lists per network, loss row lists per subdomain (ascending
  // item index: a fixed summation order)
  const int n_nets = (int)p->nets.size();
  p->net_row_ptr.assign(n_nets + 1, 0);
  p->sd_loss_ptr.assign(n_sd + 1, 0);
  for (const Item& it : p->titems) {
    p->net_row_ptr[it.q + 1]++;
    if (paired(it)) p->net_row_ptr[p->nets[it.q].pair + 1]++;
    p->sd_loss_ptr[p->nets[it.q].sd + 1]++;
  }
  for (int n = 0; n < n_nets; ++n) p->net_row_ptr[n + 1] += p->net_row_ptr[n];
  for (int q = 0; q < n_sd; ++q) p->sd_loss_ptr[q + 1] += p->sd_loss_ptr[q];
  p->net_row_item.assign(p->net_row_ptr[n_nets], 0);
  p->row_prow.assign(p->net_row_ptr[n_nets], 0);
  p->loss_rows.assign(p->titems.size(), 0);
  {
    std::vector<int> fill(p->net_row_ptr.begin(), p->net_row_ptr.end() - 1);
    std::vector<int> lfill(p->sd_loss_ptr.begin(), p->sd_loss_ptr.end() - 1);
    for (int i = 0; i < (int)p->titems.size(); ++i) {
      const Item& it = p->titems[i];
      int r = fill[it.q]++;
      p->net_row_item[r] = i;
      p->row_prow[r] = it.prow;
      if (paired(it)) {
        r = fill[p->nets[it.q].pair]++;
        p->net_row_item[r] = i;
        p->row_prow[r] = it.prow + p->nets[it.q].gsize;
      }
      p->loss_rows[lfill[p->nets[it.q].sd]++] = it.lrow;
    }
  }
  p->planned = true;
  return DDP_OK;
}

KArgs make_kargs(ddp_problem* p) {
  KArgs ka{};
  ka.kparams = p->d_kparams;
  ka.nets = p->d_nets;
  ka.ifaces = p->d_ifaces;
  ka.res_xy = p->d_res_xy;
  ka.res_f = p->d_res_f;
  ka.dat_xy = p->d_dat_xy;
  ka.dat_g = p->d_dat_g;
  ka.if_xy = p->d_if_xy;
  ka.aux_xy = p->d_aux_xy;
  ka.aux_g = p->d_aux_g;
  ka.partial = p->d_partial;
  ka.loss_part = p->d_loss_part;
  ka.scratch = p->d_scratch;
  ka.scratch_slot = p->slot_floats;
  ka.tstate = p->d_tstate;
  ka.n_eq = p->n_eq;
  ka.coef0 = (float)p->coef[0];
  return ka;
}

RArgs make_rargs(ddp_problem* p) {
  RArgs ra{};
  ra.params = p->d_params;
  ra.kparams = p->d_kparams;
  ra.adam_m = p->d_m;
  ra.adam_v = p->d_v;
  ra.partial = p->d_partial;
  ra.loss_part = p->d_loss_part;
  ra.nets = p->d_nets;
  ra.net_poff = p->d_net_poff;
  ra.net_blk = p->d_net_blk;
  ra.blk_net = p->d_blk_net;
  ra.net_row_ptr = p->d_net_row_ptr;
  ra.row_prow = p->d_row_prow;
  ra.sd_net = p->d_sd_net;
  ra.sd_loss_ptr = p->d_sd_loss_ptr;
  ra.loss_rows = p->d_loss_rows;
  ra.flags = p->d_flags;
  ra.tstate = p->d_tstate;
  return ra;
}

// reduction of subdomains [q0, q1): their networks and their loss terms
void reduce_range(ddp_problem* p, RArgs& ra, int q0, int q1) {
  ra.net_begin = p->sd_net[q0];
  ra.net_end = p->sd_net[q1];
  ra.sd_begin = q0;
  ra.sd_end = q1;
}

int reduce_grid(ddp_problem* p, int q0, int q1) {
  // one block per reduction block of the subdomains' networks (block 0 also
  // sums the loss rows, so at least one)
  return std::max(1, p->net_blk[p->sd_net[q1]] - p->net_blk[p->sd_net[q0]]);
}

// Where a step's train launches keep their work counters and activation
// stash: the plan's own buffers (sized for every resident workgroup, the
// counters re-armed by the reduction), or a caller-provided region of cap
// floats (the static scratch) whose counters are zeroed before the launches
// and whose stash slots bound the persistent grid.
struct StepBufs {
  float* scratch;
  int64_t cap_floats;
  int* counters;
};

// kernel sequence of one step (or one loss_and_grad) on stream st
int enqueue_step(ddp_problem* p, hipStream_t st, int do_adam, float* grad_out, float* loss_out,
                 const StepBufs* b = nullptr) {
  const int n_sd = (int)p->sds.size();
  float* scratch = b ? b->scratch : p->d_scratch;
  int* counters = b ? b->counters : p->d_counters;
  auto slots_for = [&](int n_slots, int64_t slot_floats) {
    if (!b) return n_slots;
    return (int)std::max<int64_t>(1, std::min<int64_t>(n_slots, b->cap_floats / std::max<int64_t>(1, slot_floats)));
  };
  if (b) HIP_TRY(launch_zero_ints(counters, p->n_counters, st));
  if (p->fused) {
    // concurrent launches (own stash regions): every launch after the first
    // runs on the side stream, forked from and joined back into st, so a
    // launch's workgroups take the compute units the other's drained ones free
    const bool side = !b && p->concurrent && p->launches.size() > 1;
    if (side) {
      HIP_TRY(hipEventRecord(p->ev_fork, st));
      HIP_TRY(hipStreamWaitEvent(p->side_stream, p->ev_fork, 0));
    }
    for (size_t g = 0; g < p->launches.size(); ++g) {
      const ddp_problem::Launch& l = p->launches[g];
      KArgs ka = make_kargs(p);
      ka.items = p->d_titems + l.begin;
      ka.n_items = l.count;
      ka.counter = counters + g;
      ka.scratch = scratch + (b ? 0 : l.scratch_off);
      ka.scratch_slot = l.slot_floats;
      ka.prologue = g == 0;
      const int grid = std::max(1, std::min(slots_for(l.n_slots, l.slot_floats), l.count));
      HIP_TRY(launch_train(p->pde, l.wpmax, p->ga, p->recompute, ka, grid, side && g > 0 ? p->side_stream : st));
    }
    if (side) {
      HIP_TRY(hipEventRecord(p->ev_join, p->side_stream));
      HIP_TRY(hipStreamWaitEvent(st, p->ev_join, 0));
    }
    RArgs ra = make_rargs(p);
    reduce_range(p, ra, 0, n_sd);
    ra.grad_out = grad_out;
    ra.loss_out = loss_out;
    ra.do_adam = do_adam;
    ra.counter_reset = b ? nullptr : p->d_counters;
    ra.n_counter_reset = b ? 0 : (int)p->launches.size();
    HIP_TRY(launch_reduce(ra, reduce_grid(p, 0, n_sd), st));
    return DDP_OK;
  }
  // plain path: the same kernels, one launch pair per subdomain; every
  // subdomain's loss and gradient use the parameters from before the step
  for (int q = 0; q < n_sd; ++q) {
    KArgs ka = make_kargs(p);
    ka.items = p->d_titems + p->t_begin[q];
    ka.n_items = p->t_begin[q + 1] - p->t_begin[q];
    ka.counter = counters + p->launches.size() + q;
    ka.scratch = scratch;
    ka.prologue = q == 0;
    if (ka.n_items == 0 && q != 0) continue;
    const int grid = std::max(1, std::min(slots_for(p->n_slots, p->slot_floats), ka.n_items));
    HIP_TRY(launch_train(p->pde, p->wpmax, p->ga, p->recompute, ka, grid, st));
  }
  for (int q = 0; q < n_sd; ++q) {
    RArgs ra = make_rargs(p);
    reduce_range(p, ra, q, q + 1);
    ra.grad_out = grad_out;
    ra.loss_out = loss_out;
    ra.do_adam = do_adam;
    ra.counter_reset = b ? nullptr : p->d_counters + p->launches.size() + q;
    ra.n_counter_reset = b ? 0 : 1;
    HIP_TRY(launch_reduce(ra, reduce_grid(p, q, q + 1), st));
  }
  return DDP_OK;
}

void release(ddp_problem* p) {
  if (p->graph_exec) hipGraphExecDestroy(p->graph_exec);
  if (p->graph) hipGraphDestroy(p->graph);
  p->graph_exec = nullptr;
  p->graph = nullptr;
  for (void* a : p->allocations) hipFree(a);
  p->allocations.clear();
  for (void* a : p->plan_allocations) hipFree(a);
  p->plan_allocations.clear();
  if (p->cap_stream) hipStreamDestroy(p->cap_stream);
  p->cap_stream = nullptr;
  if (p->side_stream) hipStreamDestroy(p->side_stream);
  p->side_stream = nullptr;
  if (p->ev_fork) hipEventDestroy(p->ev_fork);
  if (p->ev_join) hipEventDestroy(p->ev_join);
  p->ev_fork = p->ev_join = nullptr;
}

int check_open(const ddp_problem* p) {
  if (!p) return fail(DDP_EINVAL, "null problem handle");
  if (p->finalized) return fail(DDP_ESTATE, "topology is fixed after ddp_finalize");
  return DDP_OK;
}

int check_final(const ddp_problem* p) {
  if (!p) return fail(DDP_EINVAL, "null problem handle");
  if (!p->finalized) return fail(DDP_ESTATE, "call ddp_finalize first");
  if (!p->plan_ok) return fail(DDP_ESTATE, "no work plan is installed (a failed re-plan could not restore it)");
  return DDP_OK;
}

void json_ints(FILE* f, const char* name, const std::vector<int>& v) {
  std::fprintf(f, "\"%s\": [", name);
  for (size_t i = 0; i < v.size(); ++i) std::fprintf(f, "%s%d", i ? ", " : "", v[i]);
  std::fprintf(f, "]");
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI

extern "C" {

const char* ddp_last_error(void) { return g_err.c_str(); }

int ddp_create(ddp_problem** out, int method, int pde, const double* coef, int n_coef) {
  if (!out) return fail(DDP_EINVAL, "null output pointer");
  *out = nullptr;
  if (method != DDP_CPINN && method != DDP_XPINN) return fail(DDP_EINVAL, "method must be DDP_CPINN or DDP_XPINN");
  if (pde < DDP_POISSON2D || pde > DDP_DIFFUSION2D_INV) return fail(DDP_EINVAL, "unknown operator");
  if (n_coef < 0 || n_coef > 4 || (n_coef > 0 && !coef)) return fail(DDP_EINVAL, "bad coefficient array");
  if ((pde == DDP_BURGERS1D || pde == DDP_NS2D_STEADY) && n_coef < 1)
    return fail(DDP_EINVAL, "operator needs coef[0] (nu or Re)");
  for (int i = 0; i < n_coef; ++i)
    if (!std::isfinite(coef[i]) || coef[i] <= 0) return fail(DDP_EINVAL, "coefficients must be finite and > 0");
  if (method == DDP_CPINN && pde == DDP_DIFFUSION2D_INV)
    return fail(DDP_EINVAL, "the inverse diffusion problem uses XPINN interfaces");
  ddp_problem* p = new (std::nothrow) ddp_problem();
  if (!p) return fail(DDP_ENOMEM, "out of host memory");
  p->method = method;
  p->pde = pde;
  for (int i = 0; i < n_coef; ++i) p->coef[i] = coef[i];
  p->d_out = pde == DDP_NS2D_STEADY ? 3 : 1;
  p->n_eq = pde == DDP_NS2D_STEADY ? 3 : 1;
  *out = p;
  return DDP_OK;
}

namespace {
int check_widths(const int* widths, int nl, int d_out) {
  if (nl < 3) return fail(DDP_EINVAL, "a network needs input, at least one hidden and an output layer");
  if (nl - 2 > kMaxDepth) return fail(DDP_EINVAL, "at most 8 hidden layers");
  if (widths[0] != 2) return fail(DDP_EINVAL, "input width must be 2");
  if (widths[nl - 1] != d_out) return fail(DDP_EINVAL, "output width must equal the operator's outputs");
  const int w = widths[1];
  if (w < 1 || w > kMaxWidth) return fail(DDP_EINVAL, "hidden width must be in [1, 112]");
  for (int k = 1; k < nl - 1; ++k)
    if (widths[k] != w) return fail(DDP_EINVAL, "hidden layers of one network must have equal widths");
  return DDP_OK;
}
}  // namespace

int ddp_add_subdomain(ddp_problem* p, int n_nets, const int* n_layers, const int* widths, const float* loss_w,
                      float lr, int* sd_id) {
  if (int rc = check_open(p)) return rc;
  const int need = p->pde == DDP_DIFFUSION2D_INV ? 2 : 1;
  if (n_nets != need)
    return fail(DDP_EINVAL, need == 2 ? "the inverse diffusion problem needs two networks (u, K) per subdomain"
                                      : "this operator takes one network per subdomain");
  if (!n_layers || !widths || !loss_w) return fail(DDP_EINVAL, "null argument");
  const int nl = n_layers[0];
  if (int rc = check_widths(widths, nl, p->d_out)) return rc;
  if (n_nets == 2)
    if (int rc = check_widths(widths + nl, n_layers[1], 1)) return rc;
  for (int k = 0; k < 4; ++k)
    if (!std::isfinite(loss_w[k]) || loss_w[k] < 0) return fail(DDP_EINVAL, "loss weights must be finite and >= 0");
  if (!std::isfinite(lr) || lr <= 0) return fail(DDP_EINVAL, "learning rate must be finite and > 0");
  HostSd s;
  s.widths.assign(widths, widths + nl);
  if (n_nets == 2) s.aux_widths.assign(widths + nl, widths + nl + n_layers[1]);
  for (int k = 0; k < 4; ++k) s.loss_w[k] = loss_w[k];
  s.lr = lr;
  p->sds.push_back(std::move(s));
  if (sd_id) *sd_id = (int)p->sds.size() - 1;
  p->planned = false;
  return DDP_OK;
}

int ddp_set_points(ddp_problem* p, int sd, int kind, int n, const float* xy, const float* val, int on_device) {
  if (int rc = check_open(p)) return rc;
  if (sd < 0 || sd >= (int)p->sds.size()) return fail(DDP_EINVAL, "unknown subdomain");
  if (kind != DDP_RESIDUAL && kind != DDP_DATA && kind != DDP_DATA_AUX) return fail(DDP_EINVAL, "unknown point kind");
  if (kind == DDP_DATA_AUX && p->pde != DDP_DIFFUSION2D_INV)
    return fail(DDP_EINVAL, "DDP_DATA_AUX points belong to the inverse diffusion problem");
  if (n < 0) return fail(DDP_EINVAL, "negative point count");
  HostSd& s = p->sds[sd];
  const int nv = kind == DDP_RESIDUAL ? p->n_eq : (kind == DDP_DATA ? p->d_out : 1);
  std::vector<float> hxy, hval;
  if (int rc = copy_in(xy, (size_t)n * 2, on_device, hxy)) return rc;
  if (int rc = copy_in(val, (size_t)n * nv, on_device, hval)) return rc;
  if (!all_finite(hxy.data(), hxy.size()) || !all_finite(hval.data(), hval.size()))
    return fail(DDP_EINVAL, "non-finite coordinate or value");
  if (kind == DDP_RESIDUAL) {
    s.res_xy.swap(hxy);
    s.res_f.swap(hval);
    s.n_res = n;
  } else if (kind == DDP_DATA_AUX) {
    s.aux_xy.swap(hxy);
    s.aux_g.swap(hval);
    s.n_aux = n;
  } else {
    s.dat_xy.swap(hxy);
    s.dat_g.swap(hval);
    s.n_dat = n;
  }
  p->planned = false;
  return DDP_OK;
}

int ddp_add_interface(ddp_problem* p, int sd_a, int sd_b, int n, const float* xy, const float normal[2],
                      int on_device, int* if_id) {
  if (int rc = check_open(p)) return rc;
  const int n_sd = (int)p->sds.size();
  if (sd_a < 0 || sd_b < 0 || sd_a >= n_sd || sd_b >= n_sd) return fail(DDP_EINVAL, "interface names an unknown subdomain");
  if (sd_a == sd_b) return fail(DDP_EINVAL, "interface needs two different subdomains");
  if (n < 0) return fail(DDP_EINVAL, "negative point count");
  if (!normal || !std::isfinite(normal[0]) || !std::isfinite(normal[1])) return fail(DDP_EINVAL, "bad normal");
  HostIf f;
  f.a = sd_a;
  f.b = sd_b;
  f.n = n;
  f.nx = normal[0];
  f.ny = normal[1];
  if (int rc = copy_in(xy, (size_t)n * 2, on_device, f.xy)) return rc;
  if (!all_finite(f.xy.data(), f.xy.size())) return fail(DDP_EINVAL, "non-finite coordinate");
  p->ifs.push_back(std::move(f));
  if (if_id) *if_id = (int)p->ifs.size() - 1;
  p->planned = false;
  return DDP_OK;
}

static_assert(DDP_ACT_TANH == ACT_TANH && DDP_ACT_SIN == ACT_SIN && DDP_ACT_COS == ACT_COS,
              "activation codes of the ABI and the kernels agree");

int ddp_set_activation(ddp_problem* p, int sd, int act, int adaptive, float slope_n) {
  if (int rc = check_open(p)) return rc;
  if (sd < 0 || sd >= (int)p->sds.size()) return fail(DDP_EINVAL, "unknown subdomain");
  if (act != DDP_ACT_TANH && act != DDP_ACT_SIN && act != DDP_ACT_COS) return fail(DDP_EINVAL, "unknown activation");
  if (adaptive != 0 && adaptive != 1) return fail(DDP_EINVAL, "adaptive must be 0 or 1");
  if (!std::isfinite(slope_n) || slope_n <= 0.f) return fail(DDP_EINVAL, "slope scale must be finite and > 0");
  HostSd& s = p->sds[sd];
  s.act = act;
  s.adaptive = adaptive;
  s.slope_n = slope_n;
  p->planned = false;
  return DDP_OK;
}

int ddp_set_interface_method(ddp_problem* p, int if_id, int method) {
  if (int rc = check_open(p)) return rc;
  if (if_id < 0 || if_id >= (int)p->ifs.size()) return fail(DDP_EINVAL, "unknown interface");
  if (method != DDP_CPINN && method != DDP_XPINN) return fail(DDP_EINVAL, "method must be DDP_CPINN or DDP_XPINN");
  if (method == DDP_CPINN && p->pde == DDP_DIFFUSION2D_INV)
    return fail(DDP_EINVAL, "the inverse diffusion problem uses XPINN interfaces");
  p->ifs[if_id].method = method;
  p->planned = false;
  return DDP_OK;
}

int ddp_set_option(ddp_problem* p, int option, int64_t value) {
  if (int rc = check_open(p)) return rc;
  switch (option) {
    case DDP_OPT_CHUNK_POINTS:
      if (value < 1 || value > (1 << 24)) return fail(DDP_EINVAL, "chunk points out of range");
      p->chunk_points = value;
      break;
    case DDP_OPT_BLOCKS_PER_CU:
      if (value < 0 || value > 8) return fail(DDP_EINVAL, "blocks per CU out of range");
      p->blocks_per_cu = (int)value;
      break;
    case DDP_OPT_ITEMS_PER_SLOT:
      if (value < 1 || value > 64) return fail(DDP_EINVAL, "items per slot out of range");
      p->items_per_slot = (int)value;
      break;
    case DDP_OPT_RECOMPUTE:
      if (value != 0 && value != 1) return fail(DDP_EINVAL, "recompute must be 0 or 1");
      p->recompute = (int)value;
      break;
    case DDP_OPT_CONCURRENT:
      if (value != 0 && value != 1) return fail(DDP_EINVAL, "concurrent must be 0 or 1");
      p->concurrent = (int)value;
      break;
    case DDP_OPT_TAIL:
      if (value < 0 || value > 100) return fail(DDP_EINVAL, "tail share must be 0..100 percent");
      p->tail_pct = (int)value;
      break;
    default:
      return fail(DDP_EINVAL, "unknown option");
  }
  p->planned = false;
  return DDP_OK;
}

int ddp_plan(ddp_problem* p) {
  if (int rc = check_open(p)) return rc;
  return build_plan(p);
}

}  // extern "C"

namespace {

// Build the work plan for the current options and (re)create everything that
// depends on it: work items, gradient / loss partial rows, row lists, the
// activation stash, work counters and the step graph.
int install_plan(ddp_problem* p) {
  const int n_sd = (int)p->sds.size();
  p->plan_ok = false;
  if (p->graph_exec) hipGraphExecDestroy(p->graph_exec);
  if (p->graph) hipGraphDestroy(p->graph);
  p->graph_exec = nullptr;
  p->graph = nullptr;
  if (p->stream) HIP_TRY(hipStreamSynchronize(p->stream));
  for (void* a : p->plan_allocations) hipFree(a);
  p->plan_allocations.clear();
  HIP_TRY(train_occupancy(p->pde, p->wpmax, p->ga, p->recompute, &p->occupancy));
  if (p->occupancy < 1) return fail(DDP_EHIP, "train kernel cannot be resident (occupancy 0)");
  const int bpc = p->blocks_per_cu > 0 ? std::min(p->blocks_per_cu, p->occupancy) : p->occupancy;
  p->n_slots = std::max(1, p->n_cu * bpc);
  p->plan_slots = p->n_slots;
  if (int rc = build_plan(p)) return rc;
  p->slot_floats = scratch_slot_floats(p->pde, p->wpmax, p->recompute);
  int64_t scratch_floats = (int64_t)p->n_slots * p->slot_floats;
  // sequential launches reuse one stash region; concurrent ones get their own
  const bool side = p->fused && p->concurrent && p->launches.size() > 1;
  int64_t side_floats = 0;
  for (ddp_problem::Launch& l : p->launches) {
    HIP_TRY(train_occupancy(p->pde, l.wpmax, p->ga, p->recompute, &l.occupancy));
    if (l.occupancy < 1) return fail(DDP_EHIP, "train kernel cannot be resident (occupancy 0)");
    const int b = p->blocks_per_cu > 0 ? std::min(p->blocks_per_cu, l.occupancy) : l.occupancy;
    l.n_slots = std::max(1, p->n_cu * b);
    l.slot_floats = scratch_slot_floats(p->pde, l.wpmax, p->recompute);
    l.scratch_off = side ? side_floats : 0;
    side_floats += (int64_t)l.n_slots * l.slot_floats;
    scratch_floats = std::max(scratch_floats, (int64_t)l.n_slots * l.slot_floats);
  }
  if (side) {
    scratch_floats = std::max(scratch_floats, side_floats);
    if (!p->side_stream) HIP_TRY(hipStreamCreateWithFlags(&p->side_stream, hipStreamNonBlocking));
    if (!p->ev_fork) HIP_TRY(hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming));
    if (!p->ev_join) HIP_TRY(hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming));
  }
  // counters: one per fused launch, then one per subdomain (plain path)
  p->n_counters = (int)p->launches.size() + n_sd;
  int rc = 0;
  if ((rc = plan_upload(p, &p->d_counters, std::vector<int>(p->n_counters, 0)))) return rc;
  if ((rc = plan_upload(p, &p->d_titems, p->titems))) return rc;
  if ((rc = plan_alloc(p, &p->d_partial, (size_t)p->partial_floats))) return rc;
  if ((rc = plan_alloc(p, &p->d_loss_part, p->titems.size() * kLossTerms))) return rc;
  if ((rc = plan_alloc(p, &p->d_scratch, (size_t)scratch_floats))) return rc;
  if ((rc = plan_upload(p, &p->d_net_row_ptr, p->net_row_ptr))) return rc;
  if ((rc = plan_upload(p, &p->d_row_prow, p->row_prow))) return rc;
  if ((rc = plan_upload(p, &p->d_sd_loss_ptr, p->sd_loss_ptr))) return rc;
  if ((rc = plan_upload(p, &p->d_loss_rows, p->loss_rows))) return rc;
  HIP_TRY(hipMemset(p->d_partial, 0, (size_t)std::max<int64_t>(1, p->partial_floats) * sizeof(float)));
  HIP_TRY(hipMemset(p->d_loss_part, 0, std::max<size_t>(1, p->titems.size() * kLossTerms) * sizeof(float)));
  HIP_TRY(hipDeviceSynchronize());
  if (p->fused) {
    // one training step as a graph: captured on a private stream, replayed on
    // the caller's stream
    if (!p->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
    rc = enqueue_step(p, p->cap_stream, 1, nullptr, p->d_loss);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(p->cap_stream, &g);
    if (rc) {
      if (g) hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return fail(DDP_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    p->graph = g;
    HIP_TRY(hipGraphInstantiate(&p->graph_exec, p->graph, nullptr, nullptr, 0));
  }
  p->plan_ok = true;
  return DDP_OK;
}

// FNV-1a hash of everything the best plan depends on
uint64_t problem_signature(const ddp_problem* p) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](int64_t v) {
    for (int b = 0; b < 8; ++b) {
      h ^= (uint64_t)((v >> (8 * b)) & 0xff);
      h *= 1099511628211ull;
    }
  };
  mix(p->pde);
  mix(p->method);
  mix(p->fused);
  mix(p->n_cu);
  mix((int64_t)p->sds.size());
  for (const HostSd& s : p->sds) {
    for (int w : s.widths) mix(w);
    for (int w : s.aux_widths) mix(w);
    mix(s.act);
    mix(s.adaptive);
    mix(s.n_res);
    mix(s.n_dat);
    mix(s.n_aux);
  }
  for (const HostIf& f : p->ifs) {
    mix(f.a);
    mix(f.b);
    mix(f.n);
    mix(f.method >= 0 ? f.method : p->method);
  }
  return h;
}

bool cache_lookup(const char* path, uint64_t sig, int64_t* cfg) {
  if (!path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[512];
  bool found = false;
  while (std::fgets(line, sizeof line, f)) {
    unsigned long long s = 0;
    long long c = 0, ips = 0, bpc = 0, rh = 0, conc = 0, tail = 0;
    if (std::sscanf(line, "{\"signature\": \"%llx\", \"chunk_points\": %lld, \"items_per_slot\": %lld, "
                          "\"blocks_per_cu\": %lld, \"recompute\": %lld, \"concurrent\": %lld, \"tail\": %lld",
                    &s, &c, &ips, &bpc, &rh, &conc, &tail) == 7 &&
        s == sig) {
      cfg[0] = c;
      cfg[1] = ips;
      cfg[2] = bpc;
      cfg[3] = rh;
      cfg[4] = conc;
      cfg[5] = tail;
      found = true;  // the last entry for a signature wins
    }
  }
  std::fclose(f);
  return found;
}

}  // namespace

extern "C" {

int ddp_finalize(ddp_problem* p, void* hip_stream, int fused) {
  if (int rc = check_open(p)) return rc;
  p->fused = fused ? 1 : 0;
  if (int rc = build_plan(p)) return rc;  // validates and fixes wpmax
  const int n_sd = (int)p->sds.size();
  HIP_TRY(hipGetDevice(&p->device));
  p->stream = static_cast<hipStream_t>(hip_stream);
  HIP_TRY(hipDeviceGetAttribute(&p->n_cu, hipDeviceAttributeMultiprocessorCount, p->device));
  HIP_TRY(train_occupancy(p->pde, p->wpmax, p->ga, p->recompute, &p->occupancy));
  if (p->occupancy < 1) return fail(DDP_EHIP, "train kernel cannot be resident (occupancy 0)");

  int rc = 0;
  std::vector<float> zeros(p->sd_poff[n_sd], 0.f);
  if ((rc = dev_upload(p, &p->d_params, zeros))) return rc;
  if ((rc = dev_upload(p, &p->d_m, zeros))) return rc;
  if ((rc = dev_upload(p, &p->d_v, zeros))) return rc;
  if ((rc = dev_upload(p, &p->d_kparams, std::vector<float>((size_t)p->kparam_floats, 0.f)))) return rc;
  if ((rc = dev_upload(p, &p->d_tstate, std::vector<int>{0, 0}))) return rc;
  if ((rc = dev_upload(p, &p->d_flags, std::vector<int>{0, 0}))) return rc;
  if ((rc = dev_upload(p, &p->d_nets, p->nets))) return rc;
  if ((rc = dev_upload(p, &p->d_ifaces, p->ifaces))) return rc;
  if ((rc = dev_upload(p, &p->d_res_xy, p->h_res_xy))) return rc;
  if ((rc = dev_upload(p, &p->d_res_f, p->h_res_f))) return rc;
  if ((rc = dev_upload(p, &p->d_dat_xy, p->h_dat_xy))) return rc;
  if ((rc = dev_upload(p, &p->d_dat_g, p->h_dat_g))) return rc;
  if ((rc = dev_upload(p, &p->d_if_xy, p->h_if_xy))) return rc;
  if ((rc = dev_upload(p, &p->d_aux_xy, p->h_aux_xy))) return rc;
  if ((rc = dev_upload(p, &p->d_aux_g, p->h_aux_g))) return rc;
  if ((rc = dev_alloc(p, &p->d_loss, (size_t)n_sd * 5))) return rc;
  if ((rc = dev_upload(p, &p->d_net_poff, p->net_poff))) return rc;
  if ((rc = dev_upload(p, &p->d_net_blk, p->net_blk))) return rc;
  if ((rc = dev_upload(p, &p->d_blk_net, p->blk_net))) return rc;
  if ((rc = dev_upload(p, &p->d_sd_net, p->sd_net))) return rc;
  if ((rc = install_plan(p))) return rc;
  p->finalized = true;
  return DDP_OK;
}

namespace {

// The autotuner's search: every candidate plan timed over iters passes, the
// three fastest again over three interleaved rounds; best receives the
// winner.  Leaves the last candidate installed.
int autotune_search(ddp_problem* p, int iters, hipEvent_t* ev, int64_t* best, float* best_ms) {
  const int64_t chunks[] = {256, 512, 1024, 2048};
  const int ipss[] = {1, 2, 4, 8};
  struct Cand {
    int64_t c;
    int ips, bpc, rh, conc, tail;
    float ms;
  };
  std::vector<Cand> cands;
  // mean time of one loss + gradient pass (no Adam) of candidate k over n
  // passes, after one untimed pass
  auto time_cand = [&](const Cand& k, int n, float* ms) -> int {
    p->chunk_points = k.c;
    p->items_per_slot = k.ips;
    p->blocks_per_cu = k.bpc;
    p->recompute = k.rh;
    p->concurrent = k.conc;
    p->tail_pct = k.tail;
    if (int rc = install_plan(p)) return rc;
    if (int rc = enqueue_step(p, p->stream, 0, nullptr, p->d_loss)) return rc;
    HIP_TRY(hipEventRecord(ev[0], p->stream));
    for (int i = 0; i < n; ++i)
      if (int rc = enqueue_step(p, p->stream, 0, nullptr, p->d_loss)) return rc;
    HIP_TRY(hipEventRecord(ev[1], p->stream));
    HIP_TRY(hipEventSynchronize(ev[1]));
    HIP_TRY(hipEventElapsedTime(ms, ev[0], ev[1]));
    *ms /= n;
    return DDP_OK;
  };
  for (int rh = 0; rh <= 1; ++rh) {
    // resident workgroups per CU of this policy's kernels (the fused
    // launches may run narrower kernels than the per-subdomain path)
    p->recompute = rh;
    p->concurrent = 0;
    p->tail_pct = 0;
    if (int rc = install_plan(p)) return rc;
    int max_occ = p->occupancy;
    for (const ddp_problem::Launch& l : p->launches) max_occ = std::max(max_occ, l.occupancy);
    // side-by-side launches only where the step has more than one
    const int max_conc = p->fused && p->launches.size() > 1 ? 1 : 0;
    // a tail share of one-tile items only on the fused path
    const int tails[2] = {0, 30};
    const int n_tails = p->fused ? 2 : 1;
    for (int conc = 0; conc <= max_conc; ++conc)
      for (int t = 0; t < n_tails; ++t)
        for (int64_t c : chunks)
          for (int ips : ipss)
            for (int bpc = 1; bpc <= max_occ; ++bpc) {
              Cand k{c, ips, bpc, rh, conc, tails[t], 0.f};
              if (int rc = time_cand(k, iters, &k.ms)) return rc;
              cands.push_back(k);
            }
  }
  // the leading candidates are often within a percent of each other: time the
  // best three again, interleaved over three rounds of 2 x iters passes, and
  // keep the smallest total
  std::stable_sort(cands.begin(), cands.end(), [](const Cand& x, const Cand& y) { return x.ms < y.ms; });
  const int n_final = std::min<int>(3, (int)cands.size());
  std::vector<float> total(n_final, 0.f);
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < n_final; ++k) {
      float ms = 0.f;
      if (int rc = time_cand(cands[k], 2 * iters, &ms)) return rc;
      total[k] += ms;
    }
  *best_ms = 1e30f;
  for (int k = 0; k < n_final; ++k)
    if (total[k] / 3 < *best_ms) {
      *best_ms = total[k] / 3;
      best[0] = cands[k].c;
      best[1] = cands[k].ips;
      best[2] = cands[k].bpc;
      best[3] = cands[k].rh;
      best[4] = cands[k].conc;
      best[5] = cands[k].tail;
    }
  return DDP_OK;
}

}  // namespace

int ddp_autotune(ddp_problem* p, int iters, const char* cache_path, int64_t* choice) {
  if (int rc = check_final(p)) return rc;
  if (iters < 1) return fail(DDP_EINVAL, "iters must be >= 1");
  const uint64_t sig = problem_signature(p);
  const int64_t prev[6] = {p->chunk_points, p->items_per_slot, p->blocks_per_cu,
                           p->recompute,   p->concurrent,     p->tail_pct};
  int64_t best[6] = {prev[0], prev[1], prev[2], prev[3], prev[4], prev[5]};
  auto apply = [&](const int64_t* v) {
    p->chunk_points = v[0];
    p->items_per_slot = (int)v[1];
    p->blocks_per_cu = (int)v[2];
    p->recompute = (int)v[3];
    p->concurrent = (int)v[4];
    p->tail_pct = (int)v[5];
  };
  // on any failure the previous plan is put back, so the handle stays usable;
  // if even that fails, every later call reports DDP_ESTATE
  auto restore = [&](int rc) {
    const std::string msg = g_err;
    apply(prev);
    install_plan(p);
    g_err = msg;
    return rc;
  };
  if (!cache_lookup(cache_path, sig, best)) {
    hipEvent_t ev[2] = {nullptr, nullptr};
    float best_ms = 0.f;
    int rc = DDP_OK;
    hipError_t e = hipEventCreate(&ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&ev[1]);
    if (e != hipSuccess) rc = fail(DDP_EHIP, std::string("hipEventCreate: ") + hipGetErrorString(e));
    if (rc == DDP_OK) rc = autotune_search(p, iters, ev, best, &best_ms);
    if (ev[0]) hipEventDestroy(ev[0]);
    if (ev[1]) hipEventDestroy(ev[1]);
    if (rc) return restore(rc);
    if (cache_path) {
      FILE* f = std::fopen(cache_path, "a");
      if (f) {
        std::fprintf(f,
                     "{\"signature\": \"%016llx\", \"chunk_points\": %lld, \"items_per_slot\": %lld, "
                     "\"blocks_per_cu\": %lld, \"recompute\": %lld, \"concurrent\": %lld, \"tail\": %lld, "
                     "\"ms\": %.5f}\n",
                     (unsigned long long)sig, (long long)best[0], (long long)best[1], (long long)best[2],
                     (long long)best[3], (long long)best[4], (long long)best[5], best_ms);
        std::fclose(f);
      }
    }
  }
  apply(best);
  if (int rc = install_plan(p)) return restore(rc);
  if (choice)
    for (int k = 0; k < 6; ++k) choice[k] = best[k];
  return DDP_OK;
}

int ddp_param_count(const ddp_problem* p, int sd, int64_t* n) {
  if (!p || !n) return fail(DDP_EINVAL, "null argument");
  if (sd < 0 || sd >= (int)p->sds.size()) return fail(DDP_EINVAL, "unknown subdomain");
  const HostSd& s = p->sds[sd];
  *n = net_param_count(s.widths, s.adaptive) + (s.aux_widths.empty() ? 0 : net_param_count(s.aux_widths, s.adaptive));
  return DDP_OK;
}

int ddp_set_params(ddp_problem* p, int sd, const float* flat, int on_device) {
  if (int rc = check_final(p)) return rc;
  if (sd < 0 || sd >= (int)p->sds.size() || !flat) return fail(DDP_EINVAL, "bad subdomain or null pointer");
  const size_t n = (size_t)(p->sd_poff[sd + 1] - p->sd_poff[sd]);
  HIP_TRY(hipMemcpyAsync(p->d_params + p->sd_poff[sd], flat, n * sizeof(float),
                         on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, p->stream));
  HIP_TRY(launch_pack(p->d_params, p->d_kparams, p->d_nets, p->d_net_poff, p->sd_net[sd], p->sd_net[sd + 1],
                      (int64_t)n, p->stream));
  if (!on_device) HIP_TRY(hipStreamSynchronize(p->stream));
  return DDP_OK;
}

int ddp_get_params(ddp_problem* p, int sd, float* flat, int on_device) {
  if (int rc = check_final(p)) return rc;
  if (sd < 0 || sd >= (int)p->sds.size() || !flat) return fail(DDP_EINVAL, "bad subdomain or null pointer");
  const size_t n = (size_t)(p->sd_poff[sd + 1] - p->sd_poff[sd]);
  HIP_TRY(hipMemcpyAsync(flat, p->d_params + p->sd_poff[sd], n * sizeof(float),
                         on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, p->stream));
  if (!on_device) HIP_TRY(hipStreamSynchronize(p->stream));
  return DDP_OK;
}

int ddp_loss_and_grad(ddp_problem* p, float* loss_terms, float* grad) {
  if (int rc = check_final(p)) return rc;
  return enqueue_step(p, p->stream, 0, grad, loss_terms ? loss_terms : p->d_loss);
}

int ddp_loss_and_grad_static(ddp_problem* p, float* loss_terms, float* grad) {
  if (int rc = check_final(p)) return rc;
  int cur = -1;
  HIP_TRY(hipGetDevice(&cur));
  if (cur != p->device) return fail(DDP_ESTATE, "make the problem's device current before this call");
  if ((size_t)p->n_counters * sizeof(int) > kStaticCounterBytes)
    return fail(DDP_EINVAL, "the per-subdomain path of this problem needs " + std::to_string(p->n_counters) +
                                " work counters; the static scratch holds " +
                                std::to_string(kStaticCounterBytes / sizeof(int)));
  int64_t slot = p->fused ? 0 : p->slot_floats;
  for (const ddp_problem::Launch& l : p->launches) slot = std::max(slot, l.slot_floats);
  const int64_t cap = (int64_t)((kStaticScratchBytes - kStaticCounterBytes) / sizeof(float));
  if (slot > cap)
    return fail(DDP_EINVAL, "one workgroup's activation stash (" + std::to_string(slot * 4) +
                                " bytes) exceeds the static scratch (" + std::to_string(cap * 4) + " bytes)");
  void* base = nullptr;
  HIP_TRY(static_scratch(p->device, &base));
  const StepBufs b{reinterpret_cast<float*>(static_cast<char*>(base) + kStaticCounterBytes), cap,
                   static_cast<int*>(base)};
  return enqueue_step(p, p->stream, 0, grad, loss_terms ? loss_terms : p->d_loss, &b);
}

int ddp_step(ddp_problem* p, int n_steps, float* loss_terms) {
  if (int rc = check_final(p)) return rc;
  if (n_steps < 0) return fail(DDP_EINVAL, "negative step count");
  for (int s = 0; s < n_steps; ++s) {
    if (p->fused) {
      HIP_TRY(hipGraphLaunch(p->graph_exec, p->stream));
    } else {
      if (int rc = enqueue_step(p, p->stream, 1, nullptr, p->d_loss)) return rc;
    }
  }
  if (loss_terms && n_steps > 0)
    HIP_TRY(hipMemcpyAsync(loss_terms, p->d_loss, p->sds.size() * 5 * sizeof(float), hipMemcpyDeviceToDevice,
                           p->stream));
  return DDP_OK;
}

int ddp_get_state(ddp_problem* p, float* m, float* v, int64_t* t) {
  if (int rc = check_final(p)) return rc;
  const size_t n = (size_t)p->sd_poff.back();
  HIP_TRY(hipStreamSynchronize(p->stream));
  if (m) HIP_TRY(hipMemcpy(m, p->d_m, n * sizeof(float), hipMemcpyDeviceToHost));
  if (v) HIP_TRY(hipMemcpy(v, p->d_v, n * sizeof(float), hipMemcpyDeviceToHost));
  if (t) {
    int ts[2];
    HIP_TRY(hipMemcpy(ts, p->d_tstate, sizeof(ts), hipMemcpyDeviceToHost));
    *t = (int64_t)ts[0] + ts[1];
  }
  return DDP_OK;
}

int ddp_set_state(ddp_problem* p, const float* m, const float* v, int64_t t) {
  if (int rc = check_final(p)) return rc;
  if (t < 0 || t > (1 << 30)) return fail(DDP_EINVAL, "step count out of range");
  const size_t n = (size_t)p->sd_poff.back();
  HIP_TRY(hipStreamSynchronize(p->stream));
  if (m) HIP_TRY(hipMemcpy(p->d_m, m, n * sizeof(float), hipMemcpyHostToDevice));
  if (v) HIP_TRY(hipMemcpy(p->d_v, v, n * sizeof(float), hipMemcpyHostToDevice));
  int ts[2] = {(int)t, 0};
  HIP_TRY(hipMemcpy(p->d_tstate, ts, sizeof(ts), hipMemcpyHostToDevice));
  return DDP_OK;
}

int ddp_eval(ddp_problem* p, int n, const float* xy, const int* owner, float* u_out) {
  if (int rc = check_final(p)) return rc;
  if (n < 0 || (n > 0 && (!xy || !owner || !u_out))) return fail(DDP_EINVAL, "bad evaluation arguments");
  const int n_cols = p->d_out + (p->pde == DDP_DIFFUSION2D_INV ? 1 : 0);
  HIP_TRY(launch_eval(p->d_params, p->d_nets, p->d_sd_net, (int)p->sds.size(), n, xy, owner, u_out, n_cols,
                      p->stream));
  return DDP_OK;
}

int ddp_sync(ddp_problem* p) {
  if (int rc = check_final(p)) return rc;
  HIP_TRY(hipStreamSynchronize(p->stream));
  int flags[2];
  HIP_TRY(hipMemcpy(flags, p->d_flags, sizeof(flags), hipMemcpyDeviceToHost));
  if (flags[0]) {
    int zero[2] = {0, 0};
    HIP_TRY(hipMemcpy(p->d_flags, zero, sizeof(zero), hipMemcpyHostToDevice));
    return fail(DDP_ENONFINITE, "a loss was NaN or inf");
  }
  return DDP_OK;
}

int ddp_mfma_probe(int iters, double* tflops) {
  if (iters < 1 || iters > (1 << 20) || !tflops) return fail(DDP_EINVAL, "bad probe arguments");
  HIP_TRY(mfma_probe(iters, tflops));
  return DDP_OK;
}

int ddp_time_kernels(ddp_problem* p, int iters, float* ms) {
  if (int rc = check_final(p)) return rc;
  if (iters < 1 || !ms) return fail(DDP_EINVAL, "bad timing arguments");
  const int n_sd = (int)p->sds.size();
  hipEvent_t ev[2];
  HIP_TRY(hipEventCreate(&ev[0]));
  HIP_TRY(hipEventCreate(&ev[1]));
  // [0]: every train launch of one step, [1]: reduction without Adam
  for (int which = 0; which < 2; ++which) {
    float total = 0.f;
    for (int i = 0; i < iters; ++i) {
      if (which == 0)
        for (int c = 0; c < p->n_counters; ++c) HIP_TRY(launch_reset_counter(p->d_counters + c, p->stream));
      HIP_TRY(hipEventRecord(ev[0], p->stream));
      if (which == 0) {
        // as in the step: concurrent launches fork onto the side stream
        const bool side = p->fused && p->concurrent && p->launches.size() > 1;
        if (side) {
          HIP_TRY(hipEventRecord(p->ev_fork, p->stream));
          HIP_TRY(hipStreamWaitEvent(p->side_stream, p->ev_fork, 0));
        }
        const int nl = p->fused ? (int)p->launches.size() : n_sd;
        for (int q = 0; q < nl; ++q) {
          KArgs ka = make_kargs(p);
          int wpmax = p->wpmax, n_slots = p->n_slots;
          hipStream_t st = p->stream;
          if (p->fused) {
            const ddp_problem::Launch& l = p->launches[q];
            ka.items = p->d_titems + l.begin;
            ka.n_items = l.count;
            ka.counter = p->d_counters + q;
            ka.scratch += l.scratch_off;
            ka.scratch_slot = l.slot_floats;
            wpmax = l.wpmax;
            n_slots = l.n_slots;
            if (side && q > 0) st = p->side_stream;
          } else {
            ka.items = p->d_titems + p->t_begin[q];
            ka.n_items = p->t_begin[q + 1] - p->t_begin[q];
            ka.counter = p->d_counters + p->launches.size() + q;
          }
          if (ka.n_items == 0) continue;
          const int grid = std::max(1, std::min(n_slots, ka.n_items));
          HIP_TRY(launch_train(p->pde, wpmax, p->ga, p->recompute, ka, grid, st));
        }
        if (side) {
          HIP_TRY(hipEventRecord(p->ev_join, p->side_stream));
          HIP_TRY(hipStreamWaitEvent(p->stream, p->ev_join, 0));
        }
      } else {
        RArgs ra = make_rargs(p);
        reduce_range(p, ra, 0, n_sd);
        ra.loss_out = p->d_loss;
        ra.do_adam = 0;
        HIP_TRY(launch_reduce(ra, reduce_grid(p, 0, n_sd), p->stream));
      }
      HIP_TRY(hipEventRecord(ev[1], p->stream));
      HIP_TRY(hipEventSynchronize(ev[1]));
      float t = 0.f;
      HIP_TRY(hipEventElapsedTime(&t, ev[0], ev[1]));
      total += t;
    }
    ms[which] = total / iters;
  }
  for (int c = 0; c < p->n_counters; ++c) HIP_TRY(launch_reset_counter(p->d_counters + c, p->stream));
  hipEventDestroy(ev[0]);
  hipEventDestroy(ev[1]);
  return DDP_OK;
}

int ddp_time_phases(ddp_problem* p, int iters, float* ms) {
  if (int rc = check_final(p)) return rc;
  if (iters < 1 || !ms) return fail(DDP_EINVAL, "bad timing arguments");
  if (!p->fused) return fail(DDP_ESTATE, "phase timing is for the fused step");
  // the step's launches restricted to the items of one phase, in the step's order
  const int kinds[4] = {1 << KIND_RES, (1 << KIND_DATA) | (1 << KIND_AUX), 1 << KIND_IFACE,
                        (1 << KIND_RES) | (1 << KIND_DATA) | (1 << KIND_AUX) | (1 << KIND_IFACE)};
  Item* d_sel = nullptr;
  HIP_TRY(hipMalloc(&d_sel, std::max<size_t>(1, p->titems.size()) * sizeof(Item)));
  hipEvent_t ev[2] = {nullptr, nullptr};
  int rc = DDP_OK;
  auto hip_ok = [&](hipError_t e) {
    if (e != hipSuccess && rc == DDP_OK) rc = fail(DDP_EHIP, hipGetErrorString(e));
    return rc == DDP_OK;
  };
  if (hip_ok(hipEventCreate(&ev[0])) && hip_ok(hipEventCreate(&ev[1]))) {
    for (int ph = 0; ph < 4 && rc == DDP_OK; ++ph) {
      std::vector<Item> sel;
      std::vector<int> begin, count;
      for (const ddp_problem::Launch& l : p->launches) {
        begin.push_back((int)sel.size());
        for (int i = l.begin; i < l.begin + l.count; ++i)
          if (kinds[ph] & (1 << p->titems[i].kind)) sel.push_back(p->titems[i]);
        count.push_back((int)sel.size() - begin.back());
      }
      if (!sel.empty() && !hip_ok(hipMemcpy(d_sel, sel.data(), sel.size() * sizeof(Item), hipMemcpyHostToDevice)))
        break;
      float total = 0.f;
      for (int it = 0; it < iters && rc == DDP_OK; ++it) {
        for (int c = 0; c < p->n_counters && rc == DDP_OK; ++c)
          hip_ok(launch_reset_counter(p->d_counters + c, p->stream));
        if (!hip_ok(hipEventRecord(ev[0], p->stream))) break;
        for (size_t g = 0; g < p->launches.size() && rc == DDP_OK; ++g) {
          if (count[g] == 0) continue;
          const ddp_problem::Launch& l = p->launches[g];
          KArgs ka = make_kargs(p);
          ka.items = d_sel + begin[g];
          ka.n_items = count[g];
          ka.counter = p->d_counters + g;
          ka.scratch_slot = l.slot_floats;
          hip_ok(launch_train(p->pde, l.wpmax, p->ga, p->recompute, ka, std::max(1, std::min(l.n_slots, count[g])),
                              p->stream));
        }
        float t = 0.f;
        if (hip_ok(hipEventRecord(ev[1], p->stream)) && hip_ok(hipEventSynchronize(ev[1])) &&
            hip_ok(hipEventElapsedTime(&t, ev[0], ev[1])))
          total += t;
      }
      ms[ph] = total / iters;
    }
  }
  for (int c = 0; c < p->n_counters; ++c) hip_ok(launch_reset_counter(p->d_counters + c, p->stream));
  hip_ok(hipStreamSynchronize(p->stream));
  if (ev[0]) hipEventDestroy(ev[0]);
  if (ev[1]) hipEventDestroy(ev[1]);
  hipFree(d_sel);
  return rc;
}

int ddp_plan_dump(const ddp_problem* p, const char* json_path) {
  if (!p || !json_path) return fail(DDP_EINVAL, "null argument");
  if (!p->planned) return fail(DDP_ESTATE, "no plan: call ddp_plan or ddp_finalize first");
  FILE* f = std::fopen(json_path, "w");
  if (!f) return fail(DDP_EINVAL, std::string("cannot open ") + json_path);
  std::fprintf(f,
               "{\"method\": %d, \"pde\": %d, \"fused\": %d, \"wpmax\": %d, \"tile_points\": %d, \"recompute\": %d, "
               "\"concurrent\": %d, \"tail\": %d,\n",
               p->method, p->pde, p->fused, p->wpmax, kTilePts, p->recompute, p->concurrent, p->tail_pct);
  std::fprintf(f, "\"nets\": [");
  for (size_t q = 0; q < p->nets.size(); ++q) {
    const NetDesc& n = p->nets[q];
    std::fprintf(f,
                 "%s{\"sd\": %d, \"pair\": %d, \"width\": %d, \"depth\": %d, \"d_out\": %d, \"wclass\": %d, "
                 "\"poff\": %lld, \"n_params\": %d, \"koff\": %lld, \"ksize\": %d, \"gsize\": %d, \"act\": %d, "
                 "\"adaptive\": %d}",
                 q ? ", " : "", n.sd, n.pair, n.width, n.depth, n.d_out, n.wclass, (long long)n.poff, n.n_params,
                 (long long)n.koff, n.ksize, n.gsize, n.act, n.adaptive);
  }
  std::fprintf(f, "],\n\"ifaces\": [");
  for (size_t e = 0; e < p->ifaces.size(); ++e) {
    const IfaceDesc& d = p->ifaces[e];
    std::fprintf(f, "%s{\"a\": %d, \"b\": %d, \"begin\": %d, \"count\": %d, \"method\": %d}", e ? ", " : "", d.a,
                 d.b, d.begin, d.count, d.method);
  }
  auto items = [&](const char* name, const std::vector<Item>& v) {
    std::fprintf(f, "],\n\"%s\": [", name);
    for (size_t i = 0; i < v.size(); ++i) {
      const Item& it = v[i];
      std::fprintf(f, "%s[%d, %d, %d, %d, %d, %d, %d, %lld]", i ? ", " : "", it.q, it.kind, it.begin, it.count, it.iface,
                   it.side, it.lrow, (long long)it.prow);
    }
  };
  items("train_items", p->titems);
  std::fprintf(f, "],\n");
  json_ints(f, "sd_net", p->sd_net);
  std::fprintf(f, ",\n");
  json_ints(f, "net_row_ptr", p->net_row_ptr);
  std::fprintf(f, ",\n");
  json_ints(f, "net_row_item", p->net_row_item);
  std::fprintf(f, ",\n\"net_row_prow\": [");
  for (size_t r = 0; r < p->row_prow.size(); ++r) std::fprintf(f, "%s%lld", r ? ", " : "", (long long)p->row_prow[r]);
  std::fprintf(f, "],\n");
  json_ints(f, "sd_loss_ptr", p->sd_loss_ptr);
  std::fprintf(f, ",\n");
  json_ints(f, "loss_rows", p->loss_rows);
  std::fprintf(f, ",\n");
  json_ints(f, "t_begin", p->t_begin);
  std::fprintf(f, ",\n\"launches\": [");
  for (size_t g = 0; g < p->launches.size(); ++g)
    std::fprintf(f, "%s{\"wpmax\": %d, \"begin\": %d, \"count\": %d}", g ? ", " : "", p->launches[g].wpmax,
                 p->launches[g].begin, p->launches[g].count);
  std::fprintf(f, "]");
  std::fprintf(f,
               ",\n\"partial_floats\": %lld, \"n_res\": %zu, \"n_dat\": %zu, \"n_if\": %zu, \"n_aux\": %zu}\n",
               (long long)p->partial_floats, p->h_res_xy.size() / 2, p->h_dat_xy.size() / 2, p->h_if_xy.size() / 2,
               p->h_aux_xy.size() / 2);
  std::fclose(f);
  return DDP_OK;
}

int ddp_destroy(ddp_problem* p) {
  if (!p) return fail(DDP_EINVAL, "null problem handle");
  if (p->finalized) hipStreamSynchronize(p->stream);
  release(p);
  delete p;
  return DDP_OK;
}

}  // extern "C"
