// Host-only driver of the C ABI for the sanitizer build: problem set-up,
// validation errors, per-interface conditions, activations, plan building
// and dumping, parameter counts and the state errors of calls that need a
// finalized problem.  No call here touches the GPU.  Exits non-zero on the
// first unexpected return code.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>
#include "../../include/ddpinn.h"

static int failures = 0;
#define EXPECT(call, want)                                                                            \
  do {                                                                                                \
    const int rc_ = (call);                                                                           \
    if (rc_ != (want)) {                                                                              \
      std::fprintf(stderr, "line %d: %s returned %d, expected %d (%s)\n", __LINE__, #call, rc_, want, \
                   ddp_last_error());                                                                 \
      ++failures;                                                                                     \
    }                                                                                                 \
  } while (0)

static std::vector<float> box_points(std::mt19937& rng, int n, float x0, float x1, float y0, float y1) {
  std::uniform_real_distribution<float> ux(x0, x1), uy(y0, y1);
  std::vector<float> v(2 * (size_t)n);
  for (int i = 0; i < n; ++i) {
    v[2 * i] = ux(rng);
    v[2 * i + 1] = uy(rng);
  }
  return v;
}

// nx x ny boxes on [0,1]^2 with mixed widths/depths, ragged point counts and
// every interface; method / pde / activation variations
static void grid_problem(int method, int pde, int nx, int ny, int seed, bool mixed_methods, bool activations,
                         const char* dump) {
  std::mt19937 rng(seed);
  ddp_problem* p = nullptr;
  const double coef[1] = {pde == DDP_NS2D_STEADY ? 40.0 : 0.01 / M_PI};
  EXPECT(ddp_create(&p, method, pde, coef, pde == DDP_POISSON2D ? 0 : 1), DDP_OK);
  const int dout = pde == DDP_NS2D_STEADY ? 3 : 1, neq = dout;
  const int widths[] = {17, 20, 33, 48, 64, 80, 96, 112};
  const float lw[4] = {1.f, 1.f, 1.f, 1.f};
  for (int q = 0; q < nx * ny; ++q) {
    const int w = widths[rng() % 8], depth = 1 + (int)(rng() % 6);
    std::vector<int> wd = {2};
    for (int k = 0; k < depth; ++k) wd.push_back(w);
    wd.push_back(dout);
    const int nl = (int)wd.size();
    int id = -1;
    EXPECT(ddp_add_subdomain(p, 1, &nl, wd.data(), lw, 1e-3f, &id), DDP_OK);
    const int ix = q % nx, iy = q / nx;
    const float x0 = (float)ix / nx, x1 = (float)(ix + 1) / nx, y0 = (float)iy / ny, y1 = (float)(iy + 1) / ny;
    const int nr = (int)(rng() % 300), nd = (int)(rng() % 40);
    std::vector<float> r = box_points(rng, nr, x0, x1, y0, y1), f((size_t)nr * neq, 0.5f);
    std::vector<float> d = box_points(rng, nd, x0, x1, y0, y1), g((size_t)nd * dout, 0.25f);
    EXPECT(ddp_set_points(p, id, DDP_RESIDUAL, nr, r.data(), f.data(), 0), DDP_OK);
    EXPECT(ddp_set_points(p, id, DDP_DATA, nd, d.data(), g.data(), 0), DDP_OK);
    if (activations) EXPECT(ddp_set_activation(p, id, (int)(q % 3), (int)(q % 2), 10.f), DDP_OK);
  }
  int n_if = 0;
  for (int q = 0; q < nx * ny; ++q) {
    const int ix = q % nx, iy = q / nx;
    for (int dir = 0; dir < 2; ++dir) {
      if ((dir == 0 && ix + 1 >= nx) || (dir == 1 && iy + 1 >= ny)) continue;
      const int b = dir == 0 ? q + 1 : q + nx, n = 1 + (int)(rng() % 70);
      std::vector<float> xy = box_points(rng, n, 0.f, 1.f, 0.f, 1.f);
      const float nrm[2] = {dir == 0 ? 1.f : 0.f, dir == 0 ? 0.f : 1.f};
      int e = -1;
      EXPECT(ddp_add_interface(p, q, b, n, xy.data(), nrm, 0, &e), DDP_OK);
      if (mixed_methods) EXPECT(ddp_set_interface_method(p, e, dir == 0 ? DDP_CPINN : DDP_XPINN), DDP_OK);
      ++n_if;
    }
  }
  EXPECT(ddp_set_option(p, DDP_OPT_CHUNK_POINTS, 1 + (int64_t)(rng() % 500)), DDP_OK);
  EXPECT(ddp_plan(p), DDP_OK);
  EXPECT(ddp_plan_dump(p, dump), DDP_OK);
  int64_t n = 0;
  for (int q = 0; q < nx * ny; ++q) EXPECT(ddp_param_count(p, q, &n), DDP_OK);
  // rebuilding after a change re-plans
  EXPECT(ddp_set_option(p, DDP_OPT_ITEMS_PER_SLOT, 3), DDP_OK);
  EXPECT(ddp_plan(p), DDP_OK);
  // calls that need ddp_finalize
  EXPECT(ddp_step(p, 1, nullptr), DDP_ESTATE);
  EXPECT(ddp_sync(p), DDP_ESTATE);
  EXPECT(ddp_loss_and_grad_static(p, nullptr, nullptr), DDP_ESTATE);
  EXPECT(ddp_loss_and_grad_static(nullptr, nullptr, nullptr), DDP_EINVAL);
  EXPECT(ddp_destroy(p), DDP_OK);
}

static void inverse_problem(const char* dump) {
  std::mt19937 rng(7);
  ddp_problem* p = nullptr;
  EXPECT(ddp_create(&p, DDP_XPINN, DDP_DIFFUSION2D_INV, nullptr, 0), DDP_OK);
  const float lw[4] = {1.f, 1.f, 1.f, 1.f};
  for (int q = 0; q < 3; ++q) {
    const int nl[2] = {5, 4};
    const int wd[9] = {2, 40 + 20 * q, 40 + 20 * q, 40 + 20 * q, 1, 2, 100, 100, 1};
    int id = -1;
    EXPECT(ddp_add_subdomain(p, 2, nl, wd, lw, 6e-3f, &id), DDP_OK);
    std::vector<float> r = box_points(rng, 100 + 57 * q, 0.f, 1.f, 0.f, 1.f), f(100 + 57 * q, 1.f);
    EXPECT(ddp_set_points(p, id, DDP_RESIDUAL, 100 + 57 * q, r.data(), f.data(), 0), DDP_OK);
    if (q != 1) {
      std::vector<float> k = box_points(rng, 9, 0.f, 1.f, 0.f, 1.f), kv(9, 2.f);
      EXPECT(ddp_set_points(p, id, DDP_DATA_AUX, 9, k.data(), kv.data(), 0), DDP_OK);
    }
    EXPECT(ddp_set_activation(p, id, q, 1, 10.f), DDP_OK);
  }
  std::vector<float> xy = box_points(rng, 33, 0.f, 1.f, 0.f, 1.f);
  const float nrm[2] = {0.6f, 0.8f};
  EXPECT(ddp_add_interface(p, 0, 1, 33, xy.data(), nrm, 0, nullptr), DDP_OK);
  EXPECT(ddp_add_interface(p, 1, 2, 33, xy.data(), nrm, 0, nullptr), DDP_OK);
  EXPECT(ddp_set_interface_method(p, 0, DDP_CPINN), DDP_EINVAL);
  EXPECT(ddp_plan(p), DDP_OK);
  EXPECT(ddp_plan_dump(p, dump), DDP_OK);
  EXPECT(ddp_destroy(p), DDP_OK);
}

static void validation() {
  ddp_problem* p = nullptr;
  const double coef[1] = {40.0};
  EXPECT(ddp_create(nullptr, DDP_XPINN, DDP_POISSON2D, nullptr, 0), DDP_EINVAL);
  EXPECT(ddp_create(&p, 7, DDP_POISSON2D, nullptr, 0), DDP_EINVAL);
  EXPECT(ddp_create(&p, DDP_XPINN, 9, nullptr, 0), DDP_EINVAL);
  EXPECT(ddp_create(&p, DDP_XPINN, DDP_BURGERS1D, nullptr, 0), DDP_EINVAL);
  EXPECT(ddp_create(&p, DDP_CPINN, DDP_DIFFUSION2D_INV, nullptr, 0), DDP_EINVAL);
  EXPECT(ddp_create(&p, DDP_XPINN, DDP_NS2D_STEADY, coef, 1), DDP_OK);
  const float lw[4] = {1.f, 1.f, 1.f, 1.f};
  const int nl = 4;
  const int good[4] = {2, 8, 8, 3}, uneven[4] = {2, 8, 9, 3}, wide[4] = {2, 200, 200, 3}, wrong_out[4] = {2, 8, 8, 1};
  EXPECT(ddp_add_subdomain(p, 1, &nl, good, lw, 1e-3f, nullptr), DDP_OK);
  EXPECT(ddp_add_subdomain(p, 1, &nl, uneven, lw, 1e-3f, nullptr), DDP_EINVAL);
  EXPECT(ddp_add_subdomain(p, 1, &nl, wide, lw, 1e-3f, nullptr), DDP_EINVAL);
  EXPECT(ddp_add_subdomain(p, 1, &nl, wrong_out, lw, 1e-3f, nullptr), DDP_EINVAL);
  EXPECT(ddp_add_subdomain(p, 1, &nl, good, lw, 1e-3f, nullptr), DDP_OK);
  const float bad_xy[4] = {0.1f, NAN, 0.2f, 0.3f}, vals[6] = {0, 0, 0, 0, 0, 0};
  EXPECT(ddp_set_points(p, 0, DDP_RESIDUAL, 2, bad_xy, vals, 0), DDP_EINVAL);
  EXPECT(ddp_set_points(p, 5, DDP_RESIDUAL, 0, nullptr, nullptr, 0), DDP_EINVAL);
  const float xy[4] = {0.5f, 0.1f, 0.5f, 0.9f}, nrm[2] = {1.f, 0.f};
  EXPECT(ddp_add_interface(p, 0, 3, 2, xy, nrm, 0, nullptr), DDP_EINVAL);
  EXPECT(ddp_add_interface(p, 0, 0, 2, xy, nrm, 0, nullptr), DDP_EINVAL);
  EXPECT(ddp_add_interface(p, 0, 1, 2, xy, nrm, 0, nullptr), DDP_OK);
  EXPECT(ddp_set_interface_method(p, 1, DDP_CPINN), DDP_EINVAL);
  EXPECT(ddp_set_activation(p, 0, 5, 0, 10.f), DDP_EINVAL);
  EXPECT(ddp_set_activation(p, 0, DDP_ACT_SIN, 1, -1.f), DDP_EINVAL);
  EXPECT(ddp_set_option(p, 99, 1), DDP_EINVAL);
  EXPECT(ddp_set_option(p, DDP_OPT_RECOMPUTE, 2), DDP_EINVAL);
  EXPECT(ddp_set_option(p, DDP_OPT_RECOMPUTE, 0), DDP_OK);
  EXPECT(ddp_set_option(p, DDP_OPT_CONCURRENT, -1), DDP_EINVAL);
  EXPECT(ddp_set_option(p, DDP_OPT_CONCURRENT, 1), DDP_OK);
  EXPECT(ddp_set_option(p, DDP_OPT_TAIL, 101), DDP_EINVAL);
  EXPECT(ddp_set_option(p, DDP_OPT_TAIL, 30), DDP_OK);
  EXPECT(ddp_mfma_probe(0, nullptr), DDP_EINVAL);
  EXPECT(ddp_plan(p), DDP_OK);
  EXPECT(ddp_plan_dump(p, "/nonexistent-dir/x.json"), DDP_EINVAL);
  EXPECT(ddp_destroy(p), DDP_OK);
}

int main(int argc, char** argv) {
  const std::string dir = argc > 1 ? argv[1] : "/tmp";
  validation();
  grid_problem(DDP_XPINN, DDP_POISSON2D, 4, 4, 1, false, false, (dir + "/a.json").c_str());
  grid_problem(DDP_CPINN, DDP_NS2D_STEADY, 3, 3, 2, false, true, (dir + "/b.json").c_str());
  grid_problem(DDP_CPINN, DDP_BURGERS1D, 4, 2, 3, true, true, (dir + "/c.json").c_str());
  grid_problem(DDP_XPINN, DDP_POISSON2D, 1, 1, 4, false, true, (dir + "/d.json").c_str());
  inverse_problem((dir + "/e.json").c_str());
  std::printf("%s: %d unexpected return codes\n", failures ? "FAIL" : "ok", failures);
  return failures ? 1 : 0;
}
