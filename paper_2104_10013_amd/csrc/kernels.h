// Host-side entry points of the gfx950 kernels (kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include "ddp_internal.h"

namespace ddp {

// dynamic LDS bytes of the train kernel for a width class
size_t lds_bytes(int pde, int wpmax);
// floats of one workgroup's activation stash for the widest class wpmax;
// rh: the recompute policy (a^k stashed, h^{k-1} rebuilt in the reverse pass)
int64_t scratch_slot_floats(int pde, int wpmax, bool rh);
// width group of the kernel that runs classes up to wpmax: the class itself,
// or with the general activation rule (ga) the group up to 80 or up to 112
int kernel_wpmax(int wpmax, bool ga);
// resident train workgroups per compute unit (also raises the LDS limit)
hipError_t train_occupancy(int pde, int wpmax, bool ga, bool rh, int* blocks_per_cu);

// persistent loss + gradient-partial kernel over ka.items (ka.prologue:
// settle the Adam step counter first); ga: the general-activation kernel
// (wpmax from kernel_wpmax); rh: the recompute policy's kernel
hipError_t launch_train(int pde, int wpmax, bool ga, bool rh, const KArgs& ka, int grid, hipStream_t st);
// set a work counter to zero
hipError_t launch_reset_counter(int* c, hipStream_t st);
// gradient reduction, loss reduction and optional Adam; re-arms ra.counter_reset
hipError_t launch_reduce(const RArgs& ra, int grid, hipStream_t st);
// refresh the kernel-layout parameter copy of networks [n_begin, n_end)
hipError_t launch_pack(const float* params, float* kparams, const NetDesc* nets, const int64_t* net_poff,
                       int n_begin, int n_end, int64_t n, hipStream_t st);
// stitched evaluation: n_cols outputs per point from each owner's networks
hipError_t launch_eval(const float* params, const NetDesc* nets, const int* sd_net, int n_sd, int n, const float* xy,
                       const int* owner, float* out, int n_cols, hipStream_t st);

// Static device scratch of the allocation-free entry point (noalloc.hip):
// kStaticCounterBytes of work counters, then activation stash slots.
constexpr size_t kStaticScratchBytes = (size_t)256 << 20;
constexpr size_t kStaticCounterBytes = 4096;
// device address of the static scratch on device (current); looked up once
// per device with hipGetSymbolAddress
hipError_t static_scratch(int device, void** ptr);
// zero n ints with a kernel (capturable; no memset node)
hipError_t launch_zero_ints(int* p, int n, hipStream_t st);

// FP32 MFMA rate (TFLOP/s) the device sustains on a pure MFMA loop of iters
// unrolled steps per wave (probe.hip); synchronous
hipError_t mfma_probe(int iters, double* tflops);

}  // namespace ddp
