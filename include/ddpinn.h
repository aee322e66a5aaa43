/*
 * ddpinn.h -- C ABI of libddpinn, the MI355X (gfx950) training step of
 * domain-decomposed physics-informed neural networks (cPINN and XPINN).
 *
 * Problem statement (Sec. 4.2): the domain is split into N_sd non-overlapping
 * subdomains Omega_q, each with its own fully connected tanh network (Sec. 3,
 * identity output layer) and its own width and depth.  Each subdomain has
 * residual points x_F, training (boundary / initial / data) points x_u, and
 * shares interface points x_I with each neighbour q+.  One training step
 * (Algorithm 1) evaluates every network at its points together with the input
 * derivatives the PDE needs, forms the subdomain loss J(Theta_q) of
 * Eq. cPINNLoss or Eq. XPINNLoss, differentiates it with respect to Theta_q
 * with the neighbour's interface values held fixed, and applies one Adam
 * update per subdomain (Sec. 6).
 *
 * Conventions shared by every call:
 *  - Return value: DDP_OK (0) on success, a negative DDP_E* code otherwise;
 *    ddp_last_error() then returns a thread-local message.  No C++ exception
 *    crosses this interface.
 *  - Ownership: every input array is copied by the library (at the call, or
 *    at ddp_finalize for topology data); the caller keeps its buffers.
 *    Output arrays are owned by the caller.
 *  - "on_device" = 1 means the pointer is HIP device memory, 0 host memory.
 *  - Asynchrony: after ddp_finalize every call that launches work is
 *    stream-ordered on the stream given to ddp_finalize and returns without
 *    waiting; ddp_sync() waits and reports non-finite losses.
 *  - Parameters of one network use the canonical flat layout: for each layer
 *    k = 1..L, W^k as [N_k][N_{k-1}] row-major followed by b^k[N_k]; an
 *    adaptive network (ddp_set_activation) then has its slopes a^1..a^{L-1}.
 *  - A handle is not thread-safe; use one handle per thread.
 */
#ifndef DDPINN_H
#define DDPINN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ddp_problem ddp_problem; /* opaque, owned by the library */

enum {
  DDP_OK = 0,
  DDP_EINVAL = -1,     /* invalid argument or unsupported combination */
  DDP_ENOMEM = -2,     /* host or device allocation failed */
  DDP_EHIP = -3,       /* a HIP runtime call failed */
  DDP_ESTATE = -4,     /* call not valid in the handle's current state */
  DDP_ENONFINITE = -5  /* a loss computed since the last sync was NaN or inf */
};

/* Algorithm 1 selects the interface condition: cPINN (normal-flux continuity)
 * or XPINN (residual continuity); both add average-solution continuity.
 * Normal fluxes f(u) . n of the conservative forms:
 *  POISSON2D    f = -grad u.
 *  BURGERS1D    the space-time flux (u^2/2 - nu u_x, u) in (x, t).
 *  NS2D_STEADY  Table 1: x-momentum (u^2 + p - u_x/Re, uv - u_y/Re),
 *               y-momentum (uv - v_x/Re, v^2 + p - v_y/Re), mass (u, v); the
 *               three squared jumps are summed. */
enum { DDP_CPINN = 0, DDP_XPINN = 1 };

/* Operators L_x of Eq. ProSet (F = L_x(u) - f):
 *  POISSON2D      -Lap u = f, inputs (x, y), one output.
 *  BURGERS1D      u_t + u u_x - nu u_xx = f (Eq. BE), inputs (x, t), coef[0] = nu.
 *  NS2D_STEADY    steady incompressible Navier-Stokes (Eq. NSEq), inputs (x, y),
 *                 outputs (u, v, p), coef[0] = Re; three residual equations.
 *  DIFFUSION2D_INV  inverse problem of Sec. 7.6, div(K grad u) = f (Eq. heq),
 *                 inputs (x, y): every subdomain has two one-output networks,
 *                 u and the unknown conductivity K; F = K Lap u + grad K . grad u
 *                 - f.  XPINN only: the interface terms match the average of
 *                 the pair (u, K) and the operator value L(u, K). */
enum { DDP_POISSON2D = 0, DDP_BURGERS1D = 1, DDP_NS2D_STEADY = 2, DDP_DIFFUSION2D_INV = 3 };

/* hidden-layer activations Phi (Sec. 3; per subdomain, Table 4) */
enum { DDP_ACT_TANH = 0, DDP_ACT_SIN = 1, DDP_ACT_COS = 2 };

/* point kinds for ddp_set_points; DATA_AUX = points with known K values
 * (inverse problem), whose squared misfit is added to MSE_u */
enum { DDP_RESIDUAL = 0, DDP_DATA = 1, DDP_DATA_AUX = 2 };

/* tuning options (ddp_set_option), all optional */
enum {
  DDP_OPT_CHUNK_POINTS = 0, /* upper bound of points per work item (default 1024) */
  DDP_OPT_BLOCKS_PER_CU = 1, /* persistent workgroups per compute unit (0 = as many as fit) */
  DDP_OPT_ITEMS_PER_SLOT = 2, /* work items per resident workgroup the plan aims for (default 4) */
  DDP_OPT_RECOMPUTE = 3, /* activation stash policy (default 0): 1 = the forward pass stores the
                           pre-activation streams a^k only and the reverse pass rebuilds h^k from
                           them with the activation rule; 0 = it stores a^k and h^k */
  DDP_OPT_CONCURRENT = 4, /* fused step whose items need two train kernels (networks both at most
                            80 and wider than 80): 1 = the two persistent launches run side by
                            side on two streams (each with its own activation stash), so the
                            second takes the compute units the first's drained workgroups free;
                            0 (default) = one after the other.  No effect with one launch. */
  DDP_OPT_TAIL = 5 /* fused step: percent (0..100, default 0) of each subdomain's residual points
                      cut into one-tile (64-point) work items instead of the plan's longer ones;
                      the cost-ordered work queue hands them out last, so the workgroups that
                      finish their long items early share the end of the launch */
};

/* Create an empty problem.  coef holds n_coef operator constants (see the
 * operator list above).  method is DDP_CPINN or DDP_XPINN: the interface
 * condition of every interface unless ddp_set_interface_method overrides it
 * (DDP_DIFFUSION2D_INV: XPINN only). */
int ddp_create(ddp_problem** out, int method, int pde, const double* coef, int n_coef);

/* Add subdomain Omega_q with its network (Sec. 3).  n_nets is 1, or 2 for
 * DDP_DIFFUSION2D_INV (the u-network, then the K-network).  For each network
 * i, n_layers[i] = L + 1 entries of widths (concatenated over the networks)
 * = N_0..N_L with N_0 = 2, N_L = number of PDE outputs (1 for the K-network),
 * hidden widths equal and at most 112, 1..8 hidden layers.  The subdomain's
 * flat parameter vector is the u-network's canonical parameters followed by
 * the K-network's.
 * loss_w = (W_u, W_F, W_I, W_flux for cPINN | W_IF for XPINN) of Eq. cPINNLoss
 * / Eq. XPINNLoss.  lr is this subdomain's Adam learning rate.  *sd_id
 * receives q (0-based, in call order). */
int ddp_add_subdomain(ddp_problem* p, int n_nets, const int* n_layers, const int* widths,
                      const float* loss_w, float lr, int* sd_id);

/* Point sets of a subdomain (Sec. 4.2: residual points, training points of
 * the data term; Sec. 7.6: the K data of the inverse problem).
 * Set the residual points {x_F} (kind DDP_RESIDUAL; val = forcing f(x), n x
 * n_eq), training points {x_u} (kind DDP_DATA; val = targets u^(i), n x
 * N_L) or K data points (kind DDP_DATA_AUX, inverse problem; val = K, n x 1)
 * of subdomain sd.  xy is n x 2 interleaved.  Replaces earlier points of
 * that kind.  Non-finite values are rejected.  Valid before ddp_finalize. */
int ddp_set_points(ddp_problem* p, int sd, int kind, int n, const float* xy, const float* val,
                   int on_device);

/* Interface points x_I common to two subdomains (Sec. 4.2; the normal n of
 * the flux term of Eq. cPINNLoss).
 * Add a common interface between sd_a and sd_b (a != b) with n points (n x 2)
 * and unit normal (pointing from a to b) used by the cPINN flux term.  Both
 * networks are evaluated at the same points.  *if_id receives its index. */
int ddp_add_interface(ddp_problem* p, int sd_a, int sd_b, int n, const float* xy,
                      const float normal[2], int on_device, int* if_id);

/* Activation of subdomain sd's networks (default: tanh, not adaptive).  Hidden
 * layer k applies Phi(n a^k x) to its pre-activation x (Sec. 3), Phi = tanh,
 * sin or cos (act = DDP_ACT_*).  adaptive = 1 makes the slopes a^1..a^D of
 * each network trainable parameters with scale n = slope_n: they follow that
 * network's layers in the canonical flat layout (so ddp_param_count grows by
 * D per network), their gradients are dJ/da^k, Adam updates them, and the
 * paper initialises them to n a^k = 1.  adaptive = 0 fixes n a^k = 1.
 * sin and cos are evaluated to about 1e-7 absolute for |n a^k x| up to 1e5;
 * larger arguments lose accuracy (there is no check on the device).
 * DDP_EINVAL for an unknown subdomain or activation, adaptive not 0/1, or
 * slope_n not finite and > 0.  Valid before ddp_finalize. */
int ddp_set_activation(ddp_problem* p, int sd, int act, int adaptive, float slope_n);

/* Give interface if_id its own condition, DDP_CPINN (flux matching) or
 * DDP_XPINN (residual continuity), instead of the problem's: e.g. cPINN
 * across space interfaces and XPINN across time interfaces of a time-dependent
 * conservation law, the combination the paper's conclusions propose.  The
 * fourth loss term of a subdomain (weight loss_w[3], slot 4 of loss_terms) then
 * sums the flux terms of its cPINN interfaces and the residual terms of its
 * XPINN interfaces.  DDP_EINVAL for an unknown interface or method, or
 * DDP_CPINN on DDP_DIFFUSION2D_INV.  Valid before ddp_finalize. */
int ddp_set_interface_method(ddp_problem* p, int if_id, int method);

/* Set a tuning option (see DDP_OPT_*).  Valid before ddp_finalize. */
int ddp_set_option(ddp_problem* p, int option, int64_t value);

/* The set-up before Algorithm 1's iterations: every subdomain's data on the
 * one GPU (the paper's one rank per subdomain becomes one persistent launch
 * over all of them).
 * Validate, pack points and parameters into device memory, build the work
 * list, and (fused = 1) capture one training step as a HIP graph on
 * hip_stream (a hipStream_t, or NULL for the null stream).  fused = 0 selects
 * the per-subdomain path: the same kernels launched once per subdomain,
 * without the persistent schedule or a graph.  Parameters start at zero;
 * set them with ddp_set_params.  Topology calls fail with DDP_ESTATE after. */
int ddp_finalize(ddp_problem* p, void* hip_stream, int fused);

/* Autotuner: time candidate work plans on this problem (points per item
 * bound 256..2048, items per resident workgroup 1..8, workgroups per compute
 * unit 1..as many as fit, both activation stash policies of
 * DDP_OPT_RECOMPUTE, where the step has two train launches both settings
 * of DDP_OPT_CONCURRENT, and on the fused path a tail share DDP_OPT_TAIL of 0
 * or 30 percent) with iters loss-and-gradient passes each, time the
 * three fastest again (three interleaved rounds of 2 x iters passes), keep the
 * fastest and rebuild the step graph with it.  Parameters and Adam state are
 * not changed.  cache_path (may be NULL) is a JSON-lines file of earlier
 * choices keyed by a signature of the problem (operator, interface methods, fused or
 * per-subdomain path, widths, depths, point counts, CU count): a hit skips
 * the search, a miss appends the new choice.  choice (may be NULL) receives
 * the 6 chosen values (points per item, items per workgroup, workgroups per
 * compute unit, recompute policy, concurrent launches, tail share).  Not safe to call while the caller's stream runs other
 * work on this problem. */
int ddp_autotune(ddp_problem* p, int iters, const char* cache_path, int64_t* choice);

/* Number of parameters of subdomain sd (its networks' canonical layouts, concatenated). */
int ddp_param_count(const ddp_problem* p, int sd, int64_t* n);

/* Copy subdomain sd's parameters in (set) or out (get), canonical layout.
 * Stream-ordered after ddp_finalize. */
int ddp_set_params(ddp_problem* p, int sd, const float* flat, int on_device);
int ddp_get_params(ddp_problem* p, int sd, float* flat, int on_device);

/* The computation stage of Algorithm 1: the loss J(Theta_q) of
 * Eq. cPINNLoss / Eq. XPINNLoss per subdomain and its gradient, with the
 * neighbours' interface values as the received (fixed) quantities.
 * Evaluate the loss of every subdomain and dJ(Theta_q)/dTheta_q (neighbour
 * interface values held fixed), without updating parameters.
 * loss_terms: device, n_sd x 5 = (J, MSE_u, MSE_F, MSE_uavg, MSE_flux|MSE_R).
 * grad: device, all subdomains' gradients concatenated in subdomain order,
 * canonical layout (may be NULL).  Stream-ordered. */
int ddp_loss_and_grad(ddp_problem* p, float* loss_terms, float* grad);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * ddp_loss_and_grad with the work counters and the activation stash of its
 * train kernels in a static device array of the library instead of the
 * handle's buffers.  The array holds 256 MiB per device (4 KiB of counters,
 * then stash slots of one workgroup each) from the first call on that device
 * until the process ends.  The persistent launches run as many workgroups as
 * stash slots fit, at most as many as the plan's, so a plan that wants more
 * runs slower; results are those of ddp_loss_and_grad bit for bit (each work
 * item writes its own gradient and loss rows, summed in a fixed order).
 * The call launches kernels only: no hipMalloc, hipFree or other allocation
 * (its first call on a device looks the array's address up once).  All calls
 * on one device share that device's array, and its counters are zeroed at the
 * start of each call: calls that overlap on one device race (keep them on one
 * stream).  Arguments and outputs as for ddp_loss_and_grad.  Errors:
 * DDP_ESTATE before ddp_finalize or when the problem's device is not the
 * current one; DDP_EINVAL when one workgroup's stash exceeds the array or the
 * per-subdomain path needs more than 1024 work counters. */
int ddp_loss_and_grad_static(ddp_problem* p, float* loss_terms, float* grad);

/* Algorithm 1's iteration with the optimiser of Sec. 6 (Adam), one
 * optimiser per subdomain with its own learning rate.
 * Run n_steps training steps (loss, gradient, Adam with beta = (0.9, 0.999),
 * eps = 1e-8).  loss_terms (device, may be NULL) receives the terms of the
 * last step, evaluated at the parameters before its update. */
int ddp_step(ddp_problem* p, int n_steps, float* loss_terms);

/* Adam state: m and v (host, all parameters concatenated) and the number of
 * completed steps t.  ddp_get_state synchronises the stream. */
int ddp_get_state(ddp_problem* p, float* m, float* v, int64_t* t);
int ddp_set_state(ddp_problem* p, const float* m, const float* v, int64_t t);

/* Stitched solution of Eq. FSol at n points (device xy, n x 2).  The
 * indicator of Eq. FSol is geometry the library does not hold (it has point
 * sets, not subdomain shapes), so the caller supplies it: owner (device,
 * n x 4 int32, -1 padded) lists the subdomains whose closure holds each point;
 * the output (device, n x N_L; n x 2 = (u, K) for DDP_DIFFUSION2D_INV)
 * averages their networks (indicator 1/S). */
int ddp_eval(ddp_problem* p, int n, const float* xy, const int* owner, float* u_out);

/* Wait for the stream; DDP_ENONFINITE if a loss since the last sync was not
 * finite (the flag is then cleared). */
int ddp_sync(ddp_problem* p);

/* Average device time in milliseconds, measured with HIP events on the
 * problem's stream over iters repetitions: ms[0] = the train kernel launch(es)
 * of one step (per-point loss, adjoint and gradient partials: one persistent
 * launch when fused, one per subdomain otherwise), ms[1] = the reduction
 * kernel (gradient and loss sums, without Adam).  ms must hold 2 floats.
 * Leaves parameters and the Adam state unchanged. */
int ddp_time_kernels(ddp_problem* p, int iters, float* ms);

/* Phase timing of the fused step (cf. Fig. 4's data-loss / residual-loss
 * split): mean milliseconds over iters runs of the step's train launches
 * restricted to the work items of one phase, ms[0] residual points, ms[1]
 * training (data) points, ms[2] interface points, ms[3] all items.  The
 * phases' sum exceeds ms[3] by what their separate launches do not overlap.
 * Synchronous; allocates and frees a device copy of the item list.  Leaves
 * parameters and the Adam state unchanged.  DDP_ESTATE for the per-subdomain
 * path or before ddp_finalize; DDP_EINVAL for iters < 1 or a null ms (4
 * floats). */
int ddp_time_phases(ddp_problem* p, int iters, float* ms);

/* Measurement: the FP32 matrix-core rate the current device sustains, in
 * TFLOP/s, on a loop of 16x16x4 FP32 MFMAs with no memory traffic (eight
 * waves per SIMD, iters unrolled steps of four independent MFMAs per wave;
 * 2000 runs for a few milliseconds).  This attainable peak sits below the
 * published 157.3 TFLOP/s when the part clocks below 2.4 GHz under load.
 * Synchronous on the null stream; allocates and frees a small device buffer.
 * DDP_EINVAL for iters outside 1..2^20 or a null tflops. */
int ddp_mfma_probe(int iters, double* tflops);

/* Write the packed plan (subdomains, interfaces, work items, offsets) as JSON.
 * Host only; valid after ddp_plan (or ddp_finalize). */
int ddp_plan_dump(const ddp_problem* p, const char* json_path);

/* Build the packed plan on the host without touching the GPU (what
 * ddp_finalize does before it allocates); for inspection and tests. */
int ddp_plan(ddp_problem* p);

/* Thread-local message of the last failing call on this thread. */
const char* ddp_last_error(void);

/* Release all host and device resources of the handle. */
int ddp_destroy(ddp_problem* p);

#ifdef __cplusplus
}
#endif

#endif /* DDPINN_H */
