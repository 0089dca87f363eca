/*
 * lbcm_net — learned surrogate for the lattice Boltzmann step of lbcm.h: a stack of 3x3
 * convolutions with circular padding that maps the macroscopic state (phi, v_x, v_y, rho) of
 * periodic boxes to the state K lattice steps later, as state + alpha * network(state) with a
 * fixed per-channel output scale alpha.  The density carries the pressure field, without which
 * the velocity K steps on is not determined by the state.  The first layer runs in FP32 on the
 * matrix cores (its weight gradient on the BF16 ones with every FP32 state value split exactly
 * into three BF16 parts, so that the products stay exact and the sums FP32); the others run on
 * them in BF16 (BF16 activations and weights, FP32 accumulation); master parameters,
 * gradients and the Adam moments are FP32.  This is not part of the paper's method: it is
 * trained on trajectories of the method and checked against it (see lbcm_step).
 *
 * Conventions
 *   - A network is created for a fixed batch of B samples of H x W pixels (B * H * W <= 2^26).
 *     Layer 0 maps 4 -> C channels, layers 1..L-2 map C -> C (ReLU after every
 *     layer but the last), layer L-1 maps C -> 4; C is 32 or 64.
 *   - State tensors on the device are FP32 [B][H][W][4]: (phi, v_x / u_scale, v_y / u_scale,
 *     (rho - 1) / rho_scale).
 *   - The parameter vector (FP32, lbcm_net_param_count entries) holds, layer after layer, the
 *     weights W[t][ci][co] (t = 3 (dy + 1) + (dx + 1) is the tap reading the input at (y + dy,
 *     x + dx); ci, co the real channel counts) and then the biases b[co'], where co' runs over the
 *     padded output channels (C, or 32 for the last layer; the entries past 4 must be 0).
 *   - Return codes and ownership as in lbcm.h (LBCM_OK, LBCM_EINVAL, LBCM_ENOMEM, LBCM_EHIP).
 *     Work is queued on the stream given at creation; calls that return host data synchronise.
 */
#ifndef LBCM_NET_H
#define LBCM_NET_H

#include <stddef.h>
#include <stdint.h>

#include "lbcm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbcm_net lbcm_net;

/* Allocate a network and its buffers (parameters zero).  stream: hipStream_t or NULL. */
int lbcm_net_create(int32_t batch, int32_t height, int32_t width, int32_t channels, int32_t layers, void *stream,
                    lbcm_net **out);

size_t lbcm_net_param_count(const lbcm_net *n);

/* Output scale alpha[0..3] (host, each finite and > 0; default 1): out = state + alpha * z and
   the loss is mean(((out - target) / alpha)^2).  Takes effect at the next call. */
int lbcm_net_set_output_scale(lbcm_net *n, const float *alpha);

/* Copy the FP32 parameter vector in (resets the Adam moments) or out.  Synchronise. */
int lbcm_net_set_params(lbcm_net *n, const float *host, size_t count);
int lbcm_net_get_params(lbcm_net *n, float *host, size_t count);

/* Forward pass on a device state [B][H][W][4]; out (device, same shape, may be NULL) receives
   state + alpha * network(state).  The activations are kept for lbcm_net_backward. */
int lbcm_net_forward(lbcm_net *n, const float *in, float *out);

/* Forward pass from device FP64 planes [B][H][W] of phi, v_x, v_y, rho (scaled on the way in as
   in the state tensor, and back on the way out) into device FP64 planes.  The output planes may
   be the input planes (in place).  The conversions run inside the first and last layers; with 64
   channels the layers run in fused pairs.  The result equals lbcm_net_forward's on the converted
   state, converted back, bit for bit. */
int lbcm_net_forward_planes(lbcm_net *n, const double *phi, const double *ux, const double *uy, const double *rho,
                            double u_scale, double rho_scale, double *phi_out, double *ux_out, double *uy_out,
                            double *rho_out);

/* Device FP64 planes -> a device state tensor [B][H][W][4]. */
int lbcm_net_state_from_planes(lbcm_net *n, const double *phi, const double *ux, const double *uy, const double *rho,
                               double u_scale, double rho_scale, float *state);

/* A training batch from recorded frames: state sample b (b < B) is frame frame_index[b] of the
   device FP64 planes frames[c][f][y][x] (c = phi, v_x, v_y, rho, f < nframes, each H x W as the
   network), transformed by element `symmetry` (0..7) of the square's symmetry group (transpose
   if bit 2 is set, then flip y if bit 1, then flip x if bit 0; velocity components are swapped
   and negated with the grid) and scaled as in lbcm_net_state_from_planes.  frame_index: host
   int32[B], copied (each in [0, nframes)); state: device [B][H][W][4].  A transposing symmetry
   needs H == W.  Asynchronous on the network's stream. */
int lbcm_net_gather_states(lbcm_net *n, const double *frames, int64_t nframes, const int32_t *frame_index, int32_t symmetry,
                           double u_scale, double rho_scale, float *state);

/* Gradient of the loss mean(((out - target) / alpha)^2) over pixels and the 4 channels, after
   lbcm_net_forward (lbcm_net_forward_planes keeps no output state for it), into the internal FP32 gradient vector (same layout as the parameters).  *loss
   (host, may be NULL) receives the loss (then the call synchronises). */
int lbcm_net_backward(lbcm_net *n, const float *target, float *loss);

/* Copy the gradient vector of the last lbcm_net_backward to the host.  Synchronises. */
int lbcm_net_get_grads(lbcm_net *n, float *host, size_t count);

/* One Adam update of the parameters with the current gradients (t = 1, 2, ... the step count). */
int lbcm_net_adam(lbcm_net *n, float lr, float beta1, float beta2, float eps, int64_t t);

int lbcm_net_destroy(lbcm_net *n);
const char *lbcm_net_last_error(const lbcm_net *n);

/* ---- hybrid driver ------------------------------------------------------------------------
   Advances a periodic lattice in windows of J * K lattice steps.  A window reads (phi, v, rho)
   of the lattice, makes J - 1 surrogate jumps of K steps, and does the J-th jump both ways: with
   the surrogate, and with K lattice Boltzmann steps on a private scratch lattice from
   equilibrium populations of the same state.  The check error is ||phi_net - phi_LB|| /
   ||phi_LB|| (L2 over the box), the velocity error ||v_net - v_LB|| / ||v_LB||.  When the first
   is at or below the threshold (and the second at or below the velocity threshold, if that is
   > 0) the scratch state is copied into the lattice: the window ends in the lattice Boltzmann
   result.  Otherwise the lattice, which still holds the window's starting populations, runs the
   window with the plain step, and after k failed checks in a row the next min(2^(k-1), 16)
   windows too.  The lattice and the network must share a stream; the network is built for one
   box (batch 1) of the lattice's size. */

typedef struct lbcm_hybrid lbcm_hybrid;

typedef struct lbcm_hybrid_stats {
    int64_t steps;         /* lattice steps of simulated time advanced */
    int64_t jumps;         /* accepted surrogate jumps (not counting the checked jumps) */
    int64_t lb_steps_run;  /* lattice Boltzmann steps executed (checks, redone and plain windows) */
    int64_t checks;        /* checks made */
    int64_t failed_checks; /* checks above the threshold */
    double last_error;     /* error of the last check */
    double max_error;      /* largest check error so far */
    double last_velocity_error;          /* ||v_net - v_LB|| / ||v_LB|| of the last check */
    double max_accepted_error;           /* largest check error of an accepted window */
    double max_accepted_velocity_error;  /* largest velocity error of an accepted window */
    int64_t audits;                      /* audited windows (lbcm_hybrid_set_audit) */
    int64_t failed_audits;               /* audits above a threshold */
    double max_audited_error;            /* largest phi error accumulated over an audited window */
    double max_audited_velocity_error;   /* the same for the velocity */
} lbcm_hybrid_stats;

/* lattice: a periodic lattice after lbcm_init; net: the trained network (batch 1, same ny x nx);
   steps_per_jump K >= 1 (what the network was trained for); jumps_per_check J >= 1; u_scale,
   rho_scale > 0: velocity and density scales of the network's state; threshold >= 0: largest
   accepted check error; velocity_threshold: largest accepted velocity error (<= 0: not checked).  The
   driver borrows both handles (they must outlive it) and allocates its scratch lattice and
   planes. */
int lbcm_hybrid_create(lbcm_handle *lattice, lbcm_net *net, int32_t steps_per_jump, int32_t jumps_per_check,
                       double u_scale, double rho_scale, double threshold, double velocity_threshold,
                       lbcm_hybrid **out);

/* Advance by `windows` windows (each J * K lattice steps; waits once per window for the check's
   sums).  Within one call, a window that follows an accepted one starts from that check's
   lattice fields, and its first jumps (at most 2) are queued before the wait for the previous
   check; a rejection drops them.  The results equal those of `windows` calls of one window,
   bit for bit.  The lattice must not be used by the caller during the call. */
int lbcm_hybrid_advance(lbcm_hybrid *h, int64_t windows);

/* Audits (every >= 1; 0, the default, turns them off): every `every`-th window (counted over the
   driver's life, plain windows included) is an audit instead of a checked window.  The network
   makes all J jumps from the window's start, the lattice runs the whole window with the lattice
   Boltzmann step from the window's starting populations, and the network's state is compared with
   that result with the same errors and thresholds as a check.  The check of an ordinary window
   tests only its last jump, from equilibrium populations of the network's state; an audit measures
   the error accumulated over all J jumps.  The lattice ends an audit in the lattice Boltzmann
   result either way; a failed audit backs off as a failed check does.  Errors: LBCM_EINVAL. */
int lbcm_hybrid_set_audit(lbcm_hybrid *h, int32_t every);

int lbcm_hybrid_get_stats(const lbcm_hybrid *h, lbcm_hybrid_stats *out);
int lbcm_hybrid_destroy(lbcm_hybrid *h);
const char *lbcm_hybrid_last_error(const lbcm_hybrid *h);

#ifdef __cplusplus
}
#endif

#endif /* LBCM_NET_H */
