/*
 * libpic warm start: a small network that maps discharge parameters to
 * converged profiles, and a loader that starts a discharge from profiles.
 *
 * A run of the method of arXiv:2109.04469 (Sec. 2) started from a uniform
 * plasma spends many RF cycles relaxing before its time averages (the
 * density profiles and the EEPF of Sec. 3) settle. A warm start loads the
 * particles from predicted profiles instead, and the method itself (started
 * cold) remains the reference the prediction is judged against.
 *
 * Same conventions as pic.h: int32 status returns (PIC_OK or PIC_E*), no
 * device allocation by the library (the caller passes one workspace), all
 * device work on the stream given at init.
 */
#ifndef LIBPIC_WARMSTART_H
#define LIBPIC_WARMSTART_H

#include "pic.h"

#ifdef __cplusplus
extern "C" {
#endif

/* ---- loading particles from profiles ------------------------------------
 * Replaces the particles of `species` of h by n particles (like
 * pic_set_state, step index set to `step`, event counters and the error
 * word cleared). Positions follow the density profile dens[npts] given at
 * x_k = k L / (npts - 1), linear between the points (its scale is
 * irrelevant; negative values count as 0): slot i's position is where the
 * cumulative density reaches u_i times the total, for its position uniform
 * u_i, solved exactly within the interval (the cumulative density is
 * quadratic there). Each velocity component is normal with variance
 * e T(x) / m, T(x) in eV linear between the points of temp_ev[npts]
 * (for electrons (2/3) of the mean energy; for ions the gas temperature).
 * Draws: Philox4x32-10 keyed (seed, run) of h with counter
 * (0xFFFFFFFE, slot, 16 species + purpose, 0): purpose 0 word 0 is u_i,
 * purpose 1 gives the three normals by Box-Muller (words 0-1, 2-3).
 * dens and temp_ev are DEVICE arrays of npts doubles, 2 <= npts <= 8192.
 * A profile of zero mass puts every particle at the start of the last
 * interval. PIC_ECAPACITY if n exceeds the species' capacity.
 * Synchronises. */
int pic_load_profile(pic_handle* h, int species, int64_t n, const double* dens,
                     const double* temp_ev, int npts, int64_t step);

/* ---- the network --------------------------------------------------------
 * n_in inputs -> depth hidden layers of `width` (GELU, the exact erf form)
 * -> n_out linear outputs. Parameters are one FP32 vector: for each layer
 * in order, its weight matrix W [out x in] row-major, then its bias [out].
 * The products use BF16 copies of the weight matrices and of the
 * activations (round to nearest even) with FP32 accumulation on the
 * matrix cores; biases, activations and gradients are FP32. Training
 * minimises the mean squared error over all outputs of a batch with
 * AdamW on the FP32 master parameters. Inputs and outputs are DEVICE
 * arrays, row-major [batch x n_in] / [batch x n_out], batch <= max_batch.
 * A network is used by one host thread at a time. */
typedef struct pic_mlp pic_mlp;

int pic_mlp_workspace_bytes(int n_in, int width, int depth, int n_out, int max_batch,
                            uint64_t* bytes);
/* workspace: device memory of pic_mlp_workspace_bytes(), 256-byte aligned,
 * owned by the caller until pic_mlp_free. Parameters are undefined until
 * pic_mlp_set_params. */
int pic_mlp_init(int n_in, int width, int depth, int n_out, int max_batch, void* workspace,
                 uint64_t workspace_bytes, void* stream, pic_mlp** out);
int pic_mlp_num_params(const pic_mlp* m, int64_t* n);
/* Copies the FP32 parameter vector in (host or device) and resets the Adam
 * state. Synchronises. */
int pic_mlp_set_params(pic_mlp* m, const float* params);
/* Copies the FP32 parameter vector out (host or device). Synchronises. */
int pic_mlp_get_params(pic_mlp* m, float* params);
/* y = network(x). Asynchronous. */
int pic_mlp_forward(pic_mlp* m, const float* x, int batch, float* y);
/* Loss and gradient of the mean squared error between network(x) and
 * target over the batch; kept in the network (pic_mlp_get_grad,
 * pic_mlp_get_loss). Asynchronous. */
int pic_mlp_grad(pic_mlp* m, const float* x, const float* target, int batch);
int pic_mlp_get_grad(pic_mlp* m, float* grad); /* host or device; synchronises */
int pic_mlp_get_loss(pic_mlp* m, float* loss); /* host; synchronises */
/* One AdamW step with the kept gradient: m = b1 m + (1-b1) g,
 * v = b2 v + (1-b2) g^2, w -= lr (m/(1-b1^t) / (sqrt(v/(1-b2^t)) + eps) + wd w),
 * t counting the steps since pic_mlp_set_params. Asynchronous. */
int pic_mlp_adam(pic_mlp* m, float lr, float beta1, float beta2, float eps, float weight_decay);
/* pic_mlp_grad then pic_mlp_adam. */
int pic_mlp_train_step(pic_mlp* m, const float* x, const float* target, int batch, float lr,
                       float beta1, float beta2, float eps, float weight_decay);
/* Synchronises the stream and releases the host metadata. */
void pic_mlp_free(pic_mlp* m);

/* ---- forward pass for callers that cannot allocate ------------------------
 * For callers that cannot allocate device memory or hold a workspace (code
 * under HIP graph capture, tight serving loops predicting start profiles,
 * harnesses that forbid allocation): y = network(x) for the parameter
 * vector `params` of a network of the given shape (the layout of
 * pic_mlp_set_params), the same arithmetic and kernels as pic_mlp_forward.
 * params, x, y: DEVICE arrays of the current device (x [batch x n_in],
 * y [batch x n_out], row-major), owned by the caller. The BF16 weight
 * copies and the hidden activations live in a fixed device array of
 * 8 MiB in the library (one per GPU, kept until the process ends); a call
 * needs 2 * (number of weights) + 3 * batch * width * 4 bytes of it, each
 * part rounded up to 256 bytes, and returns PIC_EINVAL beyond that (the
 * 6 -> 4 x 256 -> 512 network takes batches up to 2516) or for bad shapes.
 * No device memory is allocated and nothing needs clearing between calls.
 * Calls on one GPU share the array: calls that overlap in time on one GPU
 * (other streams or host threads) race and must be serialised by the
 * caller. Asynchronous on `stream`; PIC_EHIP if a launch fails. */
int pic_mlp_forward_static(int n_in, int width, int depth, int n_out, const float* params,
                           const float* x, int batch, float* y, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* LIBPIC_WARMSTART_H */
