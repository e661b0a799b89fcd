// C ABI of the warm-start network: a fully connected network with GELU
// hidden layers and a linear output layer, BF16 weights (FP32 master copy),
// FP32 activations and accumulation, mean-squared-error loss and AdamW.
// Host code only; the arithmetic runs in k_mlp.hip.
#include <cmath>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/warmstart.h"
#include "mlp_internal.h"

using namespace pic;

struct pic_mlp {
  int n_in, width, depth, n_out, max_batch;
  int nl;                      // linear layers: depth hidden + 1 output
  std::vector<int> din, dout;  // per layer
  std::vector<int64_t> w_off, b_off, wb_off;
  int64_t np, nw;
  hipStream_t stream;
  float* w;      // FP32 master parameters
  float* m;      // Adam moments
  float* v;
  float* g;      // gradient
  uint16_t* wb;  // BF16 weights
  std::vector<float*> Z, A;  // per layer: pre-activation and output [max_batch x dout]
  float* d[2];               // backward deltas [max_batch x max width]
  float* loss;
  int64_t t;                 // Adam steps taken
};

namespace {

constexpr size_t kAl = 256;
size_t al(size_t v) { return (v + kAl - 1) / kAl * kAl; }

int check_dims(int n_in, int width, int depth, int n_out, int max_batch) {
  if (n_in < 1 || n_in > 4096 || width < 1 || width > 4096 || depth < 0 || depth > 64 ||
      n_out < 1 || n_out > 4096 || max_batch < 1 || max_batch > (1 << 16))
    return PIC_EINVAL;
  return PIC_OK;
}

// Shapes and offsets of a network (no memory).
void shape(pic_mlp* m, int n_in, int width, int depth, int n_out, int max_batch) {
  m->n_in = n_in;
  m->width = width;
  m->depth = depth;
  m->n_out = n_out;
  m->max_batch = max_batch;
  m->nl = depth + 1;
  m->din.clear();
  m->dout.clear();
  m->w_off.clear();
  m->b_off.clear();
  m->wb_off.clear();
  int64_t off = 0, woff = 0;
  for (int l = 0; l < m->nl; ++l) {
    const int di = l == 0 ? n_in : width;
    const int dn = l == m->nl - 1 ? n_out : width;
    m->din.push_back(di);
    m->dout.push_back(dn);
    m->w_off.push_back(off);
    off += (int64_t)di * dn;
    m->b_off.push_back(off);
    off += dn;
    m->wb_off.push_back(woff);
    woff += (int64_t)di * dn;
  }
  m->np = off;
  m->nw = woff;
}

size_t layout(pic_mlp* m, unsigned char* base) {
  size_t o = 0;
  auto take = [&](size_t bytes) {
    unsigned char* p = base ? base + o : nullptr;
    o += al(bytes);
    return p;
  };
  const size_t P = (size_t)m->np * 4;
  m->w = reinterpret_cast<float*>(take(P));
  m->m = reinterpret_cast<float*>(take(P));
  m->v = reinterpret_cast<float*>(take(P));
  m->g = reinterpret_cast<float*>(take(P));
  m->wb = reinterpret_cast<uint16_t*>(take((size_t)m->nw * 2));
  m->Z.assign(m->nl, nullptr);
  m->A.assign(m->nl, nullptr);
  for (int l = 0; l < m->nl; ++l) {
    m->Z[l] = reinterpret_cast<float*>(take((size_t)m->max_batch * m->dout[l] * 4));
    m->A[l] = reinterpret_cast<float*>(take((size_t)m->max_batch * m->dout[l] * 4));
  }
  const int wmax = m->width > m->n_out ? (m->width > m->n_in ? m->width : m->n_in)
                                       : (m->n_out > m->n_in ? m->n_out : m->n_in);
  for (int k = 0; k < 2; ++k) m->d[k] = reinterpret_cast<float*>(take((size_t)m->max_batch * wmax * 4));
  m->loss = reinterpret_cast<float*>(take(4));
  return o;
}

#define HIP_TRY(expr)                        \
  do {                                       \
    if ((expr) != hipSuccess) return PIC_EHIP; \
  } while (0)

int refresh_bf16(pic_mlp* m) {
  for (int l = 0; l < m->nl; ++l)
    HIP_TRY(launch_to_bf16(m->w + m->w_off[l], m->wb + m->wb_off[l],
                           (int64_t)m->din[l] * m->dout[l], m->stream));
  return PIC_OK;
}

// Forward pass of `batch` rows of x; the last layer's output goes to y
// (or to the network's own buffer when y is null).
int forward(pic_mlp* m, const float* x, int batch, float* y) {
  const float* in = x;
  for (int l = 0; l < m->nl; ++l) {
    const bool last = l == m->nl - 1;
    float* out = (last && y) ? y : m->A[l];
    HIP_TRY(launch_gemm_bf16(last ? EP_BIAS : EP_BIAS_GELU, in, m->din[l], 1, m->wb + m->wb_off[l], 1,
                             m->din[l], out, m->dout[l], m->w + m->b_off[l], m->Z[l], batch,
                             m->dout[l], m->din[l], m->stream));
    in = out;
  }
  return PIC_OK;
}

}  // namespace

extern "C" {

int pic_mlp_workspace_bytes(int n_in, int width, int depth, int n_out, int max_batch,
                            uint64_t* bytes) {
  if (!bytes) return PIC_EINVAL;
  const int v = check_dims(n_in, width, depth, n_out, max_batch);
  if (v) return v;
  pic_mlp m;
  shape(&m, n_in, width, depth, n_out, max_batch);
  *bytes = layout(&m, nullptr);
  return PIC_OK;
}

int pic_mlp_init(int n_in, int width, int depth, int n_out, int max_batch, void* workspace,
                 uint64_t workspace_bytes, void* stream, pic_mlp** out) {
  if (!out) return PIC_EINVAL;
  *out = nullptr;
  const int v = check_dims(n_in, width, depth, n_out, max_batch);
  if (v) return v;
  pic_mlp* m = new (std::nothrow) pic_mlp();
  if (!m) return PIC_EINVAL;
  shape(m, n_in, width, depth, n_out, max_batch);
  if (!workspace || ((uintptr_t)workspace % kAl) != 0 || workspace_bytes < layout(m, nullptr)) {
    delete m;
    return PIC_EINVAL;
  }
  layout(m, static_cast<unsigned char*>(workspace));
  m->stream = (hipStream_t)stream;
  m->t = 0;
  *out = m;
  return PIC_OK;
}

int pic_mlp_num_params(const pic_mlp* m, int64_t* n) {
  if (!m || !n) return PIC_EINVAL;
  *n = m->np;
  return PIC_OK;
}

int pic_mlp_set_params(pic_mlp* m, const float* params) {
  if (!m || !params) return PIC_EINVAL;
  HIP_TRY(hipMemcpyAsync(m->w, params, (size_t)m->np * 4, hipMemcpyDefault, m->stream));
  HIP_TRY(hipMemsetAsync(m->m, 0, (size_t)m->np * 4, m->stream));
  HIP_TRY(hipMemsetAsync(m->v, 0, (size_t)m->np * 4, m->stream));
  m->t = 0;
  const int st = refresh_bf16(m);
  if (st) return st;
  HIP_TRY(hipStreamSynchronize(m->stream));
  return PIC_OK;
}

int pic_mlp_get_params(pic_mlp* m, float* params) {
  if (!m || !params) return PIC_EINVAL;
  HIP_TRY(hipMemcpyAsync(params, m->w, (size_t)m->np * 4, hipMemcpyDefault, m->stream));
  HIP_TRY(hipStreamSynchronize(m->stream));
  return PIC_OK;
}

int pic_mlp_forward(pic_mlp* m, const float* x, int batch, float* y) {
  if (!m || !x || !y || batch < 1 || batch > m->max_batch) return PIC_EINVAL;
  return forward(m, x, batch, y);
}

int pic_mlp_grad(pic_mlp* m, const float* x, const float* target, int batch) {
  if (!m || !x || !target || batch < 1 || batch > m->max_batch) return PIC_EINVAL;
  int st = forward(m, x, batch, nullptr);
  if (st) return st;
  const int L = m->nl - 1;
  HIP_TRY(launch_mse(m->A[L], target, (int64_t)batch * m->n_out, m->d[0], m->loss, m->stream));
  int cur = 0;
  for (int l = L; l >= 0; --l) {
    const float* dz = m->d[cur];
    const float* xin = l == 0 ? x : m->A[l - 1];
    const int di = m->din[l], dn = m->dout[l];
    // dW[o][i] = sum_b dZ[b][o] X[b][i]; db[o] = sum_b dZ[b][o]
    HIP_TRY(launch_gemm_f32(EP_STORE, dz, 1, dn, xin, di, 1, m->g + m->w_off[l], di, nullptr,
                            nullptr, dn, di, batch, m->stream));
    HIP_TRY(launch_colsum(dz, batch, dn, m->g + m->b_off[l], m->stream));
    if (l > 0) {
      // dZ_{l-1}[b][i] = (sum_o dZ[b][o] W[o][i]) gelu'(Z_{l-1}[b][i])
      HIP_TRY(launch_gemm_bf16(EP_GELU_GRAD, dz, dn, 1, m->wb + m->wb_off[l], di, 1, m->d[1 - cur],
                               di, nullptr, m->Z[l - 1], batch, di, dn, m->stream));
      cur = 1 - cur;
    }
  }
  return PIC_OK;
}

int pic_mlp_get_grad(pic_mlp* m, float* grad) {
  if (!m || !grad) return PIC_EINVAL;
  HIP_TRY(hipMemcpyAsync(grad, m->g, (size_t)m->np * 4, hipMemcpyDefault, m->stream));
  HIP_TRY(hipStreamSynchronize(m->stream));
  return PIC_OK;
}

int pic_mlp_get_loss(pic_mlp* m, float* loss) {
  if (!m || !loss) return PIC_EINVAL;
  HIP_TRY(hipMemcpyAsync(loss, m->loss, 4, hipMemcpyDeviceToHost, m->stream));
  HIP_TRY(hipStreamSynchronize(m->stream));
  return PIC_OK;
}

int pic_mlp_adam(pic_mlp* m, float lr, float beta1, float beta2, float eps, float weight_decay) {
  if (!m || !(lr >= 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
      !(eps > 0.0f) || !(weight_decay >= 0.0f))
    return PIC_EINVAL;
  m->t += 1;
  const float bc1 = (float)(1.0 - std::pow((double)beta1, (double)m->t));
  const float bc2 = (float)(1.0 - std::pow((double)beta2, (double)m->t));
  HIP_TRY(launch_adam(m->w, m->m, m->v, m->g, m->np, lr, beta1, beta2, eps, weight_decay, bc1, bc2,
                      m->stream));
  return refresh_bf16(m);
}

int pic_mlp_train_step(pic_mlp* m, const float* x, const float* target, int batch, float lr,
                       float beta1, float beta2, float eps, float weight_decay) {
  const int st = pic_mlp_grad(m, x, target, batch);
  if (st) return st;
  return pic_mlp_adam(m, lr, beta1, beta2, eps, weight_decay);
}

void pic_mlp_free(pic_mlp* m) {
  if (!m) return;
  (void)hipStreamSynchronize(m->stream);
  delete m;
}

}  // extern "C"

// ---- forward pass without a workspace -------------------------------------
// pic_mlp_forward_static keeps the BF16 weight copies and the hidden
// activations of one call in a fixed device array instead of a caller's
// workspace. Each GPU holds its own copy of the array (at its own address,
// looked up once per device) for the life of the process.

namespace {

constexpr size_t kStaticScratchBytes = (size_t)8 << 20;
constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

std::mutex g_scratch_mu;
unsigned char* g_scratch[kMaxDevices];  // device address of `scratch` per device

// The current device's copy of the array; its address is taken once per
// device, with that device current.
int scratch_here(unsigned char** out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return PIC_EINVAL;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return PIC_EHIP;
    g_scratch[dev] = static_cast<unsigned char*>(p);
  }
  *out = g_scratch[dev];
  return PIC_OK;
}

}  // namespace

extern "C" int pic_mlp_forward_static(int n_in, int width, int depth, int n_out,
                                      const float* params, const float* x, int batch, float* y,
                                      void* stream) {
  if (!params || !x || !y || batch < 1) return PIC_EINVAL;
  const int v = check_dims(n_in, width, depth, n_out, batch);
  if (v) return v;
  // scratch: BF16 weights of every layer, two hidden activation buffers
  // (alternate layers) and the pre-activations the hidden epilogue writes
  const int nl = depth + 1;
  int64_t nw = 0;
  for (int l = 0; l < nl; ++l)
    nw += (int64_t)(l == 0 ? n_in : width) * (l == nl - 1 ? n_out : width);
  const size_t act = al((size_t)batch * (size_t)width * 4);
  const size_t wb_bytes = al((size_t)nw * 2);
  if (wb_bytes + 3 * act > kStaticScratchBytes) return PIC_EINVAL;
  unsigned char* base = nullptr;
  const int st = scratch_here(&base);
  if (st) return st;
  uint16_t* wb = reinterpret_cast<uint16_t*>(base);
  float* a[2] = {reinterpret_cast<float*>(base + wb_bytes),
                 reinterpret_cast<float*>(base + wb_bytes + act)};
  float* z = reinterpret_cast<float*>(base + wb_bytes + 2 * act);
  hipStream_t s = (hipStream_t)stream;
  // the same layer loop as a network's forward pass: weights to BF16, then
  // each layer's product with its epilogue
  int64_t off = 0, woff = 0;
  const float* in = x;
  for (int l = 0; l < nl; ++l) {
    const int di = l == 0 ? n_in : width;
    const int dn = l == nl - 1 ? n_out : width;
    const bool last = l == nl - 1;
    HIP_TRY(launch_to_bf16(params + off, wb + woff, (int64_t)di * dn, s));
    float* out = last ? y : a[l & 1];
    HIP_TRY(launch_gemm_bf16(last ? EP_BIAS : EP_BIAS_GELU, in, di, 1, wb + woff, 1, di, out, dn,
                             params + off + (int64_t)di * dn, z, batch, dn, di, s));
    in = out;
    off += (int64_t)di * dn + dn;
    woff += (int64_t)di * dn;
  }
  return PIC_OK;
}
