// mlp_api.cpp -- C ABI of the warm-start network (declared in include/fdlb.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/fdlb.h"
#include "mlp_host.h"

using namespace fdlb;

namespace {
thread_local std::string m_err;
int mfail(int code, const std::string &m) { m_err = m; return code; }
size_t al(size_t x) { return (x + 255) & ~(size_t)255; }
}  // namespace

#define MCHK(expr)                                                                                   \
  do {                                                                                               \
    hipError_t e_ = (expr);                                                                          \
    if (e_ != hipSuccess) return mfail(FDLB_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

struct fdlb_mlp_ctx {
  int nin, width, depth, nout, maxb, L;
  std::vector<int> din, dout;           // per layer
  std::vector<long> woff, boff;         // parameter offsets
  std::vector<long> wboff;              // bf16 weight offsets
  long P, PW;
  hipStream_t s;
  float *p, *m, *v, *g;
  long *wmap;
  long *wmapT;                          // parameter -> BF16 transposed copy (weights only, else -1)
  uint16_t *wbT;                        // BF16 weights transposed: W_l^T [in][out] per layer
  uint16_t *wb;
  std::vector<uint16_t *> H;            // bf16 layer inputs
  std::vector<float *> Z;               // fp32 pre-activations
  uint16_t *dZb;
  float *dZf, *dH;
  double *part;
  float *loss;
  float *ksp;                           // split-K partial products of the weight gradients
  long ksp_floats;                      // its size
  long t;
};

static void shapes(int nin, int w, int depth, int nout, std::vector<int> &din, std::vector<int> &dout) {
  din.clear(); dout.clear();
  din.push_back(nin); dout.push_back(w);
  for (int i = 1; i < depth; i++) { din.push_back(w); dout.push_back(w); }
  din.push_back(w); dout.push_back(nout);
}

static size_t layout(int nin, int w, int depth, int nout, int maxb, fdlb_mlp_ctx *c, char *base) {
  std::vector<int> din, dout;
  shapes(nin, w, depth, nout, din, dout);
  const int L = (int)din.size();
  long P = 0, PW = 0;
  std::vector<long> woff(L), boff(L), wboff(L);
  for (int l = 0; l < L; l++) {
    woff[l] = P; P += (long)din[l] * dout[l];
    boff[l] = P; P += dout[l];
    wboff[l] = PW; PW += (long)din[l] * dout[l];
  }
  int maxw = nout;
  for (int l = 0; l < L; l++) maxw = std::max(maxw, std::max(din[l], dout[l]));
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += al(bytes); return base ? base + o : nullptr; };
  char *pp = take(4 * P), *pm = take(4 * P), *pv = take(4 * P), *pg = take(4 * P);
  char *pwm = take(8 * P), *pwb = take(2 * PW), *pwmt = take(8 * P), *pwbt = take(2 * PW);
  std::vector<char *> ph(L + 1), pz(L);
  for (int l = 0; l < L; l++) ph[l] = take(2 * (size_t)maxb * din[l]);
  ph[L] = nullptr;
  for (int l = 0; l < L; l++) pz[l] = take(4 * (size_t)maxb * dout[l]);
  char *pdzb = take(2 * (size_t)maxb * maxw), *pdzf = take(4 * (size_t)maxb * maxw), *pdh = take(4 * (size_t)maxb * maxw);
  char *ppart = take(8 * (size_t)MLP_LOSS_PARTS), *ploss = take(8);
  long maxio = 0;
  for (int l = 0; l < L; l++) maxio = std::max(maxio, std::max((long)din[l] * dout[l], (long)dout[l]));
  char *pksp = take(4 * (size_t)MLP_SPLITK_MAX * maxio);
  if (c) {
    c->nin = nin; c->width = w; c->depth = depth; c->nout = nout; c->maxb = maxb; c->L = L;
    c->din = din; c->dout = dout; c->woff = woff; c->boff = boff; c->wboff = wboff; c->P = P; c->PW = PW;
    c->p = (float *)pp; c->m = (float *)pm; c->v = (float *)pv; c->g = (float *)pg;
    c->wmap = (long *)pwm; c->wb = (uint16_t *)pwb;
    c->wmapT = (long *)pwmt; c->wbT = (uint16_t *)pwbt;
    c->H.resize(L); c->Z.resize(L);
    for (int l = 0; l < L; l++) { c->H[l] = (uint16_t *)ph[l]; c->Z[l] = (float *)pz[l]; }
    c->dZb = (uint16_t *)pdzb; c->dZf = (float *)pdzf; c->dH = (float *)pdh;
    c->part = (double *)ppart; c->loss = (float *)ploss; c->ksp = (float *)pksp;
    c->ksp_floats = (long)MLP_SPLITK_MAX * maxio;
  }
  return off;
}

extern "C" size_t fdlb_mlp_workspace_bytes(int nin, int width, int depth, int nout, int max_batch) {
  if (nin <= 0 || width <= 0 || depth <= 0 || nout <= 0 || max_batch <= 0) return 0;
  return layout(nin, width, depth, nout, max_batch, nullptr, nullptr);
}

extern "C" int fdlb_mlp_init(int nin, int width, int depth, int nout, int max_batch, void *ws, size_t bytes,
                             void *stream, fdlb_mlp *out) {
  if (!out) return mfail(FDLB_EINVAL, "null handle pointer");
  *out = nullptr;
  size_t need = fdlb_mlp_workspace_bytes(nin, width, depth, nout, max_batch);
  if (need == 0) return mfail(FDLB_EINVAL, "bad network shape");
  if (!ws || bytes < need) return mfail(FDLB_ENOMEM, "workspace too small: need " + std::to_string(need));
  fdlb_mlp_ctx *c = new fdlb_mlp_ctx();
  layout(nin, width, depth, nout, max_batch, c, (char *)ws);
  c->s = (hipStream_t)stream;
  c->t = 0;
  std::vector<long> wm(c->P, -1), wmt(c->P, -1);
  for (int l = 0; l < c->L; l++)
    for (long i = 0; i < (long)c->din[l] * c->dout[l]; i++) {
      const long o = i / c->din[l], k = i % c->din[l];   // W_l[o][k]
      wm[c->woff[l] + i] = c->wboff[l] + i;
      wmt[c->woff[l] + i] = c->wboff[l] + k * c->dout[l] + o;
    }
  hipError_t e = hipMemcpyAsync(c->wmap, wm.data(), 8 * c->P, hipMemcpyHostToDevice, c->s);
  if (e == hipSuccess) e = hipMemcpyAsync(c->wmapT, wmt.data(), 8 * c->P, hipMemcpyHostToDevice, c->s);
  if (e == hipSuccess) e = hipMemsetAsync(c->m, 0, 4 * c->P, c->s);
  if (e == hipSuccess) e = hipMemsetAsync(c->v, 0, 4 * c->P, c->s);
  if (e == hipSuccess) e = hipMemsetAsync(c->p, 0, 4 * c->P, c->s);
  if (e == hipSuccess) e = hipMemsetAsync(c->wb, 0, 2 * c->PW, c->s);
  if (e == hipSuccess) e = hipMemsetAsync(c->wbT, 0, 2 * c->PW, c->s);
  if (e == hipSuccess) e = hipStreamSynchronize(c->s);
  if (e != hipSuccess) { delete c; return mfail(FDLB_EHIP, hipGetErrorString(e)); }
  *out = c;
  return FDLB_OK;
}

extern "C" void fdlb_mlp_destroy(fdlb_mlp h) { delete h; }

extern "C" const char *fdlb_mlp_last_error(void) { return m_err.c_str(); }

extern "C" int fdlb_mlp_num_params(fdlb_mlp h, long *n) {
  if (!h || !n) return mfail(FDLB_EINVAL, "null argument");
  *n = h->P;
  return FDLB_OK;
}

extern "C" int fdlb_mlp_set_params(fdlb_mlp h, const float *host) {
  if (!h || !host) return mfail(FDLB_EINVAL, "null argument");
  MCHK(hipMemcpyAsync(h->p, host, 4 * h->P, hipMemcpyHostToDevice, h->s));
  MCHK(hipMemsetAsync(h->m, 0, 4 * h->P, h->s));
  MCHK(hipMemsetAsync(h->v, 0, 4 * h->P, h->s));
  MCHK(hipMemsetAsync(h->g, 0, 4 * h->P, h->s));
  // lr = 0, wd = 0 AdamW pass refreshes the BF16 copies from the masters
  MCHK(mlp_adamw(h->p, h->m, h->v, h->g, h->P, 0.f, 0.9f, 0.999f, 1e-8f, 0.f, 1.f, 1.f, h->wmap, h->wb, h->wmapT,
                 h->wbT, h->s));
  MCHK(hipMemsetAsync(h->m, 0, 4 * h->P, h->s));
  MCHK(hipMemsetAsync(h->v, 0, 4 * h->P, h->s));
  MCHK(hipStreamSynchronize(h->s));
  h->t = 0;
  return FDLB_OK;
}

extern "C" int fdlb_mlp_get_params(fdlb_mlp h, float *host) {
  if (!h || !host) return mfail(FDLB_EINVAL, "null argument");
  MCHK(hipMemcpyAsync(host, h->p, 4 * h->P, hipMemcpyDeviceToHost, h->s));
  MCHK(hipStreamSynchronize(h->s));
  return FDLB_OK;
}

static int forward(fdlb_mlp h, const float *x, int M) {
  MCHK(mlp_to_bf16(x, h->H[0], (long)M * h->nin, h->s));
  for (int l = 0; l < h->L; l++) {
    const int in = h->din[l], out = h->dout[l];
    // Z = H_l W_l^T : A = H_l [M x in], B(k, n) = W_l[n][k]
    MCHK(mlp_gemm(h->H[l], h->wb + h->wboff[l], h->Z[l], M, out, in, in, 1, 1, in, out, 0, h->s));
    const bool hidden = l + 1 < h->L;
    MCHK(mlp_bias_act(h->Z[l], h->p + h->boff[l], hidden ? h->H[l + 1] : nullptr, M, out, hidden ? 1 : 0, h->s));
  }
  return FDLB_OK;
}

extern "C" int fdlb_mlp_forward(fdlb_mlp h, const float *x_dev, int batch, float *y_dev) {
  if (!h || !x_dev || batch <= 0 || batch > h->maxb) return mfail(FDLB_EINVAL, "bad forward arguments");
  int r = forward(h, x_dev, batch);
  if (r) return r;
  if (y_dev) MCHK(hipMemcpyAsync(y_dev, h->Z[h->L - 1], 4 * (size_t)batch * h->nout, hipMemcpyDeviceToDevice, h->s));
  return FDLB_OK;
}

static int backward(fdlb_mlp h, const float *t_dev, int M) {
  const long n = (long)M * h->nout;
  MCHK(mlp_mse(h->Z[h->L - 1], t_dev, h->dZb, h->dZf, h->part, n, h->loss, h->s));
  for (int l = h->L - 1; l >= 0; l--) {
    const int in = h->din[l], out = h->dout[l];
    // dW = dZ^T H_l : A(o, m) = dZ[m][o], B(m, i) = H_l[m][i]
    MCHK(mlp_gemm_splitk(h->dZb, h->H[l], h->g + h->woff[l], out, in, M, 1, out, in, 1, in, 0, h->ksp, h->s));
    // the output layer's bias gradient from the FP32 dY of the loss; the hidden
    // layers' ones come with their dZ below
    if (l == h->L - 1) MCHK(mlp_colsum(h->dZf, h->g + h->boff[l], M, out, h->ksp, h->s));
    if (l > 0) {
      // dH = dZ W_l : A = dZ [M x out], B(o, i) = W_l[o][i] = W_l^T[i][o], read from
      // the transposed copy so that both operands are contiguous along the depth
      MCHK(mlp_gemm(h->dZb, h->wbT + h->wboff[l], h->dH, M, in, out, out, 1, 1, out, in, 0, h->s));
      // dZ_{l-1} = dH * GELU'(Z_{l-1}) and the bias gradient of layer l - 1
      MCHK(mlp_gelu_bwd_colsum(h->dH, h->Z[l - 1], h->dZb, h->g + h->boff[l - 1], M, in, h->ksp,
                               (int)std::min<long>(64, h->ksp_floats / in), h->s));
    }
  }
  return FDLB_OK;
}

extern "C" int fdlb_mlp_loss_grad(fdlb_mlp h, const float *x_dev, const float *t_dev, int batch, float *loss_host,
                                  float *grad_host) {
  if (!h || !x_dev || !t_dev || batch <= 0 || batch > h->maxb) return mfail(FDLB_EINVAL, "bad arguments");
  int r = forward(h, x_dev, batch);
  if (!r) r = backward(h, t_dev, batch);
  if (r) return r;
  if (loss_host) MCHK(hipMemcpyAsync(loss_host, h->loss, 4, hipMemcpyDeviceToHost, h->s));
  if (grad_host) MCHK(hipMemcpyAsync(grad_host, h->g, 4 * h->P, hipMemcpyDeviceToHost, h->s));
  MCHK(hipStreamSynchronize(h->s));
  return FDLB_OK;
}

extern "C" int fdlb_mlp_train_step(fdlb_mlp h, const float *x_dev, const float *t_dev, int batch, float lr,
                                   float weight_decay, float *loss_host) {
  if (!h || !x_dev || !t_dev || batch <= 0 || batch > h->maxb) return mfail(FDLB_EINVAL, "bad arguments");
  int r = forward(h, x_dev, batch);
  if (!r) r = backward(h, t_dev, batch);
  if (r) return r;
  h->t += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - powf(b1, (float)h->t), c2 = 1.f - powf(b2, (float)h->t);
  MCHK(mlp_adamw(h->p, h->m, h->v, h->g, h->P, lr, b1, b2, 1e-8f, weight_decay, c1, c2, h->wmap, h->wb, h->wmapT,
                 h->wbT, h->s));
  if (loss_host) {
    MCHK(hipMemcpyAsync(loss_host, h->loss, 4, hipMemcpyDeviceToHost, h->s));
    MCHK(hipStreamSynchronize(h->s));
  }
  return FDLB_OK;
}

// plain GEMM through the same kernel (for checking the MFMA lane layout)
extern "C" int fdlb_mlp_gemm_bf16(const void *A, const void *B, float *C, int M, int N, int K, long sam, long sak,
                                  long sbk, long sbn, int ldc, void *stream) {
  MCHK(mlp_gemm((const uint16_t *)A, (const uint16_t *)B, C, M, N, K, sam, sak, sbk, sbn, ldc, 0, (hipStream_t)stream));
  MCHK(hipStreamSynchronize((hipStream_t)stream));
  return FDLB_OK;
}
