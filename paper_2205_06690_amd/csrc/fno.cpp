// Fourier-operator screening surrogate: parameters, buffers, forward,
// backward and Adam behind the bse_fno_* C-ABI.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "../../include/bse.h"
#include "fno_kernels.h"

using namespace bse;

namespace {

thread_local std::string f_err;
struct FFail {
  bse_status st;
};
void ffail(bse_status st, const std::string& m) {
  f_err = m;
  throw FFail{st};
}
void fchk(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
      ffail(BSE_ERR_OOM, std::string(what) + ": " + hipGetErrorString(e));
    ffail(BSE_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
  }
}
#define FCK(x) fchk((x), #x)

struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
  void alloc(size_t n) {
    if (p && n <= bytes) return;
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    if (n == 0) return;
    FCK(hipMalloc(&p, n));
    bytes = n;
  }
  ~Buf() {
    if (p) (void)hipFree(p);
  }
  float* f() const { return reinterpret_cast<float*>(p); }
  float2* c() const { return reinterpret_cast<float2*>(p); }
  double* d() const { return reinterpret_cast<double*>(p); }
};

}  // namespace

struct bse_fno {
  bse_fno_config cfg{};
  size_t ng = 0;
  int K = 0;
  hipStream_t stream = nullptr;
  // parameter layout (floats)
  size_t off_P = 0, off_p = 0, off_Q = 0, off_q0 = 0, n_params = 0;
  std::vector<size_t> off_R, off_W, off_b;
  Buf master, compute, grad, adam_m, adam_v, tw;
  int step = 0;
  int cap = 0;
  int mix_path = 0;   // per-mode channel mix: 0 matrix cores, 1 vector FMA
  std::vector<Buf> h, z, V;
  Buf s, gh_a, gh_b, work, U, GU, GV, part, gy, y, loss_part, tn;
  Buf gidx;   // sample indices of bse_fno_gather
};

namespace {

void layout(bse_fno* f) {
  const int W = f->cfg.width, ci = f->cfg.cin, L = f->cfg.layers;
  size_t o = 0;
  f->off_P = o; o += (size_t)W * ci;
  f->off_p = o; o += W;
  f->off_Q = o; o += W;
  f->off_q0 = o; o += 1;
  f->off_R.resize(L);
  f->off_W.resize(L);
  f->off_b.resize(L);
  for (int l = 0; l < L; ++l) {
    f->off_R[l] = o; o += (size_t)f->K * W * W * 2;
    f->off_W[l] = o; o += (size_t)W * W;
    f->off_b[l] = o; o += W;
  }
  f->n_params = o;
}

void ensure(bse_fno* f, int B) {
  if (B <= f->cap) return;
  const int W = f->cfg.width, L = f->cfg.layers;
  const size_t act = sizeof(float) * (size_t)B * W * f->ng;
  f->h.resize(L + 1);
  f->z.resize(L);
  f->V.resize(L);
  for (auto& b : f->h) b.alloc(act);
  for (auto& b : f->z) b.alloc(act);
  for (auto& b : f->V) b.alloc(sizeof(float2) * (size_t)B * W * f->K);
  f->s.alloc(act);
  f->gh_a.alloc(act);
  f->gh_b.alloc(act);
  f->work.alloc(sizeof(float2) * (size_t)B * W * f->ng);
  f->U.alloc(sizeof(float2) * (size_t)B * W * f->K);
  f->GU.alloc(sizeof(float2) * (size_t)B * W * f->K);
  f->GV.alloc(sizeof(float2) * (size_t)B * W * f->K);
  const int ci = f->cfg.cin;
  f->part.alloc(sizeof(float) * std::max(fno_outer_part_len(W, W, B, f->ng),
                                         fno_outer_part_len(W, std::max(ci, 1), B, f->ng)));
  f->gy.alloc(sizeof(float) * (size_t)B * f->ng);
  f->y.alloc(sizeof(float) * (size_t)B * f->ng);
  f->loss_part.alloc(sizeof(double) * 2 * (size_t)B * fno_loss_blocks(f->ng));
  f->tn.alloc(sizeof(double) * B);
  f->cap = B;
}

const float* prm(const bse_fno* f, size_t off) { return f->compute.f() + off; }

// y [B][ng] from x [B][cin][ng]; activations kept for backward
void forward(bse_fno* f, int B, const float* x, float* y) {
  const int W = f->cfg.width, L = f->cfg.layers, m = f->cfg.modes, n = f->cfg.n;
  hipStream_t st = f->stream;
  FCK(fno_pointwise(x, f->cfg.cin, prm(f, f->off_P), prm(f, f->off_p), W, nullptr, B, f->ng, 0,
                    nullptr, f->h[0].f(), st));
  for (int l = 0; l < L; ++l) {
    FCK(fno_fft_fwd(n, f->h[l].f(), B * W, f->tw.c(), m, 0, f->work.c(), f->V[l].c(), st));
    FCK(fno_spec_mix(f->V[l].c(), reinterpret_cast<const float2*>(prm(f, f->off_R[l])), B, W, f->K,
                     f->U.c(), f->mix_path, st));
    FCK(fno_fft_inv(n, f->U.c(), B * W, f->tw.c(), m, 1, f->work.c(), f->s.f(), 0, st));
    FCK(fno_pointwise(f->h[l].f(), W, prm(f, f->off_W[l]), prm(f, f->off_b[l]), W, f->s.f(), B,
                      f->ng, l < L - 1 ? 1 : 0, f->z[l].f(), f->h[l + 1].f(), st));
  }
  FCK(fno_pointwise(f->h[L].f(), W, prm(f, f->off_Q), prm(f, f->off_q0), 1, nullptr, B, f->ng, 0,
                    nullptr, y, st));
}

// loss and gradient (into f->grad)
double loss_grad(bse_fno* f, int B, const float* x, const float* t) {
  const int W = f->cfg.width, L = f->cfg.layers, m = f->cfg.modes, n = f->cfg.n, ci = f->cfg.cin;
  hipStream_t st = f->stream;
  forward(f, B, x, f->y.f());
  const int nbb = fno_loss_blocks(f->ng);
  FCK(fno_loss_partial(f->y.f(), t, B, f->ng, f->loss_part.d(), st));
  std::vector<double> lp(2 * (size_t)B * nbb);
  FCK(hipMemcpyAsync(lp.data(), f->loss_part.p, sizeof(double) * lp.size(), hipMemcpyDeviceToHost, st));
  FCK(hipStreamSynchronize(st));
  std::vector<double> tn(B, 0.0), sq(B, 0.0);
  for (int b = 0; b < B; ++b)
    for (int k = 0; k < nbb; ++k) {
      sq[b] += lp[2 * ((size_t)b * nbb + k)];
      tn[b] += lp[2 * ((size_t)b * nbb + k) + 1];
    }
  double loss = 0;
  for (int b = 0; b < B; ++b) {
    if (!(tn[b] > 0)) ffail(BSE_ERR_ARG, "target with zero norm");
    loss += sq[b] / tn[b];
  }
  loss /= B;
  FCK(hipMemcpyAsync(f->tn.p, tn.data(), sizeof(double) * B, hipMemcpyHostToDevice, st));
  FCK(fno_loss_grad(f->y.f(), t, f->tn.d(), B, f->ng, f->gy.f(), st));
  float* g = f->grad.f();
  FCK(fno_outer(f->gy.f(), 1, f->h[L].f(), W, B, f->ng, f->part.f(), g + f->off_Q, g + f->off_q0, st));
  float* gh = f->gh_a.f();
  float* gn = f->gh_b.f();
  FCK(fno_proj_bwd(f->gy.f(), prm(f, f->off_Q), W, B, f->ng, gh, st));
  for (int l = L - 1; l >= 0; --l) {
    if (l < L - 1) FCK(fno_gelu_bwd(gh, f->z[l].f(), (size_t)B * W * f->ng, st));
    FCK(fno_outer(gh, W, f->h[l].f(), W, B, f->ng, f->part.f(), g + f->off_W[l], g + f->off_b[l], st));
    FCK(fno_fft_fwd(n, gh, B * W, f->tw.c(), m, 1, f->work.c(), f->GU.c(), st));
    FCK(fno_spec_mix_bwd(f->V[l].c(), f->GU.c(), reinterpret_cast<const float2*>(prm(f, f->off_R[l])),
                         B, W, f->K, f->GV.c(), reinterpret_cast<float2*>(g + f->off_R[l]), f->mix_path,
                         st));
    FCK(fno_fft_inv(n, f->GV.c(), B * W, f->tw.c(), m, 0, f->work.c(), gn, 0, st));
    FCK(fno_pointwise_bwd(gh, W, prm(f, f->off_W[l]), W, B, f->ng, gn, st));
    std::swap(gh, gn);
  }
  FCK(fno_outer(gh, W, x, ci, B, f->ng, f->part.f(), g + f->off_P, g + f->off_p, st));
  return loss;
}

void check_batch(bse_fno* f, int B) {
  if (!f) ffail(BSE_ERR_ARG, "null surrogate");
  if (B < 1 || B > f->cfg.max_batch) ffail(BSE_ERR_ARG, "batch size outside 1..max_batch");
  ensure(f, B);
}

#define FAPI_BEGIN try {
#define FAPI_END                    \
  }                                 \
  catch (const FFail& e) {          \
    return e.st;                    \
  }                                 \
  catch (const std::exception& e) { \
    f_err = e.what();               \
    return BSE_ERR_DEVICE;          \
  }                                 \
  return BSE_OK;

}  // namespace

extern "C" {

const char* bse_fno_last_error(void) { return f_err.c_str(); }

bse_status bse_fno_create(const bse_fno_config* cfg, bse_fno** out) {
  FAPI_BEGIN
  if (!cfg || !out) ffail(BSE_ERR_ARG, "null argument");
  *out = nullptr;
  const bse_fno_config& c = *cfg;
  if (!fno_grid_supported(c.n)) ffail(BSE_ERR_ARG, "unsupported grid (16, 32 or 64)");
  if (c.cin < 1 || c.cin > 64 || c.width < 1 || c.width > 64 || c.layers < 1 || c.modes < 1 ||
      2 * c.modes > c.n || c.max_batch < 1)
    ffail(BSE_ERR_ARG, "bad surrogate configuration");
  FCK(hipSetDevice(c.device));
  auto* f = new bse_fno();
  try {
    f->cfg = c;
    f->ng = (size_t)c.n * c.n * c.n;
    f->K = (2 * c.modes) * (2 * c.modes) * c.modes;
    layout(f);
    f->master.alloc(sizeof(float) * f->n_params);
    f->compute.alloc(sizeof(float) * f->n_params);
    f->grad.alloc(sizeof(float) * f->n_params);
    f->adam_m.alloc(sizeof(float) * f->n_params);
    f->adam_v.alloc(sizeof(float) * f->n_params);
    // initial parameters: uniform ranges of the usual operator-network init
    std::vector<float> p(f->n_params, 0.f);
    std::mt19937_64 rng(c.seed);
    std::uniform_real_distribution<double> U(-1.0, 1.0), U01(0.0, 1.0);
    const int W = c.width;
    for (size_t i = 0; i < (size_t)W * c.cin; ++i) p[f->off_P + i] = (float)(U(rng) / std::sqrt((double)c.cin));
    for (int i = 0; i < W; ++i) p[f->off_Q + i] = (float)(U(rng) / std::sqrt((double)W));
    for (int l = 0; l < c.layers; ++l) {
      const double sc = 1.0 / ((double)W * W);
      for (size_t i = 0; i < (size_t)f->K * W * W * 2; ++i) p[f->off_R[l] + i] = (float)(sc * U01(rng));
      for (size_t i = 0; i < (size_t)W * W; ++i) p[f->off_W[l] + i] = (float)(U(rng) / std::sqrt((double)W));
    }
    FCK(hipMemcpy(f->master.p, p.data(), sizeof(float) * f->n_params, hipMemcpyHostToDevice));
    FCK(fno_round_copy(f->master.f(), f->compute.f(), f->n_params, c.bf16_weights, nullptr));
    FCK(hipMemset(f->adam_m.p, 0, sizeof(float) * f->n_params));
    FCK(hipMemset(f->adam_v.p, 0, sizeof(float) * f->n_params));
    std::vector<float2> tw(c.n);
    for (int q = 0; q < c.n; ++q) {
      const double a = -2.0 * M_PI * q / c.n;
      tw[q] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
    f->tw.alloc(sizeof(float2) * c.n);
    FCK(hipMemcpy(f->tw.p, tw.data(), sizeof(float2) * c.n, hipMemcpyHostToDevice));
    fno_configure(c.n);
    FCK(hipDeviceSynchronize());
  } catch (...) {
    delete f;
    throw;
  }
  *out = f;
  FAPI_END
}

int64_t bse_fno_num_params(const bse_fno* f) { return f ? (int64_t)f->n_params : -1; }
int32_t bse_fno_max_batch(const bse_fno* f) { return f ? f->cfg.max_batch : 0; }

bse_status bse_fno_set_params(bse_fno* f, const float* host) {
  FAPI_BEGIN
  if (!f || !host) ffail(BSE_ERR_ARG, "null argument");
  FCK(hipMemcpy(f->master.p, host, sizeof(float) * f->n_params, hipMemcpyHostToDevice));
  FCK(fno_round_copy(f->master.f(), f->compute.f(), f->n_params, f->cfg.bf16_weights, f->stream));
  FCK(hipMemsetAsync(f->adam_m.p, 0, sizeof(float) * f->n_params, f->stream));
  FCK(hipMemsetAsync(f->adam_v.p, 0, sizeof(float) * f->n_params, f->stream));
  FCK(hipStreamSynchronize(f->stream));
  f->step = 0;
  FAPI_END
}

bse_status bse_fno_get_params(bse_fno* f, float* host, int32_t which) {
  FAPI_BEGIN
  if (!f || !host || (which != 0 && which != 1)) ffail(BSE_ERR_ARG, "bad argument");
  FCK(hipStreamSynchronize(f->stream));
  FCK(hipMemcpy(host, which ? f->compute.p : f->master.p, sizeof(float) * f->n_params,
                hipMemcpyDeviceToHost));
  FAPI_END
}

bse_status bse_fno_set_stream(bse_fno* f, void* st) {
  FAPI_BEGIN
  if (!f) ffail(BSE_ERR_ARG, "null surrogate");
  f->stream = reinterpret_cast<hipStream_t>(st);
  FAPI_END
}

bse_status bse_fno_set_mix_path(bse_fno* f, int32_t path) {
  FAPI_BEGIN
  if (!f) ffail(BSE_ERR_ARG, "null surrogate");
  if (path != 0 && path != 1) ffail(BSE_ERR_ARG, "bse_fno_set_mix_path: path 0 or 1");
  f->mix_path = path;
  FAPI_END
}

bse_status bse_fno_forward(bse_fno* f, int32_t B, const void* x_dev, void* y_dev) {
  FAPI_BEGIN
  check_batch(f, B);
  if (!x_dev || !y_dev) ffail(BSE_ERR_ARG, "null buffer");
  forward(f, B, reinterpret_cast<const float*>(x_dev), reinterpret_cast<float*>(y_dev));
  FCK(hipStreamSynchronize(f->stream));
  FAPI_END
}

bse_status bse_fno_loss_grad(bse_fno* f, int32_t B, const void* x_dev, const void* t_dev,
                             double* loss, float* grad_host) {
  FAPI_BEGIN
  check_batch(f, B);
  if (!x_dev || !t_dev || !loss) ffail(BSE_ERR_ARG, "null buffer");
  *loss = loss_grad(f, B, reinterpret_cast<const float*>(x_dev), reinterpret_cast<const float*>(t_dev));
  if (grad_host)
    FCK(hipMemcpyAsync(grad_host, f->grad.p, sizeof(float) * f->n_params, hipMemcpyDeviceToHost,
                       f->stream));
  FCK(hipStreamSynchronize(f->stream));
  FAPI_END
}

bse_status bse_fno_train_step(bse_fno* f, int32_t B, const void* x_dev, const void* t_dev, double lr,
                              double* loss) {
  FAPI_BEGIN
  check_batch(f, B);
  if (!x_dev || !t_dev || !loss || !(lr > 0)) ffail(BSE_ERR_ARG, "bad argument");
  *loss = loss_grad(f, B, reinterpret_cast<const float*>(x_dev), reinterpret_cast<const float*>(t_dev));
  f->step += 1;
  FCK(fno_adam(f->master.f(), f->compute.f(), f->grad.f(), f->adam_m.f(), f->adam_v.f(), f->n_params,
               (float)lr, 0.9f, 0.999f, 1e-8f, f->step, f->cfg.bf16_weights, f->stream));
  FCK(hipStreamSynchronize(f->stream));
  FAPI_END
}

void bse_fno_destroy(bse_fno* f) {
  if (!f) return;
  (void)hipSetDevice(f->cfg.device);
  delete f;
}

bse_status bse_fno_gather(bse_fno* f, int32_t B, const int32_t* idx, int32_t n_src, const void* x_src,
                          const void* t_src, const int32_t* perm, int32_t flip_mask, void* x_dst, void* t_dst) {
  FAPI_BEGIN
  check_batch(f, B);
  if (!idx || !perm || !x_src || !t_src || !x_dst || !t_dst) ffail(BSE_ERR_ARG, "null argument");
  for (int b = 0; b < B; ++b)
    if (idx[b] < 0 || idx[b] >= n_src) ffail(BSE_ERR_ARG, "sample index outside 0..n_src-1");
  bool seen[3] = {false, false, false};
  for (int k = 0; k < 3; ++k) {
    if (perm[k] < 0 || perm[k] > 2 || seen[perm[k]]) ffail(BSE_ERR_ARG, "perm is not a permutation of 0, 1, 2");
    seen[perm[k]] = true;
  }
  if (flip_mask < 0 || flip_mask > 7) ffail(BSE_ERR_ARG, "flip_mask outside 0..7");
  const int pm[3] = {perm[0], perm[1], perm[2]};
  f->gidx.alloc(sizeof(int) * (size_t)f->cfg.max_batch);
  FCK(hipMemcpyAsync(f->gidx.p, idx, sizeof(int) * B, hipMemcpyHostToDevice, f->stream));
  const int n = f->cfg.n;
  FCK(fno_gather_sym(reinterpret_cast<const float*>(x_src), reinterpret_cast<const int*>(f->gidx.p), B,
                     f->cfg.cin, n, pm, flip_mask, reinterpret_cast<float*>(x_dst), f->stream));
  FCK(fno_gather_sym(reinterpret_cast<const float*>(t_src), reinterpret_cast<const int*>(f->gidx.p), B, 1, n,
                     pm, flip_mask, reinterpret_cast<float*>(t_dst), f->stream));
  FCK(hipStreamSynchronize(f->stream));
  FAPI_END
}

}  // extern "C"
