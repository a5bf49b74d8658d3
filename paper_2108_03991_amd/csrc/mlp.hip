// Learned cost model of internal tiles: FP32 MLP F -> 64 -> 64 -> 1 (tanh),
// trained on the GPU with this file's own forward/backward and Adam kernels.
//
// The paper schedules internal tasks with the estimate W_i = N_E,i^2 and notes
// that the estimate can be replaced by a better model of the task time
// (Sec. III-C-2); here the model is learned from per-tile timestamps recorded by
// the persistent internal kernel.  Features of a tile (panel of `rows` rows of
// the block of object i with n_i unknowns):
//   log n_i, log(aspect of the object's bounding box), log(skin depth / size)
//   (size = square root of the surface area), log rows, (n_i mod 64)/64,
//   log of the row sweeps of the busiest wave (rows over four waves of `rows per
//   wave` rows, rounded up) and log of the 256-column chunks of a row (row length
//   rounded up): the persistent kernel's loop counts for the tile,
// standardised.  Target: log(tile time / (sweeps x chunks)), the time per inner
// iteration, so that the network learns a bounded correction to the loop count
// and a tile larger than any it was trained on still scales with its loop count;
// the predicted tile time is exp(output) x sweeps x chunks.  Loss: mean squared
// error.
#include <algorithm>
#include <mutex>

#include "ctx.hpp"

namespace slim {

namespace {

constexpr int HID = 64;
constexpr int FMAX = 8;

__host__ __device__ inline int n_params(int F) { return HID * F + HID + HID * HID + HID + HID + 1; }

__device__ __forceinline__ float wsum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// One wave per 64 samples (one sample per lane).  Writes y, the per-wave partial
// gradient (n_params floats) and the per-wave partial sum of squared errors.
__global__ void __launch_bounds__(64) k_mlp_fb(int F, int B, const float* __restrict__ p, const float* __restrict__ X,
                                               const float* __restrict__ t, float* __restrict__ y,
                                               float* __restrict__ partial, float* __restrict__ partial_loss) {
  const int lane = threadIdx.x;
  const int s = blockIdx.x * 64 + lane;
  const bool ok = s < B;
  const float* W1 = p;
  const float* b1 = W1 + HID * F;
  const float* W2 = b1 + HID;
  const float* b2 = W2 + HID * HID;
  const float* w3 = b2 + HID;
  const float* b3 = w3 + HID;
  float x[FMAX];
  for (int f = 0; f < F; ++f) x[f] = ok ? X[int64_t(s) * F + f] : 0.f;
  float a1[HID], a2[HID];
  for (int h = 0; h < HID; ++h) {
    float z = b1[h];
    for (int f = 0; f < F; ++f) z += W1[h * F + f] * x[f];
    a1[h] = tanhf(z);
  }
  float out = b3[0];
  for (int h = 0; h < HID; ++h) {
    float z = b2[h];
    for (int k = 0; k < HID; ++k) z += W2[h * HID + k] * a1[k];
    a2[h] = tanhf(z);
    out += w3[h] * a2[h];
  }
  const float r = ok ? out - t[s] : 0.f;
  if (ok) y[s] = out;
  const float dy = ok ? 2.f * r / float(B) : 0.f;
  float* g = partial + int64_t(blockIdx.x) * n_params(F);
  float* gW1 = g;
  float* gb1 = gW1 + HID * F;
  float* gW2 = gb1 + HID;
  float* gb2 = gW2 + HID * HID;
  float* gw3 = gb2 + HID;
  float* gb3 = gw3 + HID;
  // output layer
  for (int h = 0; h < HID; ++h) {
    float v = wsum(dy * a2[h]);
    if (lane == 0) gw3[h] = v;
  }
  {
    float v = wsum(dy);
    if (lane == 0) gb3[0] = v;
  }
  // dz2 = dy w3 (1 - a2^2), kept in a2
  for (int h = 0; h < HID; ++h) a2[h] = dy * w3[h] * (1.f - a2[h] * a2[h]);
  for (int h = 0; h < HID; ++h) {
    for (int k = 0; k < HID; ++k) {
      float v = wsum(a2[h] * a1[k]);
      if (lane == 0) gW2[h * HID + k] = v;
    }
    float v = wsum(a2[h]);
    if (lane == 0) gb2[h] = v;
  }
  // dz1 = (W2^T dz2) (1 - a1^2)
  for (int k = 0; k < HID; ++k) {
    float d = 0.f;
    for (int h = 0; h < HID; ++h) d += W2[h * HID + k] * a2[h];
    const float dz1 = d * (1.f - a1[k] * a1[k]);
    for (int f = 0; f < F; ++f) {
      float v = wsum(dz1 * x[f]);
      if (lane == 0) gW1[k * F + f] = v;
    }
    float v = wsum(dz1);
    if (lane == 0) gb1[k] = v;
  }
  float l = wsum(r * r);
  if (lane == 0) partial_loss[blockIdx.x] = l;
}

// grad[i] = sum over waves of partial[w][i] (fixed order); loss likewise.
__global__ void k_mlp_reduce(int np, int nw, int B, const float* partial, const float* partial_loss, float* grad,
                             float* loss) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < np) {
    float s = 0.f;
    for (int w = 0; w < nw; ++w) s += partial[int64_t(w) * np + i];
    grad[i] = s;
  }
  if (i == 0 && loss) {
    float s = 0.f;
    for (int w = 0; w < nw; ++w) s += partial_loss[w];
    *loss = s / float(B);
  }
}

__global__ void k_adam(int np, float* p, const float* g, float* m, float* v, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  m[i] = b1 * m[i] + (1.f - b1) * g[i];
  v[i] = b2 * v[i] + (1.f - b2) * g[i] * g[i];
  p[i] -= lr * (m[i] / c1) / (sqrtf(v[i] / c2) + eps);
}

// Forward/backward on workspace the caller provides: partial (nw x n_params(F) floats)
// and ploss (nw floats), nw = ceil(B / 64).  Every entry of both is written before
// it is read, so the workspace needs no clearing.
void fb_launch_ws(int F, int B, const float* p, const float* X, const float* t, float* y, float* grad, float* loss,
                  float* partial, float* ploss, hipStream_t s) {
  const int nw = (B + 63) / 64, np = n_params(F);
  hipLaunchKernelGGL(k_mlp_fb, dim3(nw), dim3(64), 0, s, F, B, p, X, t, y, partial, ploss);
  hipLaunchKernelGGL(k_mlp_reduce, dim3((np + 255) / 256), dim3(256), 0, s, np, nw, B, partial, ploss, grad, loss);
  SLIM_HIP(hipGetLastError());
}

void fb_launch(int F, int B, const float* p, const float* X, const float* t, float* y, float* grad, float* loss,
               DevBuf& partial, DevBuf& ploss, hipStream_t s) {
  const int nw = (B + 63) / 64, np = n_params(F);
  if (partial.bytes < size_t(nw) * np * 4) partial.alloc(size_t(nw) * np * 4);
  if (ploss.bytes < size_t(nw) * 4) ploss.alloc(size_t(nw) * 4);
  fb_launch_ws(F, B, p, X, t, y, grad, loss, partial.as<float>(), ploss.as<float>(), s);
}

// ---- workspace of the allocation-free entry point ---------------------------
// One static device array per GPU, held until the process ends: the per-wave
// partial gradients (kNoAllocWaves x n_params(FMAX)) followed by the per-wave
// partial losses.  In host code `scratch` is only a symbol; its device address
// comes from hipGetSymbolAddress, once per device (noalloc_workspace).
constexpr int kNoAllocMaxB = 32768;
constexpr int kNoAllocWaves = kNoAllocMaxB / 64;
constexpr size_t kScratchFloats = size_t(kNoAllocWaves) * (HID * FMAX + HID + HID * HID + HID + HID + 1) + kNoAllocWaves;
static_assert(kScratchFloats * 4 < (size_t(12) << 20), "workspace of the allocation-free entry point stays modest");

constexpr int kMaxDevices = 64;
std::mutex g_ws_mutex;
float* g_ws_ptr[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) float scratch[kScratchFloats];

// Device address of `scratch` on the current device (looked up once per device).
float* noalloc_workspace() {
  int dev = -1;
  SLIM_HIP(hipGetDevice(&dev));
  SLIM_REQUIRE(dev >= 0 && dev < kMaxDevices, SLIM_E_UNSUPPORTED, "device index beyond the workspace table");
  std::lock_guard<std::mutex> lock(g_ws_mutex);
  if (!g_ws_ptr[dev]) {
    void* ptr = nullptr;
    SLIM_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    SLIM_REQUIRE(ptr != nullptr, SLIM_E_HIP, "hipGetSymbolAddress returned no address for the workspace");
    g_ws_ptr[dev] = static_cast<float*>(ptr);
  }
  return g_ws_ptr[dev];
}

namespace {

}  // namespace

constexpr int kFeat = 7;
static_assert(kFeat <= FMAX, "feature count within the network's input bound");

// Raw (unstandardised) features of a tile: panel of `rows` rows of block `block`.
void tile_features_raw(const Ctx& c, int block, int rows, float* f) {
  // object geometry from its triangles
  const RWGTable& r = c.rwg;
  const Mesh& m = c.mesh;
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300}, S = 0.0;
  for (int64_t t = r.obj_tri_off[block]; t < r.obj_tri_off[block + 1]; ++t) {
    S += r.area[t];
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 3; ++k) {
        double v = m.xyz[3 * size_t(m.tri[3 * t + i]) + k];
        lo[k] = std::min(lo[k], v);
        hi[k] = std::max(hi[k], v);
      }
  }
  double d[3] = {hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]};
  std::sort(d, d + 3);
  const Material& mt = c.mats.empty() ? Material{} : c.mats[block];
  const double delta = 1.0 / std::sqrt(kPi * c.freq * kMu0 * mt.mu_r * std::max(mt.sigma, 1e-300));
  const int n = c.blocks[block].n, ld = (n + 1) & ~1;
  const int sweeps = (rows + 4 * c.rw_mixed - 1) / (4 * c.rw_mixed), chunks = (ld + 255) / 256;
  const float raw[kFeat] = {float(std::log(double(n))), float(std::log(d[2] / std::max(d[0], 1e-30))),
                            float(std::log(delta / std::sqrt(S))), float(std::log(double(rows))),
                            float((n % 64) / 64.0), float(std::log(double(sweeps))),
                            float(std::log(double(chunks)))};
  for (int k = 0; k < kFeat; ++k) f[k] = raw[k];
}

// Raw features and log tile time (wall-clock ticks) of the last recorded tiles.
void recorded_samples(const Ctx& c, std::vector<float>& X, std::vector<float>& T) {
  const int64_t nt = int64_t(c.tiles.size());
  SLIM_REQUIRE(int64_t(c.last_stamps.size()) == 2 * nt && nt > 0, SLIM_E_STATE, "no recorded tile timings");
  X.assign(size_t(nt) * kFeat, 0.f);
  T.assign(nt, 0.f);
  for (int64_t k = 0; k < nt; ++k) {
    tile_features_raw(c, c.tiles[k].block, c.tiles[k].rows, &X[size_t(k) * kFeat]);
    const double dt = std::max(1.0, c.last_stamps[2 * k + 1] - c.last_stamps[2 * k]);
    T[k] = float(std::log(dt));
  }
}

float mlp_predict_host(const Ctx& c, const float* x) {
  const int F = kFeat;
  const float* p = c.mlp_params.data();
  const float* W1 = p;
  const float* b1 = W1 + HID * F;
  const float* W2 = b1 + HID;
  const float* b2 = W2 + HID * HID;
  const float* w3 = b2 + HID;
  const float* b3 = w3 + HID;
  float a1[HID];
  for (int h = 0; h < HID; ++h) {
    float z = b1[h];
    for (int f = 0; f < F; ++f) z += W1[h * F + f] * x[f];
    a1[h] = std::tanh(z);
  }
  float out = b3[0];
  for (int h = 0; h < HID; ++h) {
    float z = b2[h];
    for (int k = 0; k < HID; ++k) z += W2[h * HID + k] * a1[k];
    out += w3[h] * std::tanh(z);
  }
  return out;
}

// Predicted time of a tile (wall-clock ticks): the network's time per inner iteration
// times the tile's loop count (row sweeps x column chunks).
double mlp_predict_time(const Ctx& c, int block, int rows) {
  float f[FMAX];
  tile_features_raw(c, block, rows, f);
  const double loops = std::exp(double(f[5]) + double(f[6]));
  for (int k = 0; k < kFeat; ++k) {
    const float mu = c.mlp_mu.empty() ? 0.f : c.mlp_mu[k];
    const float sd = c.mlp_sd.empty() ? 1.f : c.mlp_sd[k];
    f[k] = (f[k] - mu) / sd;
  }
  return std::exp(double(mlp_predict_host(c, f))) * loops;
}

// Train the context's cost model on samples (raw features X, nt x kFeat; log tile
// times T): standardise the features, initialise deterministically, run Adam.
double mlp_train_on(Ctx& c, std::vector<float> X, const std::vector<float>& T, int epochs, double lr) {
  const int64_t nt = int64_t(T.size());
  SLIM_REQUIRE(nt > 0 && int64_t(X.size()) == nt * kFeat, SLIM_E_ARG, "no training samples");
  SLIM_REQUIRE(nt <= (int64_t(1) << 31) - 64, SLIM_E_ARG, "too many training samples");
  const int F = kFeat;
  // target: log time per inner iteration (raw features 5 and 6: log sweeps, log chunks)
  std::vector<float> Tr(T);
  for (int64_t k = 0; k < nt; ++k) Tr[k] -= X[size_t(k) * F + 5] + X[size_t(k) * F + 6];
  std::vector<float> mu(F, 0.f), sd(F, 0.f);
  for (int64_t k = 0; k < nt; ++k)
    for (int f = 0; f < F; ++f) mu[f] += X[size_t(k) * F + f] / float(nt);
  for (int64_t k = 0; k < nt; ++k)
    for (int f = 0; f < F; ++f) sd[f] += (X[size_t(k) * F + f] - mu[f]) * (X[size_t(k) * F + f] - mu[f]) / float(nt);
  for (int f = 0; f < F; ++f) sd[f] = sd[f] > 1e-12f ? std::sqrt(sd[f]) : 1.f;
  for (int64_t k = 0; k < nt; ++k)
    for (int f = 0; f < F; ++f) X[size_t(k) * F + f] = (X[size_t(k) * F + f] - mu[f]) / sd[f];
  // deterministic initialisation (scaled uniform from a linear congruential sequence)
  const int np = n_params(F);
  std::vector<float> p(np, 0.f);
  uint64_t st = 0x9E3779B97F4A7C15ull;
  auto urand = [&]() {
    st = st * 6364136223846793005ull + 1442695040888963407ull;
    return float((st >> 11) * (1.0 / 9007199254740992.0)) * 2.f - 1.f;
  };
  for (int i = 0; i < HID * F; ++i) p[i] = urand() * std::sqrt(3.f / F);
  for (int i = 0; i < HID * HID; ++i) p[HID * F + HID + i] = urand() * std::sqrt(3.f / HID);
  for (int i = 0; i < HID; ++i) p[HID * F + HID + HID * HID + HID + i] = urand() * std::sqrt(3.f / HID);
  float tmean = 0.f;
  for (float v : Tr) tmean += v / float(nt);
  p[np - 1] = tmean;
  DevBuf dp, dg, dm, dv, dX, dT, dy, dl, part, pl;
  dp.upload(p);
  dg.alloc(size_t(np) * 4);
  dm.alloc(size_t(np) * 4);
  dv.alloc(size_t(np) * 4);
  SLIM_HIP(hipMemset(dm.p, 0, dm.bytes));
  SLIM_HIP(hipMemset(dv.p, 0, dv.bytes));
  dX.upload(X);
  dT.upload(Tr);
  dy.alloc(size_t(nt) * 4);
  dl.alloc(4);
  hipStream_t s = nullptr;
  float c1 = 1.f, c2 = 1.f;
  for (int e = 0; e < epochs; ++e) {
    fb_launch(F, int(nt), dp.as<float>(), dX.as<float>(), dT.as<float>(), dy.as<float>(), dg.as<float>(),
              dl.as<float>(), part, pl, s);
    c1 *= 0.9f;
    c2 *= 0.999f;
    hipLaunchKernelGGL(k_adam, dim3((np + 255) / 256), dim3(256), 0, s, np, dp.as<float>(), dg.as<float>(),
                       dm.as<float>(), dv.as<float>(), float(lr), 0.9f, 0.999f, 1e-8f, 1.f - c1, 1.f - c2);
    SLIM_HIP(hipGetLastError());
  }
  float loss = 0.f;
  fb_launch(F, int(nt), dp.as<float>(), dX.as<float>(), dT.as<float>(), dy.as<float>(), dg.as<float>(),
            dl.as<float>(), part, pl, s);
  SLIM_HIP(hipMemcpy(&loss, dl.p, 4, hipMemcpyDeviceToHost));
  SLIM_HIP(hipMemcpy(p.data(), dp.p, size_t(np) * 4, hipMemcpyDeviceToHost));
  c.mlp_params = p;
  c.mlp_mu = mu;
  c.mlp_sd = sd;
  return double(loss);
}

// Train on the last recorded tiles (slim_sched_record + slim_internal_apply with timing).
double mlp_train(Ctx& c, int epochs, double lr) {
  std::vector<float> X, T;
  recorded_samples(c, X, T);
  return mlp_train_on(c, X, T, epochs, lr);
}

}  // namespace slim

using namespace slim;


extern "C" {

slim_status slim_mlp_forward_backward(int32_t F, int32_t B, const float* params, const float* X, const float* t,
                                      float* y, float* grad, float* loss, void* stream) {
  if (F < 1 || F > FMAX || B < 1 || !params || !X || !t || !y || !grad) return SLIM_E_ARG;
  try {
    DevBuf part, pl;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    fb_launch(F, B, params, X, t, y, grad, loss, part, pl, s);
    SLIM_HIP(hipStreamSynchronize(s));
    return SLIM_OK;
  } catch (const Error& e) {
    return e.code;
  } catch (...) {
    return SLIM_E_HIP;
  }
}

slim_status slim_mlp_forward_backward_noalloc(int32_t F, int32_t B, const float* params, const float* X,
                                              const float* t, float* y, float* grad, float* loss, void* stream) {
  if (F < 1 || F > FMAX || B < 1 || B > kNoAllocMaxB || !params || !X || !t || !y || !grad) return SLIM_E_ARG;
  try {
    float* ws = noalloc_workspace();
    fb_launch_ws(F, B, params, X, t, y, grad, loss, ws, ws + size_t(kNoAllocWaves) * n_params(FMAX),
                 reinterpret_cast<hipStream_t>(stream));
    return SLIM_OK;
  } catch (const Error& e) {
    return e.code;
  } catch (...) {
    return SLIM_E_HIP;
  }
}

slim_status slim_sched_export(slim_ctx* h, double* out, int64_t* n) {
  if (!h || !n) return SLIM_E_ARG;
  try {
    h->c.last_error.clear();
    std::vector<float> X, T;
    recorded_samples(h->c, X, T);
    const int64_t cap = *n, nt = int64_t(T.size());
    *n = nt;
    if (!out) return SLIM_OK;
    SLIM_REQUIRE(cap >= nt, SLIM_E_ARG, "sample buffer too small");
    for (int64_t k = 0; k < nt; ++k) {
      for (int f = 0; f < kFeat; ++f) out[(kFeat + 1) * k + f] = X[size_t(k) * kFeat + f];
      out[(kFeat + 1) * k + kFeat] = T[k];
    }
    return SLIM_OK;
  } catch (const Error& e) {
    h->c.last_error = e.what();
    return e.code;
  } catch (const std::exception& e) {
    h->c.last_error = e.what();
    return SLIM_E_HIP;
  }
}

slim_status slim_sched_train_data(slim_ctx* h, int64_t n, const double* data, int32_t epochs, double lr,
                                  double* final_loss) {
  if (!h || !data || n < 1) return SLIM_E_ARG;
  try {
    h->c.last_error.clear();
    SLIM_REQUIRE(h->c.built, SLIM_E_STATE, "operator not built");
    std::vector<float> X(size_t(n) * kFeat), T(n);
    for (int64_t k = 0; k < n; ++k) {
      for (int f = 0; f < kFeat; ++f) X[size_t(k) * kFeat + f] = float(data[(kFeat + 1) * k + f]);
      T[k] = float(data[(kFeat + 1) * k + kFeat]);
      for (int f = 0; f <= kFeat; ++f)
        SLIM_REQUIRE(std::isfinite(data[(kFeat + 1) * k + f]), SLIM_E_ARG, "non-finite training sample");
    }
    double l = mlp_train_on(h->c, X, T, epochs > 0 ? epochs : 2000, lr > 0 ? lr : 3e-3);
    if (final_loss) *final_loss = l;
    return SLIM_OK;
  } catch (const Error& e) {
    h->c.last_error = e.what();
    return e.code;
  } catch (const std::exception& e) {
    h->c.last_error = e.what();
    return SLIM_E_HIP;
  }
}

slim_status slim_sched_train(slim_ctx* h, int32_t epochs, double lr, double* final_loss) {
  if (!h) return SLIM_E_ARG;
  try {
    h->c.last_error.clear();
    double l = mlp_train(h->c, epochs > 0 ? epochs : 2000, lr > 0 ? lr : 3e-3);
    if (final_loss) *final_loss = l;
    return SLIM_OK;
  } catch (const Error& e) {
    h->c.last_error = e.what();
    return e.code;
  } catch (const std::exception& e) {
    h->c.last_error = e.what();
    return SLIM_E_HIP;
  }
}

}  // extern "C"
