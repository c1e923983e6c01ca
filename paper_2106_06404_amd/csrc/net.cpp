// Host side of the warm-start network (the msdd_net_* entry points of msdd.h):
// parameter storage, FP32 training passes (forward, projection loss, backward, Adam)
// and the BF16 inference pass used by the setup.  All arithmetic runs in mlp.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "common.h"
#include "host_util.h"
#include "kernels.h"
#include "msdd.h"
#include "net.h"

using namespace msdd_host;

namespace {
constexpr double kRidge = 1e-6;  // G = Ys^T Ys + ridge I in the projection loss
constexpr int kMaxVec = 16;      // the loss kernel keeps V x V and V x m blocks in LDS
}  // namespace

struct msdd_net {
  int n_in = 0, H = 0, V = 0, n_pos = 0, out = 0, device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  i64 off[7] = {0};  // W1, b1, W2, b2, W3, b3, total
  DVec<float> p, g, am, av;
  int step = 0;
  // training work (batch capacity cap_b)
  int cap_b = 0;
  DVec<float> xb, h1, h2, y, dy, d2, d1, lossb;
  DVec<float> part;
  DVec<int> idx;
  DVec<float> tmp_x, tmp_t, tmp_m;
  DVec<int> tmp_c;
  // inference (BF16 weights transposed, K padded to 16)
  int kp1 = 0, kp2 = 0;
  bool bf_stale = true;
  DVec<unsigned short> w1t, w2t, w3t;
  int cap_i = 0;
  DVec<unsigned short> xh, h1h, h2h;
  DVec<float> yi, xi;
};

namespace {

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    HIPCHK(hipSetDevice(dev));
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

int round16(int x) { return (x + 15) / 16 * 16; }

// split-K count that gives the launch about 512 workgroups
int choose_splits(int M, int N, int K) {
  const int tiles = ((M + 63) / 64) * ((N + 63) / 64);
  int s = (512 + tiles - 1) / tiles;
  s = std::min(s, std::max(1, K / 64));
  return std::max(1, s);
}

// out = epilogue(opA(A) opB(B)); mode -1: plain product, 0: + bias, 1: + bias then relu,
// 2: times relu'(h)
void gemm(msdd_net* n, hipStream_t s, int ta, int tb, int M, int N, int K, const float* A, int lda,
          const float* B, int ldb, float* out, const float* bias, const float* h, int mode) {
  int splits = sgemm_splits(K, choose_splits(M, N, K));
  if (splits == 1 && mode == -1) {
    launch_sgemm(s, ta, tb, M, N, K, 1, A, lda, B, ldb, out);
    return;
  }
  const size_t need = (size_t)splits * M * N;
  if (n->part.n < need) n->part.alloc(need);
  const int used = launch_sgemm(s, ta, tb, M, N, K, splits, A, lda, B, ldb, n->part.p);
  launch_splitk_epi(s, M, N, used, n->part.p, bias, h, mode < 0 ? 0 : mode, out);
}

void ensure_train(msdd_net* n, int B) {
  if (B <= n->cap_b) return;
  n->xb.alloc((size_t)B * n->n_in);
  n->h1.alloc((size_t)B * n->H);
  n->h2.alloc((size_t)B * n->H);
  n->y.alloc((size_t)B * n->out);
  n->dy.alloc((size_t)B * n->out);
  n->d2.alloc((size_t)B * n->H);
  n->d1.alloc((size_t)B * n->H);
  n->lossb.alloc(B);
  n->idx.alloc(B);
  n->cap_b = B;
}

const float* W1(msdd_net* n) { return n->p.p + n->off[0]; }
const float* b1(msdd_net* n) { return n->p.p + n->off[1]; }
const float* W2(msdd_net* n) { return n->p.p + n->off[2]; }
const float* b2(msdd_net* n) { return n->p.p + n->off[3]; }
const float* W3(msdd_net* n) { return n->p.p + n->off[4]; }
const float* b3(msdd_net* n) { return n->p.p + n->off[5]; }

// FP32 forward of the batch in n->xb: h1, h2, y
void forward_f32(msdd_net* n, hipStream_t s, int B) {
  gemm(n, s, 0, 0, B, n->H, n->n_in, n->xb.p, n->n_in, W1(n), n->H, n->h1.p, b1(n), nullptr, 1);
  gemm(n, s, 0, 0, B, n->H, n->H, n->h1.p, n->H, W2(n), n->H, n->h2.p, b2(n), nullptr, 1);
  gemm(n, s, 0, 0, B, n->out, n->H, n->h2.p, n->H, W3(n), n->out, n->y.p, b3(n), nullptr, 0);
}

// gradient of the loss whose dloss/dy is in n->dy, into n->g
void backward_f32(msdd_net* n, hipStream_t s, int B) {
  float* g = n->g.p;
  const int H = n->H, O = n->out, I = n->n_in;
  // W3, b3
  gemm(n, s, 1, 0, H, O, B, n->h2.p, H, n->dy.p, O, g + n->off[4], nullptr, nullptr, -1);
  launch_colsum(s, B, O, n->dy.p, g + n->off[5]);
  // dz2 = (dy W3^T) * relu'(h2)
  gemm(n, s, 0, 1, B, H, O, n->dy.p, O, W3(n), O, n->d2.p, nullptr, n->h2.p, 2);
  gemm(n, s, 1, 0, H, H, B, n->h1.p, H, n->d2.p, H, g + n->off[2], nullptr, nullptr, -1);
  launch_colsum(s, B, H, n->d2.p, g + n->off[3]);
  // dz1 = (dz2 W2^T) * relu'(h1)
  gemm(n, s, 0, 1, B, H, H, n->d2.p, H, W2(n), H, n->d1.p, nullptr, n->h1.p, 2);
  gemm(n, s, 1, 0, I, H, B, n->xb.p, I, n->d1.p, H, g + n->off[0], nullptr, nullptr, -1);
  launch_colsum(s, B, H, n->d1.p, g + n->off[1]);
}

template <class T>
const T* device_view(const T* ptr, size_t cnt, DVec<T>& tmp, hipStream_t s) {
  REQUIRE(ptr != nullptr || cnt == 0, "null array argument");
  if (is_device_ptr(ptr)) return ptr;
  to_device(tmp, ptr, cnt, s);
  return tmp.p;
}

// loss and gradient (into n->g) of samples idx of a training set; returns the mean loss
// (only when want_loss, which synchronises)
double loss_grad(msdd_net* n, int B, const int32_t* idx, int N, const float* x_all, const float* tgt,
                 const float* mask, const int32_t* cnt, int m_cap, bool want_loss) {
  hipStream_t s = n->stream;
  REQUIRE(B >= 1 && N >= 1, "batch and sample counts must be positive");
  REQUIRE(m_cap >= 1 && m_cap <= kMaxVec, "m_cap must lie in [1, 16]");
  ensure_train(n, B);
  // indices are checked on the host so that no kernel reads outside the training set
  std::vector<int32_t> hidx = to_host(idx, (size_t)B);
  for (int b = 0; b < B; ++b) REQUIRE(hidx[b] >= 0 && hidx[b] < N, "sample index out of range");
  HIPCHK(hipMemcpyAsync(n->idx.p, hidx.data(), B * sizeof(int), hipMemcpyHostToDevice, s));
  const float* dx = device_view(x_all, (size_t)N * n->n_in, n->tmp_x, s);
  const float* dt = device_view(tgt, (size_t)N * m_cap * n->n_pos, n->tmp_t, s);
  const float* dm = device_view(mask, (size_t)N * n->n_pos, n->tmp_m, s);
  const int32_t* dc = device_view(cnt, (size_t)N, n->tmp_c, s);
  launch_gather_rows(s, B, n->n_in, n->idx.p, dx, n->xb.p);
  forward_f32(n, s, B);
  launch_proj_loss(s, B, n->V, n->n_pos, m_cap, n->idx.p, n->y.p, dt, dm, dc, kRidge, n->dy.p,
                   n->lossb.p);
  backward_f32(n, s, B);
  HIPCHK(hipGetLastError());
  // the index copy (and copies of host-resident inputs) read caller or stack memory
  HIPCHK(hipStreamSynchronize(s));
  if (!want_loss) return 0.0;
  std::vector<float> lb = n->lossb.download(s, B);
  double sum = 0.0;
  for (float v : lb) sum += v;
  return sum / B;
}

void refresh_bf16(msdd_net* n, hipStream_t s) {
  if (!n->bf_stale) return;
  launch_to_bf16_t(s, n->n_in, n->H, n->kp1, W1(n), n->H, n->w1t.p);
  launch_to_bf16_t(s, n->H, n->H, n->kp2, W2(n), n->H, n->w2t.p);
  launch_to_bf16_t(s, n->H, n->out, n->kp2, W3(n), n->out, n->w3t.p);
  HIPCHK(hipGetLastError());
  n->bf_stale = false;
}

int fail(msdd_net* n, const MsddError& e) {
  if (n) n->err = e.msg;
  return e.code;
}

}  // namespace

namespace msdd_net_internal {
int n_in(const msdd_net* net) { return net->n_in; }
int n_hidden(const msdd_net* net) { return net->H; }
int n_vec(const msdd_net* net) { return net->V; }
int n_pos(const msdd_net* net) { return net->n_pos; }
int device(const msdd_net* net) { return net->device; }

void infer(msdd_net* n, int B, const float* x, float* y, hipStream_t s) {
  REQUIRE(B >= 1, "inference batch must be positive");
  // training launches on the network's own stream must be done before the weights are read
  if (n->stream != s) HIPCHK(hipStreamSynchronize(n->stream));
  refresh_bf16(n, s);
  if (B > n->cap_i) {
    n->xh.alloc((size_t)B * n->kp1);
    n->h1h.alloc((size_t)B * n->kp2);
    n->h2h.alloc((size_t)B * n->kp2);
    n->h1h.zero(s);  // padding columns H..kp2 stay zero
    n->h2h.zero(s);
    n->cap_i = B;
  }
  launch_to_bf16(s, B, n->n_in, n->kp1, x, n->n_in, n->xh.p);
  launch_hgemm(s, B, n->H, n->kp1, n->xh.p, n->w1t.p, b1(n), 1, 1, n->h1h.p, n->kp2);
  launch_hgemm(s, B, n->H, n->kp2, n->h1h.p, n->w2t.p, b2(n), 1, 1, n->h2h.p, n->kp2);
  launch_hgemm(s, B, n->out, n->kp2, n->h2h.p, n->w3t.p, b3(n), 0, 0, y, n->out);
  HIPCHK(hipGetLastError());
}
}  // namespace msdd_net_internal

extern "C" {

int msdd_net_create(msdd_net** out, int32_t n_in, int32_t n_hidden, int32_t n_vec, int32_t n_pos,
                    uint64_t seed, int32_t device, void* stream) {
  if (!out) return MSDD_EINVAL;
  *out = nullptr;
  auto* n = new msdd_net();
  try {
    REQUIRE(n_in >= 1 && n_hidden >= 1 && n_pos >= 1, "network sizes must be positive");
    REQUIRE(n_vec >= 1 && n_vec <= kMaxVec, "n_vec must lie in [1, 16]");
    REQUIRE((int64_t)n_vec * n_pos < (1ll << 30), "output layer too large");
    int ndev = 0;
    HIPCHK(hipGetDeviceCount(&ndev));
    REQUIRE(device >= 0 && device < ndev, "no such device");
    n->device = device;
    n->stream = (hipStream_t)stream;
    DeviceGuard dg(device);
    n->n_in = n_in;
    n->H = n_hidden;
    n->V = n_vec;
    n->n_pos = n_pos;
    n->out = n_vec * n_pos;
    const i64 sz[6] = {(i64)n_in * n_hidden, n_hidden, (i64)n_hidden * n_hidden, n_hidden,
                       (i64)n_hidden * n->out, n->out};
    n->off[0] = 0;
    for (int k = 0; k < 6; ++k) n->off[k + 1] = n->off[k] + sz[k];
    const i64 P = n->off[6];
    n->p.alloc(P);
    n->g.alloc(P);
    n->am.alloc(P);
    n->av.alloc(P);
    hipStream_t s = n->stream;
    n->p.zero(s);
    n->g.zero(s);
    n->am.zero(s);
    n->av.zero(s);
    const float a1 = (float)std::sqrt(6.0 / (n_in + n_hidden));
    const float a2 = (float)std::sqrt(6.0 / (2.0 * n_hidden));
    const float a3 = (float)std::sqrt(6.0 / ((double)n_hidden + n->out));
    launch_init_uniform(s, n->off[0], n->off[1], a1, seed ^ 0x1111111111111111ull, n->p.p);
    launch_init_uniform(s, n->off[2], n->off[3], a2, seed ^ 0x2222222222222222ull, n->p.p);
    launch_init_uniform(s, n->off[4], n->off[5], a3, seed ^ 0x3333333333333333ull, n->p.p);
    n->kp1 = round16(n_in);
    n->kp2 = round16(n_hidden);
    n->w1t.alloc((size_t)n_hidden * n->kp1);
    n->w2t.alloc((size_t)n_hidden * n->kp2);
    n->w3t.alloc((size_t)n->out * n->kp2);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
  } catch (const MsddError& e) {
    const int code = e.code;
    delete n;
    return code;
  }
  *out = n;
  return MSDD_OK;
}

int64_t msdd_net_param_count(const msdd_net* net) { return net ? net->off[6] : -1; }

int msdd_net_set_params(msdd_net* n, const float* p) {
  if (!n) return MSDD_EINVAL;
  try {
    DeviceGuard dg(n->device);
    REQUIRE(p != nullptr, "null parameter array");
    hipStream_t s = n->stream;
    HIPCHK(hipMemcpyAsync(n->p.p, p, n->off[6] * sizeof(float),
                          is_device_ptr(p) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
    n->am.zero(s);
    n->av.zero(s);
    n->step = 0;
    n->bf_stale = true;
    HIPCHK(hipStreamSynchronize(s));
  } catch (const MsddError& e) {
    return fail(n, e);
  }
  return MSDD_OK;
}

int msdd_net_get_params(const msdd_net* n, float* p) {
  if (!n || !p) return MSDD_EINVAL;
  try {
    DeviceGuard dg(n->device);
    HIPCHK(hipMemcpyAsync(p, n->p.p, n->off[6] * sizeof(float),
                          is_device_ptr(p) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                          n->stream));
    HIPCHK(hipStreamSynchronize(n->stream));
  } catch (const MsddError& e) {
    return fail(const_cast<msdd_net*>(n), e);
  }
  return MSDD_OK;
}

int msdd_net_forward(msdd_net* n, int32_t batch, const float* x, float* y, int32_t mode) {
  if (!n) return MSDD_EINVAL;
  try {
    DeviceGuard dg(n->device);
    REQUIRE(batch >= 1, "batch must be positive");
    REQUIRE(mode == 0 || mode == 1, "mode must be 0 (FP32) or 1 (BF16)");
    REQUIRE(y != nullptr, "null output array");
    hipStream_t s = n->stream;
    const bool ydev = is_device_ptr(y);
    const size_t ny = (size_t)batch * n->out;
    if (mode == 0) {
      ensure_train(n, batch);
      to_device(n->tmp_x, x, (size_t)batch * n->n_in, s);
      HIPCHK(hipMemcpyAsync(n->xb.p, n->tmp_x.p, (size_t)batch * n->n_in * sizeof(float),
                            hipMemcpyDeviceToDevice, s));
      forward_f32(n, s, batch);
      HIPCHK(hipMemcpyAsync(y, n->y.p, ny * sizeof(float),
                            ydev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
    } else {
      to_device(n->xi, x, (size_t)batch * n->n_in, s);
      float* yt = y;
      if (!ydev) {
        if (n->yi.n < ny) n->yi.alloc(ny);
        yt = n->yi.p;
      }
      msdd_net_internal::infer(n, batch, n->xi.p, yt, s);
      if (!ydev) HIPCHK(hipMemcpyAsync(y, yt, ny * sizeof(float), hipMemcpyDeviceToHost, s));
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
  } catch (const MsddError& e) {
    return fail(n, e);
  }
  return MSDD_OK;
}

int msdd_net_grad(msdd_net* n, int32_t batch, const int32_t* idx, int32_t n_samples,
                  const float* x_all, const float* tgt, const float* mask, const int32_t* cnt,
                  int32_t m_cap, float* loss, float* grad) {
  if (!n) return MSDD_EINVAL;
  try {
    DeviceGuard dg(n->device);
    const double l = loss_grad(n, batch, idx, n_samples, x_all, tgt, mask, cnt, m_cap, true);
    if (loss) *loss = (float)l;
    if (grad)
      HIPCHK(hipMemcpyAsync(grad, n->g.p, n->off[6] * sizeof(float),
                            is_device_ptr(grad) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                            n->stream));
    HIPCHK(hipStreamSynchronize(n->stream));
  } catch (const MsddError& e) {
    return fail(n, e);
  }
  return MSDD_OK;
}

int msdd_net_train_step(msdd_net* n, int32_t batch, const int32_t* idx, int32_t n_samples,
                        const float* x_all, const float* tgt, const float* mask,
                        const int32_t* cnt, int32_t m_cap, float lr, float* loss) {
  if (!n) return MSDD_EINVAL;
  try {
    DeviceGuard dg(n->device);
    REQUIRE(std::isfinite(lr) && lr > 0.f, "learning rate must be positive");
    const double l = loss_grad(n, batch, idx, n_samples, x_all, tgt, mask, cnt, m_cap, loss != nullptr);
    n->step += 1;
    launch_adam(n->stream, n->off[6], n->p.p, n->g.p, n->am.p, n->av.p, lr, n->step);
    HIPCHK(hipGetLastError());
    n->bf_stale = true;
    if (loss) *loss = (float)l;
  } catch (const MsddError& e) {
    return fail(n, e);
  }
  return MSDD_OK;
}

const char* msdd_net_last_error(const msdd_net* n) { return n ? n->err.c_str() : "null network"; }

void msdd_net_destroy(msdd_net* n) {
  if (!n) return;
  {
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(n->device);
    (void)hipStreamSynchronize(n->stream);
    delete n;
    if (prev >= 0) (void)hipSetDevice(prev);
  }
}

}  // extern "C"
