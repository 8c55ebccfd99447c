// Small multilayer perceptron for the schedule cost model: FP64 forward,
// backward and Adam kernels on the device.  Network: D inputs -> H tanh ->
// H tanh -> 1 linear, mean-squared-error loss.  The batch is small (tens to
// hundreds of measured schedules) and so is the net, so every kernel is a
// plain one-thread-per-output loop in FP64 with fixed summation order
// (deterministic gradients); MFMA would not pay at this size.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ooc.h"

namespace {

#define MCHK(x)                                  \
  do {                                           \
    if ((x) != hipSuccess) return OOC_E_DEVICE;  \
  } while (0)

// Y[n,o] = act(b[o] + sum_i X[n,i] W[o,i]) ; act: 0 linear, 1 tanh
__global__ void k_dense_fwd(const double *X, const double *W, const double *b, double *Y, int N, int I, int O,
                            int act) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N * O) return;
  const int n = t / O, o = t % O;
  double s = b[o];
  for (int i = 0; i < I; i++) s += X[n * I + i] * W[o * I + i];
  Y[t] = act ? tanh(s) : s;
}

// dY[n] = 2 (yhat[n] - y[n]) / N
__global__ void k_out_grad(const double *yhat, const double *y, double *dY, int N) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n < N) dY[n] = 2.0 * (yhat[n] - y[n]) / (double)N;
}

// dW[o,i] = sum_n dZ[n,o] X[n,i]; db[o] = sum_n dZ[n,o]  (n in order)
__global__ void k_dense_bwd_w(const double *dZ, const double *X, double *dW, double *db, int N, int I, int O) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < O * I) {
    const int o = t / I, i = t % I;
    double s = 0.0;
    for (int n = 0; n < N; n++) s += dZ[n * O + o] * X[n * I + i];
    dW[t] = s;
  } else if (t < O * I + O) {
    const int o = t - O * I;
    double s = 0.0;
    for (int n = 0; n < N; n++) s += dZ[n * O + o];
    db[o] = s;
  }
}

// dZprev[n,i] = (sum_o dZ[n,o] W[o,i]) * (1 - A[n,i]^2)   (A: tanh output of the previous layer)
__global__ void k_dense_bwd_x(const double *dZ, const double *W, const double *A, double *dZprev, int N, int I,
                              int O) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N * I) return;
  const int n = t / I, i = t % I;
  double s = 0.0;
  for (int o = 0; o < O; o++) s += dZ[n * O + o] * W[o * I + i];
  const double a = A[t];
  dZprev[t] = s * (1.0 - a * a);
}

__global__ void k_mse(const double *yhat, const double *y, int N, double *loss) {
  __shared__ double sm[256];
  double s = 0.0;
  for (int n = threadIdx.x; n < N; n += 256) {
    const double d = yhat[n] - y[n];
    s += d * d;
  }
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) sm[threadIdx.x] += sm[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = sm[0] / (double)N;
}

// Adam (Kingma & Ba): m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
// p -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)
__global__ void k_adam(double *p, const double *g, double *m, double *v, int P, double lr, double b1, double b2,
                       double eps, double c1, double c2) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= P) return;
  const double gt = g[t];
  const double mt = b1 * m[t] + (1.0 - b1) * gt;
  const double vt = b2 * v[t] + (1.0 - b2) * gt * gt;
  m[t] = mt;
  v[t] = vt;
  p[t] -= lr * (mt / c1) / (sqrt(vt / c2) + eps);
}

unsigned blocks(int n) { return (unsigned)((n + 255) / 256); }

}  // namespace

// Device scratch of the allocation-free prediction (ooc_mlp_predict_noalloc):
// one call's inputs, both hidden activations and its outputs.  Every device
// the library runs on holds its own copy until the process ends; host code
// reaches it only through the address hipGetSymbolAddress returns for that
// device (the array's name is a host-side stand-in, not a device address).
static __device__ __align__(256) double scratch[OOC_MLP_SCRATCH_DOUBLES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};  // device address of `scratch`, per device, once looked up

// Address of `scratch` on device `dev`, which must be the current device.
int scratch_on(int dev, double **out) {
  if (dev < 0 || dev >= kMaxDevices) return OOC_E_ARG;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return OOC_E_DEVICE;
    g_scratch_ptr[dev] = static_cast<double *>(p);
  }
  *out = g_scratch_ptr[dev];
  return OOC_OK;
}

// element counts rounded up to 32 doubles, so every scratch part starts 256-byte aligned
size_t pad32(size_t n) { return (n + 31) & ~size_t(31); }

}  // namespace

struct ooc_mlp {
  int D = 0, Hd = 0, P = 0, cap = 0;  // inputs, hidden width, parameter count, batch capacity
  // parameter layout: W0[H*D] b0[H] W1[H*H] b1[H] W2[H] b2[1]
  double *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  double *X = nullptr, *y = nullptr, *A1 = nullptr, *A2 = nullptr, *out = nullptr;
  double *dO = nullptr, *dZ2 = nullptr, *dZ1 = nullptr, *loss = nullptr;
  int step = 0;
  int dev = 0;  // device the network lives on
  hipStream_t s = nullptr;
  int off_W0() const { return 0; }
  int off_b0() const { return Hd * D; }
  int off_W1() const { return Hd * D + Hd; }
  int off_b1() const { return Hd * D + Hd + Hd * Hd; }
  int off_W2() const { return Hd * D + 2 * Hd + Hd * Hd; }
  int off_b2() const { return Hd * D + 3 * Hd + Hd * Hd; }
};

namespace {

int ensure_batch(ooc_mlp *m, int N) {
  if (N <= m->cap) return OOC_OK;
  for (double **q : {&m->X, &m->y, &m->A1, &m->A2, &m->out, &m->dO, &m->dZ2, &m->dZ1})
    if (*q) (void)hipFree(*q);
  m->cap = N;
  MCHK(hipMalloc((void **)&m->X, sizeof(double) * N * m->D));
  MCHK(hipMalloc((void **)&m->y, sizeof(double) * N));
  MCHK(hipMalloc((void **)&m->A1, sizeof(double) * N * m->Hd));
  MCHK(hipMalloc((void **)&m->A2, sizeof(double) * N * m->Hd));
  MCHK(hipMalloc((void **)&m->out, sizeof(double) * N));
  MCHK(hipMalloc((void **)&m->dO, sizeof(double) * N));
  MCHK(hipMalloc((void **)&m->dZ2, sizeof(double) * N * m->Hd));
  MCHK(hipMalloc((void **)&m->dZ1, sizeof(double) * N * m->Hd));
  return OOC_OK;
}

// forward pass of N rows: X (N x D) -> A1, A2 (N x H) -> out (N)
void forward_into(ooc_mlp *m, int N, const double *X, double *A1, double *A2, double *out) {
  const int H = m->Hd, D = m->D;
  hipLaunchKernelGGL(k_dense_fwd, dim3(blocks(N * H)), dim3(256), 0, m->s, X, m->p + m->off_W0(),
                     m->p + m->off_b0(), A1, N, D, H, 1);
  hipLaunchKernelGGL(k_dense_fwd, dim3(blocks(N * H)), dim3(256), 0, m->s, A1, m->p + m->off_W1(),
                     m->p + m->off_b1(), A2, N, H, H, 1);
  hipLaunchKernelGGL(k_dense_fwd, dim3(blocks(N)), dim3(256), 0, m->s, A2, m->p + m->off_W2(),
                     m->p + m->off_b2(), out, N, H, 1, 0);
}

void forward(ooc_mlp *m, int N) { forward_into(m, N, m->X, m->A1, m->A2, m->out); }

void backward(ooc_mlp *m, int N) {
  const int H = m->Hd, D = m->D;
  hipLaunchKernelGGL(k_out_grad, dim3(blocks(N)), dim3(256), 0, m->s, m->out, m->y, m->dO, N);
  hipLaunchKernelGGL(k_dense_bwd_w, dim3(blocks(H + 1)), dim3(256), 0, m->s, m->dO, m->A2, m->g + m->off_W2(),
                     m->g + m->off_b2(), N, H, 1);
  hipLaunchKernelGGL(k_dense_bwd_x, dim3(blocks(N * H)), dim3(256), 0, m->s, m->dO, m->p + m->off_W2(), m->A2,
                     m->dZ2, N, H, 1);
  hipLaunchKernelGGL(k_dense_bwd_w, dim3(blocks(H * H + H)), dim3(256), 0, m->s, m->dZ2, m->A1,
                     m->g + m->off_W1(), m->g + m->off_b1(), N, H, H);
  hipLaunchKernelGGL(k_dense_bwd_x, dim3(blocks(N * H)), dim3(256), 0, m->s, m->dZ2, m->p + m->off_W1(), m->A1,
                     m->dZ1, N, H, H);
  hipLaunchKernelGGL(k_dense_bwd_w, dim3(blocks(H * D + H)), dim3(256), 0, m->s, m->dZ1, m->X,
                     m->g + m->off_W0(), m->g + m->off_b0(), N, D, H);
}

int upload_batch(ooc_mlp *m, const double *X, const double *y, int N) {
  int rc = ensure_batch(m, N);
  if (rc) return rc;
  MCHK(hipMemcpyAsync(m->X, X, sizeof(double) * N * m->D, hipMemcpyHostToDevice, m->s));
  if (y) MCHK(hipMemcpyAsync(m->y, y, sizeof(double) * N, hipMemcpyHostToDevice, m->s));
  return OOC_OK;
}

}  // namespace

extern "C" {

int ooc_mlp_create(ooc_mlp **out, int n_inputs, int n_hidden, uint64_t seed) {
  if (!out || n_inputs < 1 || n_inputs > 256 || n_hidden < 1 || n_hidden > 1024) return OOC_E_ARG;
  ooc_mlp *m = new ooc_mlp();
  m->D = n_inputs;
  m->Hd = n_hidden;
  m->P = m->off_b2() + 1;
  if (hipGetDevice(&m->dev) != hipSuccess || hipStreamCreateWithFlags(&m->s, hipStreamNonBlocking) != hipSuccess ||
      hipMalloc((void **)&m->p, sizeof(double) * m->P) != hipSuccess ||
      hipMalloc((void **)&m->g, sizeof(double) * m->P) != hipSuccess ||
      hipMalloc((void **)&m->m, sizeof(double) * m->P) != hipSuccess ||
      hipMalloc((void **)&m->v, sizeof(double) * m->P) != hipSuccess ||
      hipMalloc((void **)&m->loss, sizeof(double)) != hipSuccess) {
    delete m;
    return OOC_E_DEVICE;
  }
  // Glorot-uniform weights from SplitMix64(seed); zero biases
  std::vector<double> h(m->P, 0.0);
  uint64_t st = seed;
  auto u01 = [&] {
    st += 0x9E3779B97F4A7C15ull;
    uint64_t z = st;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
  };
  auto fill = [&](int off, int fan_in, int fan_out, int count) {
    const double lim = std::sqrt(6.0 / (fan_in + fan_out));
    for (int k = 0; k < count; k++) h[off + k] = lim * (2.0 * u01() - 1.0);
  };
  fill(m->off_W0(), m->D, m->Hd, m->Hd * m->D);
  fill(m->off_W1(), m->Hd, m->Hd, m->Hd * m->Hd);
  fill(m->off_W2(), m->Hd, 1, m->Hd);
  if (hipMemcpy(m->p, h.data(), sizeof(double) * m->P, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(m->m, 0, sizeof(double) * m->P) != hipSuccess ||
      hipMemset(m->v, 0, sizeof(double) * m->P) != hipSuccess) {
    delete m;
    return OOC_E_DEVICE;
  }
  *out = m;
  return OOC_OK;
}

int ooc_mlp_num_params(ooc_mlp *m) { return m ? m->P : OOC_E_ARG; }

int ooc_mlp_get_params(ooc_mlp *m, double *out) {
  if (!m || !out) return OOC_E_ARG;
  MCHK(hipMemcpy(out, m->p, sizeof(double) * m->P, hipMemcpyDeviceToHost));
  return OOC_OK;
}

int ooc_mlp_set_params(ooc_mlp *m, const double *in) {
  if (!m || !in) return OOC_E_ARG;
  MCHK(hipMemcpy(m->p, in, sizeof(double) * m->P, hipMemcpyHostToDevice));
  m->step = 0;
  MCHK(hipMemset(m->m, 0, sizeof(double) * m->P));
  MCHK(hipMemset(m->v, 0, sizeof(double) * m->P));
  return OOC_OK;
}

int ooc_mlp_predict(ooc_mlp *m, const double *X, int N, double *out) {
  if (!m || !X || !out || N < 1) return OOC_E_ARG;
  int rc = upload_batch(m, X, nullptr, N);
  if (rc) return rc;
  forward(m, N);
  MCHK(hipGetLastError());
  MCHK(hipMemcpyAsync(out, m->out, sizeof(double) * N, hipMemcpyDeviceToHost, m->s));
  MCHK(hipStreamSynchronize(m->s));
  return OOC_OK;
}

int ooc_mlp_predict_noalloc(ooc_mlp *m, const double *X, int N, double *out) {
  if (!m || !X || !out || N < 1) return OOC_E_ARG;
  const size_t nX = pad32((size_t)N * m->D), nA = pad32((size_t)N * m->Hd), nO = pad32((size_t)N);
  if (nX + 2 * nA + nO > (size_t)OOC_MLP_SCRATCH_DOUBLES) return OOC_E_ARG;
  int prev = 0;
  MCHK(hipGetDevice(&prev));
  if (prev != m->dev) MCHK(hipSetDevice(m->dev));
  double *base = nullptr;
  int rc = scratch_on(m->dev, &base);
  if (rc == OOC_OK) {
    double *sX = base, *sA1 = sX + nX, *sA2 = sA1 + nA, *sO = sA2 + nA;
    if (hipMemcpyAsync(sX, X, sizeof(double) * N * m->D, hipMemcpyHostToDevice, m->s) != hipSuccess) {
      rc = OOC_E_DEVICE;
    } else {
      forward_into(m, N, sX, sA1, sA2, sO);
      if (hipGetLastError() != hipSuccess ||
          hipMemcpyAsync(out, sO, sizeof(double) * N, hipMemcpyDeviceToHost, m->s) != hipSuccess ||
          hipStreamSynchronize(m->s) != hipSuccess)
        rc = OOC_E_DEVICE;
    }
  }
  if (prev != m->dev) (void)hipSetDevice(prev);
  return rc;
}

int ooc_mlp_gradient(ooc_mlp *m, const double *X, const double *y, int N, double *grad, double *loss) {
  if (!m || !X || !y || N < 1) return OOC_E_ARG;
  int rc = upload_batch(m, X, y, N);
  if (rc) return rc;
  forward(m, N);
  backward(m, N);
  hipLaunchKernelGGL(k_mse, dim3(1), dim3(256), 0, m->s, m->out, m->y, N, m->loss);
  MCHK(hipGetLastError());
  if (grad) MCHK(hipMemcpyAsync(grad, m->g, sizeof(double) * m->P, hipMemcpyDeviceToHost, m->s));
  if (loss) MCHK(hipMemcpyAsync(loss, m->loss, sizeof(double), hipMemcpyDeviceToHost, m->s));
  MCHK(hipStreamSynchronize(m->s));
  return OOC_OK;
}

int ooc_mlp_train(ooc_mlp *m, const double *X, const double *y, int N, int epochs, double lr, double *loss) {
  if (!m || !X || !y || N < 1 || epochs < 0 || !(lr > 0)) return OOC_E_ARG;
  int rc = upload_batch(m, X, y, N);
  if (rc) return rc;
  const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
  for (int e = 0; e < epochs; e++) {
    forward(m, N);
    backward(m, N);
    m->step++;
    const double c1 = 1.0 - std::pow(b1, m->step), c2 = 1.0 - std::pow(b2, m->step);
    hipLaunchKernelGGL(k_adam, dim3(blocks(m->P)), dim3(256), 0, m->s, m->p, m->g, m->m, m->v, m->P, lr, b1, b2,
                       eps, c1, c2);
  }
  forward(m, N);
  hipLaunchKernelGGL(k_mse, dim3(1), dim3(256), 0, m->s, m->out, m->y, N, m->loss);
  MCHK(hipGetLastError());
  if (loss) MCHK(hipMemcpyAsync(loss, m->loss, sizeof(double), hipMemcpyDeviceToHost, m->s));
  MCHK(hipStreamSynchronize(m->s));
  return OOC_OK;
}

int ooc_mlp_destroy(ooc_mlp *m) {
  if (!m) return OOC_E_ARG;
  (void)hipStreamSynchronize(m->s);
  for (double *q : {m->p, m->g, m->m, m->v, m->X, m->y, m->A1, m->A2, m->out, m->dO, m->dZ2, m->dZ1, m->loss})
    if (q) (void)hipFree(q);
  (void)hipStreamDestroy(m->s);
  delete m;
  return OOC_OK;
}

}  // extern "C"
