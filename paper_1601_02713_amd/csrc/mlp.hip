// Learned SCF guess: features, network kernels (MFMA GEMM, loss, ReLU masks,
// bias sums, Adam), prediction and training (see mlp.h).
#include "mlp.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <random>
#include <stdexcept>

namespace bscf {
namespace mlp {

namespace {

void chk(hipError_t e, const char* what) {
  if (e != hipSuccess) throw std::runtime_error(std::string(what) + ": " + hipGetErrorString(e));
}

typedef float v4f __attribute__((ext_vector_type(4)));

// C (M x N, row-major, ldc) = op(A) op(B) + bias (per column), optional ReLU.
// op(A) is A (M x K, lda) or, with TA, the transpose of A stored K x M; op(B)
// is B (K x N, ldb) or, with TB, the transpose of B stored N x K.  A block of
// four wavefronts computes a 64 x 64 tile from 16-deep LDS stages; each
// wavefront owns 32 x 32 as 2 x 2 MFMA 16x16x4 (FP32) tiles.
// With gridDim.z > 1 the K range is split into chunks of kchunk (a multiple
// of 16) and every block adds its partial tile to C with atomics (C zeroed
// beforehand, no bias or ReLU).
template <bool TA, bool TB>
__global__ __launch_bounds__(256) void gemm_f32_kernel(int M, int N, int K, const float* __restrict__ A,
                                                       int lda, const float* __restrict__ B, int ldb,
                                                       float* __restrict__ C, int ldc,
                                                       const float* __restrict__ bias, int relu,
                                                       int kchunk) {
  __shared__ float As[16][64 + 4];
  __shared__ float Bs[16][64 + 4];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int kbeg = blockIdx.z * kchunk, kend = min(K, kbeg + kchunk);
  v4f acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
  for (int k0 = kbeg; k0 < kend; k0 += 16) {
    for (int e = tid; e < 1024; e += 256) {
      int mm, kk;
      if (TA) {
        mm = e & 63;
        kk = e >> 6;
      } else {
        kk = e & 15;
        mm = e >> 4;
      }
      const int gm = m0 + mm, gk = k0 + kk;
      float x = 0.f;
      if (gm < M && gk < kend) x = TA ? A[(long)gk * lda + gm] : A[(long)gm * lda + gk];
      As[kk][mm] = x;
    }
    for (int e = tid; e < 1024; e += 256) {
      int nn, kk;
      if (TB) {
        kk = e & 15;
        nn = e >> 4;
      } else {
        nn = e & 63;
        kk = e >> 6;
      }
      const int gn = n0 + nn, gk = k0 + kk;
      float x = 0.f;
      if (gn < N && gk < kend) x = TB ? B[(long)gn * ldb + gk] : B[(long)gk * ldb + gn];
      Bs[kk][nn] = x;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) {
      const int kr = kk + (lane >> 4), c = lane & 15;
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const float a = As[kr][wm + 16 * i + c];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const float b = Bs[kr][wn + 16 * j + c];
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[i][j], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  // lane l holds rows 4 (l / 16) + r, column l % 16 of each 16 x 16 tile
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
        const int gn = n0 + wn + 16 * j + (lane & 15);
        if (gm < M && gn < N) {
          float x = acc[i][j][r];
          if (gridDim.z > 1) {
            atomicAdd(&C[(long)gm * ldc + gn], x);
          } else {
            if (bias) x += bias[gn];
            if (relu) x = fmaxf(x, 0.f);
            C[(long)gm * ldc + gn] = x;
          }
        }
      }
}

void gemm(bool ta, bool tb, int M, int N, int K, const float* A, int lda, const float* B, int ldb,
          float* C, int ldc, const float* bias, bool relu, hipStream_t s) {
  const int tiles = ((N + 63) / 64) * ((M + 63) / 64);
  // few output tiles over a long reduction (weight gradients): split K so
  // that about 512 blocks share it
  int split = 1, kchunk = K;
  if (!bias && !relu && tiles < 256 && K >= 1024) {
    split = std::min((512 + tiles - 1) / tiles, K / 256);
    kchunk = ((K + split - 1) / split + 15) / 16 * 16;
    split = (K + kchunk - 1) / kchunk;
    if (ldc == N) {
      chk(hipMemsetAsync(C, 0, sizeof(float) * (size_t)M * N, s), "gemm zero");
    } else {
      for (int r = 0; r < M; ++r)
        chk(hipMemsetAsync(C + (long)r * ldc, 0, sizeof(float) * N, s), "gemm zero");
    }
  }
  const dim3 g((N + 63) / 64, (M + 63) / 64, split), b(256);
  const int rl = relu ? 1 : 0;
  if (!ta && !tb)
    hipLaunchKernelGGL((gemm_f32_kernel<false, false>), g, b, 0, s, M, N, K, A, lda, B, ldb, C, ldc, bias, rl, kchunk);
  else if (ta && !tb)
    hipLaunchKernelGGL((gemm_f32_kernel<true, false>), g, b, 0, s, M, N, K, A, lda, B, ldb, C, ldc, bias, rl, kchunk);
  else if (!ta && tb)
    hipLaunchKernelGGL((gemm_f32_kernel<false, true>), g, b, 0, s, M, N, K, A, lda, B, ldb, C, ldc, bias, rl, kchunk);
  else
    hipLaunchKernelGGL((gemm_f32_kernel<true, true>), g, b, 0, s, M, N, K, A, lda, B, ldb, C, ldc, bias, rl, kchunk);
}

// dY = 2 M (Y - T) / cnt; acc += sum M (Y - T)^2
__global__ void loss_grad_kernel(long n, const float* Y, const float* T, const float* Mk, float scale,
                                 float* dY, double* acc) {
  __shared__ double red[256];
  double part = 0.0;
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
    const float d = Mk[k] * (Y[k] - T[k]);
    dY[k] = 2.f * scale * d;
    part += (double)d * d;
  }
  red[threadIdx.x] = part;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(acc, red[0]);
}

// residual connection: Y[r][j] += X[r][din - dout + j]
__global__ void skip_kernel(long n, int din, int dout, const float* X, float* Y) {
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
    const long r = k / dout;
    Y[k] += X[r * din + (din - dout) + (k - r * dout)];
  }
}

__global__ void relu_back_kernel(long n, const float* H, float* dH) {
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x)
    if (!(H[k] > 0.f)) dH[k] = 0.f;
}

// out[j] += sum_i A[i][j] over the rows of this block's chunk (rows x cols,
// row-major; out zeroed beforehand)
constexpr int kColChunk = 256;
__global__ void colsum_kernel(int rows, int cols, const float* A, float* out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cols) return;
  const int i0 = blockIdx.y * kColChunk, i1 = min(rows, i0 + kColChunk);
  float s = 0.f;
  for (int i = i0; i < i1; ++i) s += A[(long)i * cols + j];
  atomicAdd(&out[j], s);
}

void colsum(int rows, int cols, const float* A, float* out, hipStream_t s) {
  chk(hipMemsetAsync(out, 0, sizeof(float) * cols, s), "colsum zero");
  hipLaunchKernelGGL(colsum_kernel, dim3((cols + 255) / 256, (rows + kColChunk - 1) / kColChunk),
                     dim3(256), 0, s, rows, cols, A, out);
}

__global__ void adam_kernel(long n, float* th, const float* g, float* m, float* v, float lr, float b1,
                            float b2, float eps, float bc1, float bc2) {
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
    const float mk = b1 * m[k] + (1.f - b1) * g[k];
    const float vk = b2 * v[k] + (1.f - b2) * g[k] * g[k];
    m[k] = mk;
    v[k] = vk;
    th[k] -= lr * (mk / bc1) / (sqrtf(vk / bc2) + eps);
  }
}

// row table: 8 ints per row (type, bf0 of A, nA, bf0 of B, nB, n, diagonal, pad) and
// the instance's matrix offset
struct RowDev {
  const int* info;
  const long long* moff;
  int bmax;
};

__global__ void features_kernel(int rows, RowDev rd, int ntp, const float* geo, const double* Pstd,
                                const double* Rprev, float scale, int din, float* X) {
  const int r = blockIdx.x;
  if (r >= rows) return;
  const int* f = rd.info + 8 * r;
  const int type = f[0], a0 = f[1], na = f[2], b0 = f[3], nb = f[4], n = f[5];
  const long long mo = rd.moff[r];
  const int B2 = rd.bmax * rd.bmax;
  float* x = X + (long)r * din;
  for (int k = threadIdx.x; k < din; k += blockDim.x) {
    float val = 0.f;
    if (k < ntp) {
      val = (k == type) ? 1.f : 0.f;
    } else if (k < ntp + kGeoFeatures) {
      val = geo[(long)r * kGeoFeatures + (k - ntp)];
    } else {
      const int e = (k - ntp - kGeoFeatures) % B2, which = (k - ntp - kGeoFeatures) / B2;
      const int i = e / rd.bmax, j = e % rd.bmax;
      if (i < na && j < nb) {
        const long long idx = mo + (long long)(a0 + i) * n + b0 + j;
        val = which == 0 ? (float)Pstd[idx] : (float)(scale * Rprev[idx]);
      }
    }
    x[k] = val;
  }
}

// targets: T = scale * R block, mask of the valid entries; acc += sum R^2
__global__ void targets_kernel(int rows, RowDev rd, const double* R, float scale, float* T, float* Mk,
                               double* acc) {
  const int r = blockIdx.x;
  if (r >= rows) return;
  const int* f = rd.info + 8 * r;
  const int a0 = f[1], na = f[2], b0 = f[3], nb = f[4], n = f[5];
  const long long mo = rd.moff[r];
  const int B2 = rd.bmax * rd.bmax;
  double part = 0.0;
  for (int e = threadIdx.x; e < B2; e += blockDim.x) {
    const int i = e / rd.bmax, j = e % rd.bmax;
    float t = 0.f, m = 0.f;
    if (i < na && j < nb) {
      const double v = R[mo + (long long)(a0 + i) * n + b0 + j];
      t = (float)(scale * v);
      m = 1.f;
      part += v * v;
    }
    T[(long)r * B2 + e] = t;
    Mk[(long)r * B2 + e] = m;
  }
  if (part != 0.0) atomicAdd(acc, part);
}

// flag = 1 if any valid output is non-finite or larger than limit
__global__ void check_kernel(long n, const float* Y, const float* Mk, float limit, int* flag) {
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x)
    if (Mk[k] != 0.f && !(fabsf(Y[k]) <= limit)) atomicOr(flag, 1);
}

// P += Y / scale on the blocks (A,B) and (B,A); diagonal blocks symmetrised
__global__ void scatter_kernel(int rows, RowDev rd, const float* Y, float inv_scale, double* P) {
  const int r = blockIdx.x;
  if (r >= rows) return;
  const int* f = rd.info + 8 * r;
  const int a0 = f[1], na = f[2], b0 = f[3], nb = f[4], n = f[5], diag = f[6];
  const long long mo = rd.moff[r];
  const int bm = rd.bmax;
  const float* y = Y + (long)r * bm * bm;
  for (int e = threadIdx.x; e < na * nb; e += blockDim.x) {
    const int i = e / nb, j = e % nb;
    if (diag) {
      P[mo + (long long)(a0 + i) * n + b0 + j] += 0.5 * inv_scale * ((double)y[i * bm + j] + y[j * bm + i]);
    } else {
      const double d = inv_scale * (double)y[i * bm + j];
      P[mo + (long long)(a0 + i) * n + b0 + j] += d;
      P[mo + (long long)(b0 + j) * n + a0 + i] += d;
    }
  }
}

__global__ void sub_kernel(long n, const double* A, const double* B, double* C) {
  for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x)
    C[k] = A[k] - B[k];
}

dim3 grid1d(long n) { return dim3((unsigned)std::min<long>((n + 255) / 256, 4096)); }

}  // namespace

template <typename T>
Buf<T>::~Buf() {
  if (p) (void)hipFree(p);
}

template <typename T>
void Buf<T>::resize(size_t m) {
  if (m <= n && p) return;
  if (p) (void)hipFree(p);
  p = nullptr;
  n = 0;
  if (m == 0) m = 1;
  chk(hipMalloc(&p, m * sizeof(T)), "hipMalloc (learned guess)");
  n = m;
}

template struct Buf<float>;
template struct Buf<double>;
template struct Buf<int>;
template struct Buf<long long>;

Guess::~Guess() = default;

long Guess::nparams() const {
  return (long)din_ * kHidden + kHidden + (long)kHidden * kHidden + kHidden + (long)kHidden * dout_ + dout_;
}

void Guess::configure(int din, int dout, unsigned seed) {
  if (din <= 0 || dout <= 0 || dout > din) throw std::runtime_error("learned guess: bad dimensions");
  din_ = din;
  dout_ = dout;
  const long np = nparams();
  theta_.resize(np);
  grad_.resize(np);
  m_.resize(np);
  v_.resize(np);
  // He-style weights, zero biases, a small last layer (first predictions ~ 0)
  std::vector<float> h(np, 0.f);
  std::mt19937 gen(seed);
  std::normal_distribution<float> nd(0.f, 1.f);
  long k = 0;
  auto fill = [&](long cnt, float sd) {
    for (long i = 0; i < cnt; ++i) h[k++] = sd * nd(gen);
  };
  fill((long)din * kHidden, std::sqrt(2.f / din));
  k += kHidden;
  fill((long)kHidden * kHidden, std::sqrt(2.f / kHidden));
  k += kHidden;
  fill((long)kHidden * dout, 0.01f * std::sqrt(2.f / kHidden));
  chk(hipMemcpy(theta_.p, h.data(), np * sizeof(float), hipMemcpyHostToDevice), "params");
  chk(hipMemset(m_.p, 0, np * sizeof(float)), "adam m");
  chk(hipMemset(v_.p, 0, np * sizeof(float)), "adam v");
  adam_steps_ = 0;
  work_rows_ = 0;
}

void Guess::configure_detached(int din, int dout, unsigned seed) {
  configure(din, dout, seed);
  types_.clear();
  bmax_ = 0;
  scale_ = 0.f;
  replay_next_ = replay_count_ = 0;
}

void Guess::set_params(const float* h, long n, hipStream_t s) {
  if (n != nparams()) throw std::runtime_error("learned guess: parameter count mismatch");
  chk(hipMemcpyAsync(theta_.p, h, n * sizeof(float), hipMemcpyHostToDevice, s), "set params");
  chk(hipMemsetAsync(m_.p, 0, n * sizeof(float), s), "adam m");
  chk(hipMemsetAsync(v_.p, 0, n * sizeof(float), s), "adam v");
  chk(hipStreamSynchronize(s), "sync");
  adam_steps_ = 0;
}

void Guess::get_params(float* h, long n, hipStream_t s) {
  if (n != nparams()) throw std::runtime_error("learned guess: parameter count mismatch");
  chk(hipMemcpyAsync(h, theta_.p, n * sizeof(float), hipMemcpyDeviceToHost, s), "get params");
  chk(hipStreamSynchronize(s), "sync");
}

void Guess::alloc_work(int rows) {
  if (rows <= work_rows_) return;
  h1_.resize((size_t)rows * kHidden);
  h2_.resize((size_t)rows * kHidden);
  dh1_.resize((size_t)rows * kHidden);
  dh2_.resize((size_t)rows * kHidden);
  y_.resize((size_t)rows * dout_);
  dy_.resize((size_t)rows * dout_);
  lossacc_.resize(1);
  work_rows_ = rows;
}

void Guess::forward(int rows, const float* X, hipStream_t s) {
  alloc_work(rows);
  forward_into(rows, X, h1_.p, h2_.p, y_.p, s);
}

// the three layers and the residual connection into caller buffers
// (h1, h2: rows x kHidden; y: rows x dout); kernel launches only
void Guess::forward_into(int rows, const float* X, float* h1, float* h2, float* y, hipStream_t s) {
  const float* W1 = theta_.p;
  const float* b1 = W1 + (long)din_ * kHidden;
  const float* W2 = b1 + kHidden;
  const float* b2 = W2 + (long)kHidden * kHidden;
  const float* W3 = b2 + kHidden;
  const float* b3 = W3 + (long)kHidden * dout_;
  gemm(false, false, rows, kHidden, din_, X, din_, W1, kHidden, h1, kHidden, b1, true, s);
  gemm(false, false, rows, kHidden, kHidden, h1, kHidden, W2, kHidden, h2, kHidden, b2, true, s);
  gemm(false, false, rows, dout_, kHidden, h2, kHidden, W3, dout_, y, dout_, b3, false, s);
  const long ny = (long)rows * dout_;
  hipLaunchKernelGGL(skip_kernel, grid1d(ny), dim3(256), 0, s, ny, din_, dout_, X, y);
}

// ------------------------------------------------- allocation-free evaluation

namespace {
// Hidden activations of the allocation-free forward pass: h1 then h2, each
// kNoAllocRows x kHidden floats.  One copy per GPU, held until the process
// ends.  Host code never passes this name to a kernel: it uses the device
// address found by hipGetSymbolAddress, kept per device below.
__device__ __align__(256) float scratch[2 * (size_t)kNoAllocRows * kHidden];

std::mutex g_scratch_mu;
std::map<int, float*> g_scratch_ptr;   // device ordinal -> address of its copy of scratch
}  // namespace

void init_noalloc_scratch(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr.count(device)) return;
  int cur = -1;
  chk(hipGetDevice(&cur), "current device");
  if (cur != device) throw std::runtime_error("init_noalloc_scratch: device not current");
  void* p = nullptr;
  chk(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "address of the allocation-free scratch");
  if (p == nullptr) throw std::runtime_error("allocation-free scratch has no device address");
  g_scratch_ptr[device] = static_cast<float*>(p);
}

void Guess::eval_noalloc(int device, int rows, const float* X, float* Y, hipStream_t s) {
  if (din_ == 0) throw std::runtime_error("learned guess: network not configured");
  if (rows <= 0 || rows > kNoAllocRows)
    throw std::runtime_error("learned guess: the allocation-free evaluation takes 1.." +
                             std::to_string(kNoAllocRows) + " rows, not " + std::to_string(rows));
  float* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    if (it == g_scratch_ptr.end())
      throw std::runtime_error("allocation-free scratch not set up on this device");
    base = it->second;
  }
  forward_into(rows, X, base, base + (size_t)kNoAllocRows * kHidden, Y, s);
  chk(hipGetLastError(), "allocation-free forward launch");
}

// gradient of the loss of the last forward pass into grad_; returns the loss
float Guess::backward(int rows, const float* X, const float* T, const float* M, double cnt,
                      hipStream_t s) {
  const float* W2 = theta_.p + (long)din_ * kHidden + kHidden;
  const float* W3 = W2 + (long)kHidden * kHidden + kHidden;
  float* gW1 = grad_.p;
  float* gb1 = gW1 + (long)din_ * kHidden;
  float* gW2 = gb1 + kHidden;
  float* gb2 = gW2 + (long)kHidden * kHidden;
  float* gW3 = gb2 + kHidden;
  float* gb3 = gW3 + (long)kHidden * dout_;
  chk(hipMemsetAsync(lossacc_.p, 0, sizeof(double), s), "loss");
  const long ny = (long)rows * dout_, nh = (long)rows * kHidden;
  hipLaunchKernelGGL(loss_grad_kernel, grid1d(ny), dim3(256), 0, s, ny, y_.p, T, M,
                     (float)(1.0 / cnt), dy_.p, lossacc_.p);
  gemm(true, false, kHidden, dout_, rows, h2_.p, kHidden, dy_.p, dout_, gW3, dout_, nullptr, false, s);
  colsum(rows, dout_, dy_.p, gb3, s);
  gemm(false, true, rows, kHidden, dout_, dy_.p, dout_, W3, dout_, dh2_.p, kHidden, nullptr, false, s);
  hipLaunchKernelGGL(relu_back_kernel, grid1d(nh), dim3(256), 0, s, nh, h2_.p, dh2_.p);
  gemm(true, false, kHidden, kHidden, rows, h1_.p, kHidden, dh2_.p, kHidden, gW2, kHidden, nullptr, false, s);
  colsum(rows, kHidden, dh2_.p, gb2, s);
  gemm(false, true, rows, kHidden, kHidden, dh2_.p, kHidden, W2, kHidden, dh1_.p, kHidden, nullptr, false, s);
  hipLaunchKernelGGL(relu_back_kernel, grid1d(nh), dim3(256), 0, s, nh, h1_.p, dh1_.p);
  gemm(true, false, din_, kHidden, rows, X, din_, dh1_.p, kHidden, gW1, kHidden, nullptr, false, s);
  colsum(rows, kHidden, dh1_.p, gb1, s);
  chk(hipGetLastError(), "backward launch");
  double l = 0.0;
  chk(hipMemcpyAsync(&l, lossacc_.p, sizeof(double), hipMemcpyDeviceToHost, s), "loss");
  chk(hipStreamSynchronize(s), "sync");
  return (float)(l / cnt);
}

void Guess::adam(float lr, hipStream_t s) {
  ++adam_steps_;
  const float b1 = 0.9f, b2 = 0.999f;
  const float bc1 = 1.f - std::pow(b1, (float)adam_steps_);
  const float bc2 = 1.f - std::pow(b2, (float)adam_steps_);
  const long n = nparams();
  hipLaunchKernelGGL(adam_kernel, grid1d(n), dim3(256), 0, s, n, theta_.p, grad_.p, m_.p, v_.p, lr,
                     b1, b2, 1e-8f, bc1, bc2);
  chk(hipGetLastError(), "adam launch");
}

void Guess::eval_rows(int rows, const float* X, const float* T, const float* M, float* Y,
                      float* grad, float* loss, hipStream_t s) {
  if (din_ == 0) throw std::runtime_error("learned guess: network not configured");
  if (rows <= 0) throw std::runtime_error("learned guess: no rows");
  Buf<float> x, t, m;
  x.resize((size_t)rows * din_);
  chk(hipMemcpyAsync(x.p, X, (size_t)rows * din_ * sizeof(float), hipMemcpyHostToDevice, s), "X");
  forward(rows, x.p, s);
  if (Y) chk(hipMemcpyAsync(Y, y_.p, (size_t)rows * dout_ * sizeof(float), hipMemcpyDeviceToHost, s), "Y");
  if (T && M) {
    t.resize((size_t)rows * dout_);
    m.resize((size_t)rows * dout_);
    chk(hipMemcpyAsync(t.p, T, (size_t)rows * dout_ * sizeof(float), hipMemcpyHostToDevice, s), "T");
    chk(hipMemcpyAsync(m.p, M, (size_t)rows * dout_ * sizeof(float), hipMemcpyHostToDevice, s), "M");
    double cnt = 0.0;
    for (long k = 0; k < (long)rows * dout_; ++k) cnt += M[k];
    if (cnt <= 0.0) throw std::runtime_error("learned guess: empty mask");
    const float l = backward(rows, x.p, t.p, m.p, cnt, s);
    if (loss) *loss = l;
    if (grad) chk(hipMemcpyAsync(grad, grad_.p, nparams() * sizeof(float), hipMemcpyDeviceToHost, s), "grad");
  }
  chk(hipStreamSynchronize(s), "sync");
}

float Guess::fit_rows(int rows, const float* X, const float* T, const float* M, int steps, float lr,
                      hipStream_t s) {
  if (din_ == 0) throw std::runtime_error("learned guess: network not configured");
  if (rows <= 0 || steps <= 0) throw std::runtime_error("learned guess: no rows or steps");
  Buf<float> x, t, m;
  x.resize((size_t)rows * din_);
  t.resize((size_t)rows * dout_);
  m.resize((size_t)rows * dout_);
  chk(hipMemcpyAsync(x.p, X, (size_t)rows * din_ * sizeof(float), hipMemcpyHostToDevice, s), "X");
  chk(hipMemcpyAsync(t.p, T, (size_t)rows * dout_ * sizeof(float), hipMemcpyHostToDevice, s), "T");
  chk(hipMemcpyAsync(m.p, M, (size_t)rows * dout_ * sizeof(float), hipMemcpyHostToDevice, s), "M");
  double cnt = 0.0;
  for (long k = 0; k < (long)rows * dout_; ++k) cnt += M[k];
  if (cnt <= 0.0) throw std::runtime_error("learned guess: empty mask");
  float l = 0.f;
  for (int k = 0; k < steps; ++k) {
    forward(rows, x.p, s);
    l = backward(rows, x.p, t.p, m.p, cnt, s);
    adam(lr, s);
  }
  chk(hipStreamSynchronize(s), "sync");
  return l;
}

// ------------------------------------------------------------------ in-run use

void Guess::reset_batch(int ninst) {
  ninst_ = ninst;
  have_std_ = have_prev_ = false;
  replay_next_ = replay_count_ = 0;
  xyz_prev_.clear();
}

void Guess::ensure_model(const Batch& b) {
  std::vector<int> zs;
  int bmax = 0;
  int tot = 0;
  for (int i = 0; i < b.ninst; ++i) tot += b.natoms[i];
  for (int a = 0; a < tot; ++a) {
    zs.push_back(b.Z[a]);
    bmax = std::max(bmax, b.atom_nbf[a]);
  }
  std::sort(zs.begin(), zs.end());
  zs.erase(std::unique(zs.begin(), zs.end()), zs.end());
  const int nt = (int)zs.size();
  const int ntp = nt * (nt + 1) / 2;
  const int din = ntp + kGeoFeatures + 2 * bmax * bmax, dout = bmax * bmax;
  if (din != din_ || dout != dout_ || zs != types_) {
    types_ = zs;
    bmax_ = bmax;
    configure(din, dout, 2000u);
    scale_ = 0.f;
    replay_next_ = replay_count_ = 0;
  }
}

// rows of every instance: atom pairs within the cutoff, lower (Z, index) first
void Guess::build_rows(const Batch& b) {
  rows_.clear();
  rowinfo_h_.clear();
  geo_h_.clear();
  std::vector<long long> rowoff;
  const int nt = (int)types_.size();
  auto tix = [&](int z) { return int(std::lower_bound(types_.begin(), types_.end(), z) - types_.begin()); };
  const bool disp = xyz_prev_.size() == b.xyz_len();
  for (int i = 0; i < b.ninst; ++i) {
    const int a0 = b.atom_off[i], na = b.natoms[i];
    for (int p = 0; p < na; ++p)
      for (int q = p; q < na; ++q) {
        int A = a0 + p, B = a0 + q;
        if (b.Z[B] < b.Z[A]) std::swap(A, B);
        double R[3], r2 = 0.0;
        for (int d = 0; d < 3; ++d) {
          R[d] = b.xyz[3 * B + d] - b.xyz[3 * A + d];
          r2 += R[d] * R[d];
        }
        if (r2 > kCutoff * kCutoff) continue;
        int ta = tix(b.Z[A]), tb = tix(b.Z[B]);   // ta <= tb
        const int type = ta * nt - ta * (ta - 1) / 2 + (tb - ta);
        rows_.push_back({i, A, B, type});
        const int info[8] = {type, b.atom_bf0[A], b.atom_nbf[A], b.atom_bf0[B], b.atom_nbf[B],
                             b.nbf[i], A == B ? 1 : 0, 0};
        rowinfo_h_.insert(rowinfo_h_.end(), info, info + 8);
        rowoff.push_back(b.moff[i]);
        const double r = std::sqrt(r2);
        float g[kGeoFeatures] = {(float)(0.1 * R[0]), (float)(0.1 * R[1]), (float)(0.1 * R[2]),
                                 (float)(0.1 * r), 0, 0, 0, 0, 0, 0};
        if (disp)
          for (int d = 0; d < 3; ++d) {
            g[4 + d] = (float)(10.0 * (b.xyz[3 * A + d] - xyz_prev_[3 * A + d]));
            g[7 + d] = (float)(10.0 * (b.xyz[3 * B + d] - xyz_prev_[3 * B + d]));
          }
        geo_h_.insert(geo_h_.end(), g, g + kGeoFeatures);
      }
  }
  const int nr = (int)rows_.size();
  rowinfo_.resize((size_t)8 * nr + 2 * (size_t)nr);   // ints, then the 64-bit offsets
  geo_.resize((size_t)kGeoFeatures * nr);
  chk(hipMemcpyAsync(rowinfo_.p, rowinfo_h_.data(), rowinfo_h_.size() * sizeof(int),
                     hipMemcpyHostToDevice, b.stream), "row table");
  chk(hipMemcpyAsync(rowinfo_.p + 8 * (size_t)nr, rowoff.data(), rowoff.size() * sizeof(long long),
                     hipMemcpyHostToDevice, b.stream), "row offsets");
  chk(hipMemcpyAsync(geo_.p, geo_h_.data(), geo_h_.size() * sizeof(float), hipMemcpyHostToDevice,
                     b.stream), "geometry features");
}

void Guess::features(const Batch& b, float* X) {
  const int nr = (int)rows_.size();
  const int nt = (int)types_.size();
  RowDev rd{rowinfo_.p, reinterpret_cast<const long long*>(rowinfo_.p + 8 * (size_t)nr), bmax_};
  hipLaunchKernelGGL(features_kernel, dim3(nr), dim3(256), 0, b.stream, nr, rd, nt * (nt + 1) / 2,
                     geo_.p, pstd_.p, rprev_.p, have_prev_ ? scale_ : 0.f, din_, X);
  chk(hipGetLastError(), "features launch");
}

void Guess::begin_step(const Batch& b, bool have_std) {
  have_std_ = have_std;
  if (!have_std) return;
  pstd_.resize(b.mtot);
  chk(hipMemcpyAsync(pstd_.p, b.P, b.mtot * sizeof(double), hipMemcpyDeviceToDevice, b.stream), "standard guess");
}

bool Guess::predict(const Batch& b) {
  if (!have_std_ || !have_prev_ || adam_steps_ == 0 || scale_ <= 0.f) return false;
  ensure_model(b);
  if (adam_steps_ == 0) return false;   // the model was reconfigured
  build_rows(b);
  const int nr = (int)rows_.size();
  if (nr == 0) return false;
  X_.resize((size_t)nr * din_);
  features(b, X_.p);
  forward(nr, X_.p, b.stream);
  // reject non-finite or implausibly large corrections (|dP| > 0.5)
  Buf<float> mk;
  mk.resize((size_t)nr * dout_);
  Buf<float> tt;
  tt.resize((size_t)nr * dout_);
  Buf<int> flag;
  flag.resize(1);
  lossacc_.resize(1);
  RowDev rd{rowinfo_.p, reinterpret_cast<const long long*>(rowinfo_.p + 8 * (size_t)nr), bmax_};
  // the mask of the valid entries comes with the target kernel (targets unused)
  hipLaunchKernelGGL(targets_kernel, dim3(nr), dim3(256), 0, b.stream, nr, rd, rprev_.p, 0.f, tt.p,
                     mk.p, lossacc_.p);
  chk(hipMemsetAsync(flag.p, 0, sizeof(int), b.stream), "flag");
  const long ny = (long)nr * dout_;
  hipLaunchKernelGGL(check_kernel, grid1d(ny), dim3(256), 0, b.stream, ny, y_.p, mk.p, 0.5f * scale_,
                     flag.p);
  int bad = 0;
  chk(hipMemcpyAsync(&bad, flag.p, sizeof(int), hipMemcpyDeviceToHost, b.stream), "flag");
  chk(hipStreamSynchronize(b.stream), "sync");
  if (bad) return false;
  hipLaunchKernelGGL(scatter_kernel, dim3(nr), dim3(64), 0, b.stream, nr, rd, y_.p, 1.f / scale_, b.P);
  chk(hipGetLastError(), "scatter launch");
  return true;
}

void Guess::record(const Batch& b) {
  if (!have_std_) {
    xyz_prev_.assign(b.xyz, b.xyz + b.xyz_len());
    have_prev_ = false;
    return;
  }
  ensure_model(b);
  rprev_.resize(b.mtot);
  r_.resize(b.mtot);
  if (!have_prev_) chk(hipMemsetAsync(rprev_.p, 0, b.mtot * sizeof(double), b.stream), "residual");
  build_rows(b);
  const int nr = (int)rows_.size();
  // residual of this step
  hipLaunchKernelGGL(sub_kernel, grid1d((long)b.mtot), dim3(256), 0, b.stream, (long)b.mtot, b.P,
                     pstd_.p, r_.p);
  RowDev rd{rowinfo_.p, reinterpret_cast<const long long*>(rowinfo_.p + 8 * (size_t)nr), bmax_};
  if (scale_ <= 0.f) {
    // the residual scale: 1 / rms over the blocks of the first recorded step
    Buf<float> t, m;
    t.resize((size_t)nr * dout_);
    m.resize((size_t)nr * dout_);
    lossacc_.resize(1);
    chk(hipMemsetAsync(lossacc_.p, 0, sizeof(double), b.stream), "acc");
    hipLaunchKernelGGL(targets_kernel, dim3(nr), dim3(256), 0, b.stream, nr, rd, r_.p, 1.f, t.p, m.p,
                       lossacc_.p);
    double ss = 0.0;
    chk(hipMemcpyAsync(&ss, lossacc_.p, sizeof(double), hipMemcpyDeviceToHost, b.stream), "acc");
    chk(hipStreamSynchronize(b.stream), "sync");
    double cnt = 0.0;
    for (int r = 0; r < nr; ++r) cnt += (double)rowinfo_h_[8 * r + 2] * rowinfo_h_[8 * r + 4];
    const double rms = std::sqrt(ss / std::max(cnt, 1.0));
    scale_ = rms > 0.0 ? (float)(1.0 / rms) : 1.f;
  }
  Step& st = replay_[replay_next_];
  st.X.resize((size_t)nr * din_);
  st.T.resize((size_t)nr * dout_);
  st.M.resize((size_t)nr * dout_);
  st.rows = nr;
  st.cnt = 0.0;
  for (int r = 0; r < nr; ++r) st.cnt += (double)rowinfo_h_[8 * r + 2] * rowinfo_h_[8 * r + 4];
  features(b, st.X.p);
  lossacc_.resize(1);
  hipLaunchKernelGGL(targets_kernel, dim3(nr), dim3(256), 0, b.stream, nr, rd, r_.p, scale_, st.T.p,
                     st.M.p, lossacc_.p);
  chk(hipGetLastError(), "record launch");
  replay_next_ = (replay_next_ + 1) % kReplaySteps;
  replay_count_ = std::min(replay_count_ + 1, kReplaySteps);
  // this step's residual is the next step's input
  std::swap(rprev_.p, r_.p);
  std::swap(rprev_.n, r_.n);
  have_prev_ = true;
  xyz_prev_.assign(b.xyz, b.xyz + b.xyz_len());
  chk(hipStreamSynchronize(b.stream), "sync");
}

float Guess::train(int steps, hipStream_t s) {
  if (replay_count_ == 0 || din_ == 0 || steps <= 0) return -1.f;
  int rows = 0;
  double cnt = 0.0;
  for (int k = 0; k < replay_count_; ++k) {
    rows += replay_[k].rows;
    cnt += replay_[k].cnt;
  }
  tx_.resize((size_t)rows * din_);
  tt_.resize((size_t)rows * dout_);
  tm_.resize((size_t)rows * dout_);
  size_t off = 0;
  for (int k = 0; k < replay_count_; ++k) {
    const Step& st = replay_[k];
    chk(hipMemcpyAsync(tx_.p + off * din_, st.X.p, (size_t)st.rows * din_ * sizeof(float),
                       hipMemcpyDeviceToDevice, s), "replay X");
    chk(hipMemcpyAsync(tt_.p + off * dout_, st.T.p, (size_t)st.rows * dout_ * sizeof(float),
                       hipMemcpyDeviceToDevice, s), "replay T");
    chk(hipMemcpyAsync(tm_.p + off * dout_, st.M.p, (size_t)st.rows * dout_ * sizeof(float),
                       hipMemcpyDeviceToDevice, s), "replay M");
    off += st.rows;
  }
  float l = 0.f;
  for (int k = 0; k < steps; ++k) {
    forward(rows, tx_.p, s);
    l = backward(rows, tx_.p, tt_.p, tm_.p, cnt, s);
    adam(lr_, s);
  }
  chk(hipStreamSynchronize(s), "sync");
  return l;
}

// file: magic, din, dout, bmax, ntypes, types, scale, adam steps, theta, m, v
void Guess::save(const std::string& path) {
  if (din_ == 0) throw std::runtime_error("learned guess: nothing to save");
  std::ofstream f(path, std::ios::binary);
  if (!f) throw std::runtime_error("learned guess: cannot write " + path);
  save(f);
}

void Guess::save(std::ostream& f) {
  if (din_ == 0) throw std::runtime_error("learned guess: nothing to save");
  const long n = nparams();
  std::vector<float> th(n), m(n), v(n);
  chk(hipMemcpy(th.data(), theta_.p, n * sizeof(float), hipMemcpyDeviceToHost), "save");
  chk(hipMemcpy(m.data(), m_.p, n * sizeof(float), hipMemcpyDeviceToHost), "save");
  chk(hipMemcpy(v.data(), v_.p, n * sizeof(float), hipMemcpyDeviceToHost), "save");
  const int head[5] = {0x42534347, din_, dout_, bmax_, (int)types_.size()};
  f.write(reinterpret_cast<const char*>(head), sizeof(head));
  f.write(reinterpret_cast<const char*>(types_.data()), types_.size() * sizeof(int));
  f.write(reinterpret_cast<const char*>(&scale_), sizeof(float));
  f.write(reinterpret_cast<const char*>(&adam_steps_), sizeof(long));
  f.write(reinterpret_cast<const char*>(th.data()), n * sizeof(float));
  f.write(reinterpret_cast<const char*>(m.data()), n * sizeof(float));
  f.write(reinterpret_cast<const char*>(v.data()), n * sizeof(float));
  if (!f) throw std::runtime_error("learned guess: write failed");
}

// run state: have_prev, mtot, rprev [mtot if have_prev], n_xyz, xyz_prev,
// next, count, then per replay step rows, cnt, X [rows din], T, M [rows dout]
void Guess::save_run(std::ostream& f, long long mtot) {
  auto put = [&](const void* p, size_t n) { f.write(reinterpret_cast<const char*>(p), n); };
  const int hp = have_prev_ && rprev_.n >= (size_t)mtot ? 1 : 0;
  put(&hp, sizeof(int));
  put(&mtot, sizeof(long long));
  if (hp) {
    std::vector<double> r(mtot);
    chk(hipMemcpy(r.data(), rprev_.p, mtot * sizeof(double), hipMemcpyDeviceToHost), "save");
    put(r.data(), r.size() * sizeof(double));
  }
  const long long nx = (long long)xyz_prev_.size();
  put(&nx, sizeof(long long));
  put(xyz_prev_.data(), nx * sizeof(double));
  put(&replay_next_, sizeof(int));
  put(&replay_count_, sizeof(int));
  for (int k = 0; k < replay_count_; ++k) {
    const Step& st = replay_[k];
    put(&st.rows, sizeof(int));
    put(&st.cnt, sizeof(double));
    std::vector<float> X((size_t)st.rows * din_), T((size_t)st.rows * dout_), M(T.size());
    chk(hipMemcpy(X.data(), st.X.p, X.size() * sizeof(float), hipMemcpyDeviceToHost), "save");
    chk(hipMemcpy(T.data(), st.T.p, T.size() * sizeof(float), hipMemcpyDeviceToHost), "save");
    chk(hipMemcpy(M.data(), st.M.p, M.size() * sizeof(float), hipMemcpyDeviceToHost), "save");
    put(X.data(), X.size() * sizeof(float));
    put(T.data(), T.size() * sizeof(float));
    put(M.data(), M.size() * sizeof(float));
  }
}

Guess::RunState Guess::read_run(std::istream& f, int din, int dout) {
  auto get = [&](void* p, size_t n) {
    f.read(reinterpret_cast<char*>(p), n);
    if (!f) throw std::runtime_error("learned guess: truncated run state");
  };
  RunState r;
  long long mtot = 0, nx = 0;
  get(&r.have_prev, sizeof(int));
  get(&mtot, sizeof(long long));
  if (mtot < 0 || mtot > (1LL << 34)) throw std::runtime_error("learned guess: bad run state");
  if (r.have_prev) {
    r.rprev.resize(mtot);
    get(r.rprev.data(), mtot * sizeof(double));
  }
  get(&nx, sizeof(long long));
  if (nx < 0 || nx > (1LL << 24)) throw std::runtime_error("learned guess: bad run state");
  r.xyz_prev.resize(nx);
  get(r.xyz_prev.data(), nx * sizeof(double));
  get(&r.next, sizeof(int));
  get(&r.count, sizeof(int));
  if (r.count < 0 || r.count > kReplaySteps || r.next < 0 || r.next >= kReplaySteps)
    throw std::runtime_error("learned guess: bad run state");
  for (int k = 0; k < r.count; ++k) {
    int rows = 0;
    double cnt = 0.0;
    get(&rows, sizeof(int));
    get(&cnt, sizeof(double));
    if (rows < 0 || rows > (1 << 24)) throw std::runtime_error("learned guess: bad run state");
    r.rows.push_back(rows);
    r.cnt.push_back(cnt);
    r.X.emplace_back((size_t)rows * din);
    r.T.emplace_back((size_t)rows * dout);
    r.M.emplace_back((size_t)rows * dout);
    get(r.X.back().data(), r.X.back().size() * sizeof(float));
    get(r.T.back().data(), r.T.back().size() * sizeof(float));
    get(r.M.back().data(), r.M.back().size() * sizeof(float));
  }
  return r;
}

void Guess::apply_run(const RunState& r, long long mtot) {
  if (r.have_prev && (long long)r.rprev.size() != mtot)
    throw std::runtime_error("learned guess: run state of another batch");
  have_prev_ = r.have_prev != 0;
  if (have_prev_) {
    rprev_.resize(mtot);
    r_.resize(mtot);
    chk(hipMemcpy(rprev_.p, r.rprev.data(), mtot * sizeof(double), hipMemcpyHostToDevice), "load");
  }
  xyz_prev_ = r.xyz_prev;
  for (int k = 0; k < r.count; ++k) {
    Step& st = replay_[k];
    st.rows = r.rows[k];
    st.cnt = r.cnt[k];
    st.X.resize(r.X[k].size());
    st.T.resize(r.T[k].size());
    st.M.resize(r.M[k].size());
    chk(hipMemcpy(st.X.p, r.X[k].data(), r.X[k].size() * sizeof(float), hipMemcpyHostToDevice), "load");
    chk(hipMemcpy(st.T.p, r.T[k].data(), r.T[k].size() * sizeof(float), hipMemcpyHostToDevice), "load");
    chk(hipMemcpy(st.M.p, r.M[k].data(), r.M[k].size() * sizeof(float), hipMemcpyHostToDevice), "load");
  }
  replay_next_ = r.next;
  replay_count_ = r.count;
}

void Guess::load(const std::string& path) {
  std::ifstream f(path, std::ios::binary);
  if (!f) throw std::runtime_error("learned guess: cannot read " + path);
  const Saved m = read(f);
  apply(m);
}

Guess::Saved Guess::read(std::istream& f) {
  // the whole model is read and checked into host vectors before anything
  // changes, so a bad or truncated file leaves the current model in place
  int head[5];
  f.read(reinterpret_cast<char*>(head), sizeof(head));
  // widths as ensure_model makes them (dout = bmax^2, din = element pairs +
  // geometric features + two blocks), or those of a network fixed by
  // configure() alone (no element types, bmax 0, 0 < dout <= din)
  const int nt = head[4];
  const bool sized = nt > 0 && nt <= 128 && head[3] > 0 && head[3] <= 64 &&
                     head[2] == head[3] * head[3] &&
                     head[1] == nt * (nt + 1) / 2 + kGeoFeatures + 2 * head[3] * head[3];
  const bool bare = nt == 0 && head[3] == 0 && head[2] > 0 && head[2] <= head[1] &&
                    head[1] <= (1 << 20);
  if (!f || head[0] != 0x42534347 || !(sized || bare))
    throw std::runtime_error("learned guess: not a model file");
  std::vector<int> types(head[4]);
  f.read(reinterpret_cast<char*>(types.data()), types.size() * sizeof(int));
  float scale;
  long steps;
  f.read(reinterpret_cast<char*>(&scale), sizeof(float));
  f.read(reinterpret_cast<char*>(&steps), sizeof(long));
  const long n = (long)head[1] * kHidden + kHidden + (long)kHidden * kHidden + kHidden +
                 (long)kHidden * head[2] + head[2];
  std::vector<float> th(n), m(n), v(n);
  f.read(reinterpret_cast<char*>(th.data()), n * sizeof(float));
  f.read(reinterpret_cast<char*>(m.data()), n * sizeof(float));
  f.read(reinterpret_cast<char*>(v.data()), n * sizeof(float));
  if (!f) throw std::runtime_error("learned guess: truncated model file");
  if (!std::isfinite(scale) || steps < 0) throw std::runtime_error("learned guess: not a model file");
  Saved r;
  r.din = head[1];
  r.dout = head[2];
  r.bmax = head[3];
  r.types = std::move(types);
  r.scale = scale;
  r.adam_steps = steps;
  r.theta = std::move(th);
  r.m = std::move(m);
  r.v = std::move(v);
  return r;
}

void Guess::apply(const Saved& r) {
  const long n = (long)r.theta.size();
  configure(r.din, r.dout, 2000u);
  chk(hipMemcpy(theta_.p, r.theta.data(), n * sizeof(float), hipMemcpyHostToDevice), "load");
  chk(hipMemcpy(m_.p, r.m.data(), n * sizeof(float), hipMemcpyHostToDevice), "load");
  chk(hipMemcpy(v_.p, r.v.data(), n * sizeof(float), hipMemcpyHostToDevice), "load");
  bmax_ = r.bmax;
  types_ = r.types;
  scale_ = r.scale;
  adam_steps_ = r.adam_steps;
}

}  // namespace mlp
}  // namespace bscf
