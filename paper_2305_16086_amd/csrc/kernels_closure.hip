// Learned tail closure kernels.
//
// The series terms t_l(e) = sum_k w_k lambda_k^l (w_k >= 0) of every edge make
// the pair sums u_k = t_{2k} + t_{2k+1} a non-negative mixture of geometric
// sequences, so after the odd truncation tau0 = 2K+1 the tail lies in
// [u_K r_K/(1-r_K), u_K lambda*^2/(1-lambda*^2)] with r_K = u_K/u_{K-1}.  A
// small network predicts where in that interval the tail sits; the clamp makes
// the error of any prediction at most the interval width, and edges whose
// width exceeds eps fall back to the full traversal.
//
// Network 16 -> 64 -> 64 -> 1 with silu activations.  Parameters are one flat
// float vector: W1[64][16], b1[64], W2[64][64], b2[64], W3[64], b3.
// Training (FP32): per-workgroup forward/backward on 64-sample tiles, partial
// gradients reduced in a fixed order, Adam.  Inference: BF16 MFMA
// (gfx950's v_mfma_f32_16x16x32_bf16) with FP32 accumulation.
#include "sc_internal.hpp"

#include <hip/hip_bf16.h>

namespace sc {

namespace {

constexpr int kThreads = 64 * kWavesPerBlock;
constexpr int kIn = 16, kHid = 64;
constexpr int oW1 = 0, oB1 = oW1 + kHid * kIn, oW2 = oB1 + kHid, oB2 = oW2 + kHid * kHid,
              oW3 = oB2 + kHid, oB3 = oW3 + kHid, kNParam = oB3 + 1;
static_assert(kNParam == 5313, "parameter count");
constexpr int kL0 = 8, kRec = kL0 + 1, kK = 3;

inline unsigned grid_for(int64_t items, int per_block) {
  return static_cast<unsigned>((items + per_block - 1) / per_block);
}

__device__ inline float silu_f(float a) { return a / (1.0f + __expf(-a)); }
__device__ inline float silu_grad_f(float a) {
  const float s = 1.0f / (1.0f + __expf(-a));
  return s * (1.0f + a * (1.0f - s));
}

// ------------------------------------------------------------------ recordings
// rec[k][0..8] = p_l(s,s) and p_l(j,s) for slot k = (s -> j); l = 0, 1 in closed form.
template <typename T>
__global__ void k_record_init(int64_t nslots, const int32_t* __restrict__ col,
                              const T* __restrict__ inv_deg, T* __restrict__ rdiag,
                              T* __restrict__ roff) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= nslots) return;
  rdiag[k * kRec + 0] = T(1);
  roff[k * kRec + 0] = T(0);
  rdiag[k * kRec + 1] = T(0);
  roff[k * kRec + 1] = inv_deg[col[k]];
}

template <typename T, int B>
__global__ void k_record(int kbeg, int kend, int s0, int ell, const int32_t* __restrict__ slot_row,
                         const int32_t* __restrict__ col, const T* __restrict__ Y,
                         T* __restrict__ rdiag, T* __restrict__ roff) {
  const int k = kbeg + blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= kend) return;
  const int s = slot_row[k];
  const int c = s - s0;
  rdiag[static_cast<int64_t>(k) * kRec + ell] = Y[static_cast<size_t>(s) * B + c];
  roff[static_cast<int64_t>(k) * kRec + ell] = Y[static_cast<size_t>(col[k]) * B + c];
}

// The last recorded step without a full dense step: only p_L(s,s) and p_L(j,s)
// of the block's slots are read, so each is summed from the neighbour rows of
// Y = the state at L - 1 directly (Algorithm 2 lines 6-9 restricted to those
// rows).  Waves [0, nsrc) take a source s = s0 + w (p_L(s,s) for all its
// slots), the others one slot k = (s -> j) each (p_L(j,s), and the step L - 1
// recordings read from Y).  Lanes stride over the neighbours; fixed butterfly.
template <typename T>
__device__ inline T wave_sum_t(T v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <typename T, int B>
__global__ __launch_bounds__(kThreads) void k_record_last(
    int kbeg, int kend, int s0, int nsrc, int ell, const int32_t* __restrict__ rowptr,
    const int32_t* __restrict__ col, const int32_t* __restrict__ slot_row,
    const T* __restrict__ inv_deg, const T* __restrict__ Y, T* __restrict__ rdiag,
    T* __restrict__ roff) {
  const int lane = threadIdx.x & 63;
  const int w = static_cast<int>(blockIdx.x) * kWavesPerBlock + static_cast<int>(threadIdx.x >> 6);
  if (w < nsrc) {
    const int s = s0 + w;
    const int b = rowptr[s], e = rowptr[s + 1];
    T sum = T(0);
    for (int q = b + lane; q < e; q += 64) sum += Y[static_cast<size_t>(col[q]) * B + w];
    const T p = wave_sum_t(sum) * inv_deg[s];
    for (int q = b + lane; q < e; q += 64) rdiag[static_cast<int64_t>(q) * kRec + ell] = p;
    return;
  }
  const int k = kbeg + (w - nsrc);
  if (k >= kend) return;
  const int s = slot_row[k];
  const int c = s - s0;
  const int j = col[k];
  const int b = rowptr[j], e = rowptr[j + 1];
  T sum = T(0);
  for (int q = b + lane; q < e; q += 64) sum += Y[static_cast<size_t>(col[q]) * B + c];
  sum = wave_sum_t(sum);
  if (lane == 0) {
    const int64_t o = static_cast<int64_t>(k) * kRec;
    roff[o + ell] = sum * inv_deg[j];
    rdiag[o + ell - 1] = Y[static_cast<size_t>(s) * B + c];
    roff[o + ell - 1] = Y[static_cast<size_t>(j) * B + c];
  }
}

// ------------------------------------------------------------------ features and bounds
__device__ inline double sdiv(double a, double b) { return b != 0.0 ? a / b : 0.0; }

template <typename T>
__global__ void k_features(int64_t m, double m_edges, const int32_t* __restrict__ half_slot,
                           const int32_t* __restrict__ slot_row, const int32_t* __restrict__ col,
                           const int32_t* __restrict__ deg, const T* __restrict__ rdiag,
                           const T* __restrict__ roff, double lam, float* __restrict__ X,
                           double* __restrict__ s0_out, double* __restrict__ uK_out,
                           double* __restrict__ lo_out, double* __restrict__ hi_out) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= m) return;
  const int64_t k1 = half_slot[e];       // (u -> v)
  const int64_t k2 = half_slot[e + m];   // (v -> u)
  const double di = static_cast<double>(deg[slot_row[k1]]);
  const double dj = static_cast<double>(deg[col[k1]]);
  double t[kRec], a[kRec], b[kRec];
#pragma unroll
  for (int l = 0; l < kRec; ++l) {
    a[l] = static_cast<double>(rdiag[k1 * kRec + l]) / di + static_cast<double>(rdiag[k2 * kRec + l]) / dj;
    b[l] = 2.0 * static_cast<double>(roff[k1 * kRec + l]) / di;
    t[l] = a[l] - b[l];
  }
  double u[kK + 1];
#pragma unroll
  for (int q = 0; q <= kK; ++q) u[q] = t[2 * q] + t[2 * q + 1];
  float f[kIn];
  f[0] = static_cast<float>(1.0 / di + 1.0 / dj);
  f[1] = static_cast<float>(1.0 / (di * dj));
  f[2] = static_cast<float>(sdiv(u[1], u[0]));
  f[3] = static_cast<float>(sdiv(u[2], u[1]));
  f[4] = static_cast<float>(sdiv(u[3], u[2]));
  f[5] = static_cast<float>(sdiv(t[8], u[3]));
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    f[6 + q] = static_cast<float>(m_edges * a[6 + q]);
    f[9 + q] = static_cast<float>(m_edges * b[6 + q]);
    f[12 + q] = static_cast<float>(t[1 + q] / t[0]);
  }
  f[15] = static_cast<float>(u[3] / t[0]);
#pragma unroll
  for (int q = 0; q < kIn; ++q) X[e * kIn + q] = f[q];
  double s0 = 0.0;
#pragma unroll
  for (int l = 0; l <= 2 * kK + 1; ++l) s0 += t[l];
  const double lam2 = lam * lam;
  double r = sdiv(u[kK], u[kK - 1]);
  r = r < 0.0 ? 0.0 : (r > lam2 ? lam2 : r);
  s0_out[e] = s0;
  uK_out[e] = u[kK];
  lo_out[e] = r / (1.0 - r);
  hi_out[e] = lam2 / (1.0 - lam2);
}

// targets z = (s_ref - s0) / u_K, weight 0 where u_K = 0
__global__ void k_targets(int64_t m, const double* __restrict__ s_ref, const double* __restrict__ s0,
                          const double* __restrict__ uK, float* __restrict__ z,
                          float* __restrict__ w) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= m) return;
  const double u = uK[e];
  z[e] = u > 0.0 ? static_cast<float>((s_ref[e] - s0[e]) / u) : 0.0f;
  if (w) w[e] = u > 0.0 ? 1.0f : 0.0f;
}

// ------------------------------------------------------------------ normalisation statistics
// one workgroup per feature: mean and 1/std over N rows, fixed-order tree sums in double
__global__ __launch_bounds__(256) void k_norm_stats(const float* __restrict__ X, int64_t N,
                                                    float* __restrict__ norm) {
  __shared__ double s1[256], s2[256];
  const int f = blockIdx.x;
  double a = 0.0, b = 0.0;
  for (int64_t i = threadIdx.x; i < N; i += 256) {
    const double x = X[i * kIn + f];
    a += x;
    b += x * x;
  }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = b;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (threadIdx.x < w) {
      s1[threadIdx.x] += s1[threadIdx.x + w];
      s2[threadIdx.x] += s2[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double mean = s1[0] / static_cast<double>(N);
    const double var = s2[0] / static_cast<double>(N) - mean * mean;
    const double sd = var > 1e-24 ? sqrt(var) : 1.0;
    norm[f] = static_cast<float>(mean);
    norm[kIn + f] = static_cast<float>(1.0 / sd);
  }
}

// ------------------------------------------------------------------ training: forward + backward
// One workgroup of 64 threads per tile of 64 samples (thread = sample).
// grads: [tiles][kNParam] partial sums; lossp: [tiles] partial loss sums.
__global__ __launch_bounds__(64) void k_mlp_train_tile(const float* __restrict__ theta,
                                                       const float* __restrict__ norm,
                                                       const float* __restrict__ X,
                                                       const float* __restrict__ z,
                                                       const float* __restrict__ w,
                                                       const int64_t* __restrict__ idx,
                                                       int64_t nbatch, float inv_count,
                                                       float* __restrict__ grads,
                                                       float* __restrict__ lossp) {
  // weights are read with wave-uniform addresses straight from global memory
  const float* __restrict__ P = theta;
  __shared__ float sX[64][kIn + 1];
  __shared__ float sH1[64][kHid + 1];
  __shared__ float sD2[64][kHid + 1];
  __shared__ float sD1[64][kHid + 1];
  __shared__ float sdy[64];
  __shared__ float sl[64];
  const int t = threadIdx.x;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 64 + t;
  const bool live = i < nbatch;
  const int64_t row = live ? idx[i] : 0;
  float x[kIn];
#pragma unroll
  for (int f = 0; f < kIn; ++f) {
    x[f] = live ? (X[row * kIn + f] - norm[f]) * norm[kIn + f] : 0.0f;
    sX[t][f] = x[f];
  }
  __syncthreads();
  // forward
  float a1[kHid], a2[kHid];
  for (int o = 0; o < kHid; ++o) {
    float acc = P[oB1 + o];
#pragma unroll
    for (int f = 0; f < kIn; ++f) acc += P[oW1 + o * kIn + f] * x[f];
    a1[o] = acc;
    sH1[t][o] = silu_f(acc);
  }
  float y = P[oB3];
  for (int o = 0; o < kHid; ++o) {
    float acc = P[oB2 + o];
    for (int q = 0; q < kHid; ++q) acc += P[oW2 + o * kHid + q] * sH1[t][q];
    a2[o] = acc;
    y += P[oW3 + o] * silu_f(acc);
  }
  const float wt = live ? (w ? w[row] : 1.0f) : 0.0f;
  const float r = live ? y - z[row] : 0.0f;
  sl[t] = wt * r * r;
  const float dy = 2.0f * wt * r * inv_count;
  sdy[t] = dy;
  // backward through layer 3 and silu 2
  for (int o = 0; o < kHid; ++o) sD2[t][o] = dy * P[oW3 + o] * silu_grad_f(a2[o]);
  __syncthreads();
  // dA1 = (W2^T dA2) * silu'(a1)
  for (int q = 0; q < kHid; ++q) {
    float acc = 0.0f;
    for (int o = 0; o < kHid; ++o) acc += P[oW2 + o * kHid + q] * sD2[t][o];
    sD1[t][q] = acc * silu_grad_f(a1[q]);
  }
  __syncthreads();
  // weight gradients for this tile: thread t owns hidden unit t (fixed sample order)
  float* g = grads + static_cast<size_t>(blockIdx.x) * kNParam;
  {
    const int o = t;
    float gb1 = 0.0f, gb2 = 0.0f;
    float gw1[kIn];
#pragma unroll
    for (int f = 0; f < kIn; ++f) gw1[f] = 0.0f;
    for (int s = 0; s < 64; ++s) {
      const float d1 = sD1[s][o];
      gb1 += d1;
#pragma unroll
      for (int f = 0; f < kIn; ++f) gw1[f] += d1 * sX[s][f];
      gb2 += sD2[s][o];
    }
#pragma unroll
    for (int f = 0; f < kIn; ++f) g[oW1 + o * kIn + f] = gw1[f];
    g[oB1 + o] = gb1;
    g[oB2 + o] = gb2;
    for (int q = 0; q < kHid; ++q) {
      float acc = 0.0f;
      for (int s = 0; s < 64; ++s) acc += sD2[s][o] * sH1[s][q];
      g[oW2 + o * kHid + q] = acc;
    }
  }
  // layer-3 gradients need h2 = silu(a2) per sample: recompute into sD1 (no longer needed)
  __syncthreads();
  for (int o = 0; o < kHid; ++o) sD1[t][o] = silu_f(a2[o]);
  __syncthreads();
  {
    float acc = 0.0f;
    for (int s = 0; s < 64; ++s) acc += sdy[s] * sD1[s][t];
    g[oW3 + t] = acc;
  }
  if (t == 0) {
    float gb3 = 0.0f, ls = 0.0f;
    for (int s = 0; s < 64; ++s) {
      gb3 += sdy[s];
      ls += sl[s];
    }
    g[oB3] = gb3;
    lossp[blockIdx.x] = ls;
  }
}

// grad[p] = sum over tiles in order; loss = sum of tile losses * inv_count
__global__ void k_grad_reduce(const float* __restrict__ grads, int tiles,
                              const float* __restrict__ lossp, float inv_count,
                              float* __restrict__ grad, float* __restrict__ loss_out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < kNParam) {
    float acc = 0.0f;
    for (int b = 0; b < tiles; ++b) acc += grads[static_cast<size_t>(b) * kNParam + p];
    grad[p] = acc;
  }
  if (p == 0 && loss_out) {
    float l = 0.0f;
    for (int b = 0; b < tiles; ++b) l += lossp[b];
    *loss_out = l * inv_count;
  }
}

__global__ void k_adam(float* __restrict__ theta, const float* __restrict__ grad,
                       float* __restrict__ m1, float* __restrict__ m2, float lr, float b1,
                       float b2, float eps, float bc1, float bc2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kNParam) return;
  const float g = grad[p];
  const float a = b1 * m1[p] + (1.0f - b1) * g;
  const float b = b2 * m2[p] + (1.0f - b2) * g * g;
  m1[p] = a;
  m2[p] = b;
  theta[p] -= lr * (a / bc1) / (sqrtf(b / bc2) + eps);
}

// ------------------------------------------------------------------ inference
// FP32 reference path: one thread per sample.
__global__ __launch_bounds__(256) void k_mlp_infer_f32(const float* __restrict__ theta,
                                                       const float* __restrict__ norm,
                                                       const float* __restrict__ X, int64_t N,
                                                       float* __restrict__ y) {
  __shared__ float P[kNParam];
  for (int p = threadIdx.x; p < kNParam; p += blockDim.x) P[p] = theta[p];
  __syncthreads();
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= N) return;
  float x[kIn], h1[kHid];
#pragma unroll
  for (int f = 0; f < kIn; ++f) x[f] = (X[i * kIn + f] - norm[f]) * norm[kIn + f];
  for (int o = 0; o < kHid; ++o) {
    float acc = P[oB1 + o];
#pragma unroll
    for (int f = 0; f < kIn; ++f) acc += P[oW1 + o * kIn + f] * x[f];
    h1[o] = silu_f(acc);
  }
  float out = P[oB3];
  for (int o = 0; o < kHid; ++o) {
    float acc = P[oB2 + o];
    for (int q = 0; q < kHid; ++q) acc += P[oW2 + o * kHid + q] * h1[q];
    out += P[oW3 + o] * silu_f(acc);
  }
  y[i] = out;
}

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

// LDS hand-off between lanes of one wave (no workgroup barrier: waves iterate independently)
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline __bf16 as_bf16(short bits) { return __builtin_bit_cast(__bf16, bits); }

__device__ inline short to_bf16(float v) {
  // round to nearest even
  unsigned int u = __float_as_uint(v);
  const unsigned int lsb = (u >> 16) & 1u;
  u += 0x7FFFu + lsb;
  return static_cast<short>(u >> 16);
}

// BF16 MFMA path.  One wave handles 16 samples per iteration; layer products
// use v_mfma_f32_16x16x32_bf16 with the operand layout
//   A (16 x 32, row-major i,k): lane l supplies A[l%16][8*(l/16) .. +7]
//   B (32 x 16, k,j):           lane l supplies B[8*(l/16) .. +7][l%16]
//   D (16 x 16):                lane l holds D[4*(l/16) .. +3][l%16]
// Layer 1 (16 inputs) fills the upper half of k with zeros; layer 2 (64
// hidden inputs) takes two k-blocks of 32.  Activations move from the D layout
// to the A layout through LDS.
__global__ __launch_bounds__(256) void k_mlp_infer_bf16(const float* __restrict__ theta,
                                                        const float* __restrict__ norm,
                                                        const float* __restrict__ X, int64_t N,
                                                        float* __restrict__ y) {
  __shared__ short sW1[kHid * kIn];     // W1[o][f] in bf16
  __shared__ short sW2[kHid * kHid];    // W2[o][q]
  __shared__ float sB1[kHid], sB2[kHid], sW3[kHid];
  __shared__ float sAct[kWavesPerBlock][16][kHid + 1];
  for (int p = threadIdx.x; p < kHid * kIn; p += blockDim.x) sW1[p] = to_bf16(theta[oW1 + p]);
  for (int p = threadIdx.x; p < kHid * kHid; p += blockDim.x) sW2[p] = to_bf16(theta[oW2 + p]);
  for (int p = threadIdx.x; p < kHid; p += blockDim.x) {
    sB1[p] = theta[oB1 + p];
    sB2[p] = theta[oB2 + p];
    sW3[p] = theta[oW3 + p];
  }
  __syncthreads();
  const float b3 = theta[oB3];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int li = lane & 15;        // row (sample) for A, column for B / D
  const int lk = lane >> 4;        // k-quad for A / B, row-quad for D
  const int64_t ntiles = (N + 15) / 16;
  for (int64_t tile = static_cast<int64_t>(blockIdx.x) * kWavesPerBlock + wv; tile < ntiles;
       tile += static_cast<int64_t>(gridDim.x) * kWavesPerBlock) {
    const int64_t base = tile * 16;
    // layer 1: A = normalised X tile (16 x 16, k padded to 32 with zeros),
    // B = W1^T (16 x 64) in four 16-column blocks
    bf16x8_t ax;
    {
      const int64_t s = base + li;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int f = 8 * lk + q;
        const float v = s < N && f < kIn ? (X[s * kIn + f] - norm[f]) * norm[kIn + f] : 0.0f;
        ax[q] = as_bf16(to_bf16(v));
      }
    }
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
      bf16x8_t bw;
#pragma unroll
      for (int q = 0; q < 8; ++q)
        bw[q] = as_bf16(8 * lk + q < kIn ? sW1[(nb * 16 + li) * kIn + 8 * lk + q] : short(0));
      f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ax, bw, acc, 0, 0, 0);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int o = nb * 16 + li;
        sAct[wv][4 * lk + q][o] = silu_f(acc[q] + sB1[o]);
      }
    }
    wave_sync();
    // layer 2: A = H1 (16 x 64) as four k-blocks, B = W2^T
    f32x4_t acc2[4];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) acc2[nb] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
      bf16x8_t ah;
#pragma unroll
      for (int q = 0; q < 8; ++q) ah[q] = as_bf16(to_bf16(sAct[wv][li][kb * 32 + 8 * lk + q]));
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) {
        bf16x8_t bw;
#pragma unroll
        for (int q = 0; q < 8; ++q)
          bw[q] = as_bf16(sW2[(nb * 16 + li) * kHid + kb * 32 + 8 * lk + q]);
        acc2[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bw, acc2[nb], 0, 0, 0);
      }
    }
    wave_sync();
    // silu and layer 3 (dot with W3) in FP32: lane holds 4 samples x 4 columns per block
    float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
      const int o = nb * 16 + li;
#pragma unroll
      for (int q = 0; q < 4; ++q) part[q] += sW3[o] * silu_f(acc2[nb][q] + sB2[o]);
    }
    // sum over the 16 lanes sharing lk (columns), fixed butterfly
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      float v = part[q];
#pragma unroll
      for (int off = 8; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
      part[q] = v;
    }
    if (li == 0) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t s = base + 4 * lk + q;
        if (s < N) y[s] = part[q] + b3;
      }
    }
  }
}

// ------------------------------------------------------------------ closure and fallback
__global__ void k_closure_apply(int64_t m, const float* __restrict__ zpred,
                                const double* __restrict__ s0, const double* __restrict__ uK,
                                const double* __restrict__ lo, const double* __restrict__ hi,
                                const float* __restrict__ X, const float* __restrict__ fmin,
                                const float* __restrict__ fmax, double eps,
                                const int32_t* __restrict__ half_slot,
                                const int32_t* __restrict__ slot_row,
                                const int32_t* __restrict__ col, int B, int force,
                                double* __restrict__ out, unsigned char* __restrict__ fb,
                                int* __restrict__ block_flag, unsigned long long* count) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= m) return;
  const double width = uK[e] * (hi[e] - lo[e]);
  bool fall = force != 0 || !(width <= eps);
  if (!fall && fmin) {
    for (int f = 0; f < kIn; ++f) {
      const float x = X[e * kIn + f];
      if (!(x >= fmin[f] && x <= fmax[f])) fall = true;
    }
  }
  double z = static_cast<double>(zpred[e]);
  z = z < lo[e] ? lo[e] : (z > hi[e] ? hi[e] : z);
  out[e] = s0[e] + uK[e] * z;
  fb[e] = fall ? 1 : 0;
  if (fall) {
    const int k = half_slot[e];
    block_flag[slot_row[k] / B] = 1;
    block_flag[col[k] / B] = 1;
    atomicAdd(count, 1ull);
  }
}

__global__ void k_combine_masked(int64_t m, const int32_t* __restrict__ half_slot,
                                 const double* __restrict__ gacc,
                                 const unsigned char* __restrict__ fb, double* __restrict__ out) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= m || !fb[e]) return;
  out[e] = gacc[half_slot[e]] + gacc[half_slot[e + m]];
}

// feature range over N rows (for the out-of-range fallback): one workgroup per feature
__global__ __launch_bounds__(256) void k_feature_range(const float* __restrict__ X, int64_t N,
                                                       float* __restrict__ fmin,
                                                       float* __restrict__ fmax) {
  __shared__ float a[256], b[256];
  const int f = blockIdx.x;
  float lo = 3.0e38f, hi = -3.0e38f;
  for (int64_t i = threadIdx.x; i < N; i += 256) {
    const float x = X[i * kIn + f];
    lo = fminf(lo, x);
    hi = fmaxf(hi, x);
  }
  a[threadIdx.x] = lo;
  b[threadIdx.x] = hi;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (threadIdx.x < w) {
      a[threadIdx.x] = fminf(a[threadIdx.x], a[threadIdx.x + w]);
      b[threadIdx.x] = fmaxf(b[threadIdx.x], b[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    fmin[f] = a[0];
    fmax[f] = b[0];
  }
}

}  // namespace

#define SC_DISPATCH_B(B, CALL)                        \
  switch (B) {                                        \
    case 64: { constexpr int kB = 64; CALL; } break;  \
    case 32: { constexpr int kB = 32; CALL; } break;  \
    case 16: { constexpr int kB = 16; CALL; } break;  \
    default: return hipErrorInvalidValue;             \
  }

template <typename T>
const T* inv_deg_sel(const DeviceGraph& g);
template <>
const float* inv_deg_sel<float>(const DeviceGraph& g) { return g.inv_deg_f; }
template <>
const double* inv_deg_sel<double>(const DeviceGraph& g) { return g.inv_deg_d; }

template <typename T>
hipError_t launch_record_init(const DeviceGraph& g, T* rdiag, T* roff, hipStream_t st) {
  k_record_init<T><<<grid_for(g.nslots, 256), 256, 0, st>>>(g.nslots, g.col, inv_deg_sel<T>(g),
                                                             rdiag, roff);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_record(const DeviceGraph& g, int kbeg, int kend, int s0, int B, int ell,
                         const T* Y, T* rdiag, T* roff, hipStream_t st) {
  if (kend <= kbeg) return hipSuccess;
  SC_DISPATCH_B(B, (k_record<T, kB><<<grid_for(kend - kbeg, 256), 256, 0, st>>>(
                        kbeg, kend, s0, ell, g.slot_row, g.col, Y, rdiag, roff)));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_record_last(const DeviceGraph& g, int kbeg, int kend, int s0, int B, int ell,
                              const T* Y, T* rdiag, T* roff, hipStream_t st) {
  if (kend <= kbeg || ell < 3 || ell >= kRec) return hipErrorInvalidValue;
  const int nsrc = static_cast<int>(std::min<int64_t>(B, static_cast<int64_t>(g.n) - s0));
  if (nsrc <= 0) return hipErrorInvalidValue;
  const int waves = nsrc + (kend - kbeg);
  SC_DISPATCH_B(B, (k_record_last<T, kB><<<grid_for(waves, kWavesPerBlock), kThreads, 0, st>>>(
                        kbeg, kend, s0, nsrc, ell, g.rowptr, g.col, g.slot_row, inv_deg_sel<T>(g),
                        Y, rdiag, roff)));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_features(const DeviceGraph& g, const T* rdiag, const T* roff, double lam,
                           float* X, double* s0, double* uK, double* lo, double* hi,
                           hipStream_t st) {
  k_features<T><<<grid_for(g.m, 256), 256, 0, st>>>(g.m, static_cast<double>(g.nslots) / 2.0,
                                                     g.half_slot, g.slot_row, g.col, g.deg, rdiag,
                                                     roff, lam, X, s0, uK, lo, hi);
  return hipGetLastError();
}

hipError_t launch_targets(int64_t m, const double* s_ref, const double* s0, const double* uK,
                          float* z, float* w, hipStream_t st) {
  k_targets<<<grid_for(m, 256), 256, 0, st>>>(m, s_ref, s0, uK, z, w);
  return hipGetLastError();
}

hipError_t launch_norm_stats(const float* X, int64_t N, float* norm, hipStream_t st) {
  k_norm_stats<<<kIn, 256, 0, st>>>(X, N, norm);
  return hipGetLastError();
}

hipError_t launch_feature_range(const float* X, int64_t N, float* fmin, float* fmax,
                                hipStream_t st) {
  k_feature_range<<<kIn, 256, 0, st>>>(X, N, fmin, fmax);
  return hipGetLastError();
}

hipError_t launch_mlp_train_step(const float* theta, const float* norm, const float* X,
                                 const float* z, const float* w, const int64_t* idx,
                                 int64_t nbatch, float inv_count, float* grads, float* lossp,
                                 float* grad, float* loss_out, hipStream_t st) {
  const int tiles = static_cast<int>((nbatch + 63) / 64);
  k_mlp_train_tile<<<tiles, 64, 0, st>>>(theta, norm, X, z, w, idx, nbatch, inv_count, grads,
                                         lossp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_grad_reduce<<<grid_for(kNParam, 256), 256, 0, st>>>(grads, tiles, lossp, inv_count, grad,
                                                        loss_out);
  return hipGetLastError();
}

hipError_t launch_adam(float* theta, const float* grad, float* m1, float* m2, float lr,
                       float b1, float b2, float eps, int step, hipStream_t st) {
  const float bc1 = 1.0f - powf(b1, static_cast<float>(step));
  const float bc2 = 1.0f - powf(b2, static_cast<float>(step));
  k_adam<<<grid_for(kNParam, 256), 256, 0, st>>>(theta, grad, m1, m2, lr, b1, b2, eps, bc1, bc2);
  return hipGetLastError();
}

hipError_t launch_mlp_infer(const float* theta, const float* norm, const float* X, int64_t N,
                            int bf16, float* y, hipStream_t st) {
  if (N <= 0) return hipSuccess;
  if (bf16) {
    const int64_t tiles = (N + 15) / 16;
    int64_t blocks = (tiles + kWavesPerBlock - 1) / kWavesPerBlock;
    if (blocks > 4096) blocks = 4096;
    k_mlp_infer_bf16<<<static_cast<unsigned>(blocks), kThreads, 0, st>>>(theta, norm, X, N, y);
  } else {
    k_mlp_infer_f32<<<grid_for(N, 256), 256, 0, st>>>(theta, norm, X, N, y);
  }
  return hipGetLastError();
}

hipError_t launch_closure_apply(const DeviceGraph& g, const float* zpred, const double* s0,
                                const double* uK, const double* lo, const double* hi,
                                const float* X, const float* fmin, const float* fmax, double eps,
                                int B, int force, double* out, unsigned char* fb,
                                int* block_flag, unsigned long long* count, hipStream_t st) {
  k_closure_apply<<<grid_for(g.m, 256), 256, 0, st>>>(g.m, zpred, s0, uK, lo, hi, X, fmin, fmax,
                                                       eps, g.half_slot, g.slot_row, g.col, B,
                                                       force, out, fb, block_flag, count);
  return hipGetLastError();
}

hipError_t launch_combine_masked(const DeviceGraph& g, const double* gacc,
                                 const unsigned char* fb, double* out, hipStream_t st) {
  k_combine_masked<<<grid_for(g.m, 256), 256, 0, st>>>(g.m, g.half_slot, gacc, fb, out);
  return hipGetLastError();
}

template hipError_t launch_record_init<float>(const DeviceGraph&, float*, float*, hipStream_t);
template hipError_t launch_record_init<double>(const DeviceGraph&, double*, double*, hipStream_t);
template hipError_t launch_record<float>(const DeviceGraph&, int, int, int, int, int, const float*,
                                         float*, float*, hipStream_t);
template hipError_t launch_record<double>(const DeviceGraph&, int, int, int, int, int,
                                          const double*, double*, double*, hipStream_t);
template hipError_t launch_record_last<float>(const DeviceGraph&, int, int, int, int, int,
                                              const float*, float*, float*, hipStream_t);
template hipError_t launch_record_last<double>(const DeviceGraph&, int, int, int, int, int,
                                               const double*, double*, double*, hipStream_t);
template hipError_t launch_features<float>(const DeviceGraph&, const float*, const float*, double,
                                           float*, double*, double*, double*, double*,
                                           hipStream_t);
template hipError_t launch_features<double>(const DeviceGraph&, const double*, const double*,
                                            double, float*, double*, double*, double*, double*,
                                            hipStream_t);

}  // namespace sc
