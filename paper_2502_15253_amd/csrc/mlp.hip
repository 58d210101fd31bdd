// MLP surrogate of the folded spectrum: dense layers with GELU, BF16 operands
// on the matrix cores (v_mfma_f32_16x16x32_bf16), FP32 accumulation, FP32
// master weights with Adam. Used only to propose fit start points; every
// reported NLL comes from the exact fold.
//
// GEMM: C (M x N) = A (M x K) * B^T, with both operands stored with the
// contraction index contiguous (A as [m][k], B as [n][k]), so tiles go from
// global memory to LDS with 16-byte loads and every lane reads its 8
// consecutive k values with one 16-byte LDS load. A workgroup of 256 threads
// computes a 128 x 128 tile (64 x 64 when that leaves too few workgroups to
// fill the chip); each wavefront a quarter of it as MFMA 16 x 16 blocks; K
// advances by 32 with the next step's global loads in flight. Out-of-range
// rows, columns and k are zero-filled, so any shape is accepted.
//
// Layouts that make every product k-contiguous: the forward pass uses W^T
// (kept as a second bf16 copy of the weights); the input gradient uses W as
// stored; the weight gradient dW = H^T dZ contracts over the batch, so the
// epilogues that produce activations H and back-propagated gradients dZ also
// write bf16 transposed copies ([feature][batch]), one 8-byte store per lane
// (the 4 consecutive rows an MFMA result lane holds). Weight gradients split
// the batch (K) over workgroups and add the slices in a fixed order.
// MFMA lane layout (16x16x32): lane l holds A[l % 16][8 (l / 16) + 0..7] and
// B[8 (l / 16) + 0..7][l % 16]; the result lane holds D[4 (l / 16) + i][l % 16].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/nufold.h"

namespace nufold {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

// float -> bf16 bits, round to nearest even (NaN kept quiet)
__host__ __device__ inline uint16_t f2bf(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ inline float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ inline float gelu_prime(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

enum { EPI_F32 = 0, EPI_BIAS_F32 = 1, EPI_BIAS_GELU = 2, EPI_DGELU = 3, EPI_PARTIAL = 4 };

struct GemmArgs {
  int M, N, K;
  int kslice;          // contraction range per blockIdx.z (multiple of 32)
  const uint16_t* A;   // [M][lda] bf16, k contiguous
  int lda;
  const uint16_t* B;   // [N][ldb] bf16, k contiguous
  int ldb;
  float* Cf;           // fp32 [M][ldc]: C (F32, BIAS_F32), pre-activation (BIAS_GELU), dz (DGELU);
                       // PARTIAL: slice z at Cf + z M ldc
  int ldc;
  uint16_t* Cb;        // bf16 [M][ldc] copy (BIAS_GELU: activation, DGELU: dz), nullable
  uint16_t* Ct;        // bf16 [N][ldt] transposed copy of the same, nullable
  int ldt;
  const float* bias;   // N (BIAS_*)
  const float* Zin;    // DGELU: pre-activation of the layer below, [M][ldc]
};

constexpr int TK = 32;  // contraction of one MFMA (and the granularity of K slices)

// One operand tile (ROWS x KT, k contiguous in memory) into registers; rows
// >= R and k >= K read as zero. LDS rows are padded by 8 bf16 against bank
// conflicts.
template <int ROWS, int KT>
struct TileRegs {
  static constexpr int LDK = KT + 8;
  static constexpr int NV = ROWS * KT / 8 / 256;  // 16-byte vectors per thread
  bf16x8 v[NV];

  __device__ void load(const uint16_t* __restrict__ src, int ld, int r0, int R, int k0, int K, int tid) {
    const bool vec_ok = (ld & 7) == 0 && ((uintptr_t)src & 15) == 0;
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      const int e = tid + 256 * j;
      const int r = e / (KT / 8), k = (e % (KT / 8)) * 8;
      const int gr = r0 + r, gk = k0 + k;
      if (vec_ok && gr < R && gk + 8 <= K) {
        v[j] = *reinterpret_cast<const bf16x8*>(src + (int64_t)gr * ld + gk);
      } else {
        union { bf16x8 b; uint16_t u[8]; } t;
#pragma unroll
        for (int i = 0; i < 8; ++i) t.u[i] = (gr < R && gk + i < K) ? src[(int64_t)gr * ld + gk + i] : 0;
        v[j] = t.b;
      }
    }
  }

  __device__ void store(uint16_t (*lds)[LDK], int tid) const {
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      const int e = tid + 256 * j;
      *reinterpret_cast<bf16x8*>(&lds[e / (KT / 8)][(e % (KT / 8)) * 8]) = v[j];
    }
  }
};

// C tile BM x BN per workgroup of four waves (2 x 2 wave tiles), K in steps
// of KT: the next step's operands are loaded into registers while this
// step's KT/32 MFMA chunks run from LDS (double-buffered).
template <int BM, int BN, int EPI, int KT>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g) {
  constexpr int FM = BM / 32, FN = BN / 32;
  constexpr int LDK = KT + 8;
  __shared__ __attribute__((aligned(16))) uint16_t As[2][BM][LDK];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[2][BN][LDK];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int wm = (wv >> 1) * (BM / 2), wn = (wv & 1) * (BN / 2);
  const int kb = blockIdx.z * g.kslice;
  const int ke = min(g.K, kb + g.kslice);
  f32x4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  TileRegs<BM, KT> ra;
  TileRegs<BN, KT> rb;
  const int nk = ke > kb ? (ke - kb + KT - 1) / KT : 0;
  if (nk > 0) {
    ra.load(g.A, g.lda, m0, g.M, kb, ke, tid);
    rb.load(g.B, g.ldb, n0, g.N, kb, ke, tid);
    ra.store(As[0], tid);
    rb.store(Bs[0], tid);
  }
  __syncthreads();
  const int r = lane & 15, kq = (lane >> 4) * 8;
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) {
      ra.load(g.A, g.lda, m0, g.M, kb + (kt + 1) * KT, ke, tid);
      rb.load(g.B, g.ldb, n0, g.N, kb + (kt + 1) * KT, ke, tid);
    }
#pragma unroll
    for (int kc = 0; kc < KT; kc += TK) {
      bf16x8 af[FM], bfr[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) af[i] = *reinterpret_cast<const bf16x8*>(&As[cur][wm + i * 16 + r][kc + kq]);
#pragma unroll
      for (int j = 0; j < FN; ++j) bfr[j] = *reinterpret_cast<const bf16x8*>(&Bs[cur][wn + j * 16 + r][kc + kq]);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
    }
    if (kt + 1 < nk) {
      ra.store(As[cur ^ 1], tid);
      rb.store(Bs[cur ^ 1], tid);
    }
    __syncthreads();
  }
  const int col = lane & 15, rq = (lane >> 4) * 4;
  float* Cf = g.Cf;
  if (EPI == EPI_PARTIAL) Cf += (int64_t)blockIdx.z * g.M * g.ldc;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int n = n0 + wn + j * 16 + col;
      const int mb = m0 + wm + i * 16 + rq;
      if (n >= g.N) continue;
      uint16_t tb[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = mb + q;
        tb[q] = 0;
        if (m >= g.M) continue;
        const float v = acc[i][j][q];
        const int64_t o = (int64_t)m * g.ldc + n;
        if (EPI == EPI_F32 || EPI == EPI_PARTIAL) {
          Cf[o] = v;
        } else if (EPI == EPI_BIAS_F32) {
          Cf[o] = v + g.bias[n];
        } else if (EPI == EPI_BIAS_GELU) {
          const float z = v + g.bias[n];
          Cf[o] = z;
          tb[q] = f2bf(gelu(z));
          if (g.Cb) g.Cb[o] = tb[q];
        } else {  // EPI_DGELU: v is dL/dh
          const float dz = v * gelu_prime(g.Zin[o]);
          Cf[o] = dz;
          tb[q] = f2bf(dz);
          if (g.Cb) g.Cb[o] = tb[q];
        }
      }
      if ((EPI == EPI_BIAS_GELU || EPI == EPI_DGELU) && g.Ct) {
        uint16_t* t = g.Ct + (int64_t)n * g.ldt + mb;
        if (mb + 3 < g.M && (g.ldt & 3) == 0) {
          *reinterpret_cast<uint2*>(t) =
              uint2{(uint32_t)tb[0] | ((uint32_t)tb[1] << 16), (uint32_t)tb[2] | ((uint32_t)tb[3] << 16)};
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (mb + q < g.M) t[q] = tb[q];
        }
      }
    }
}

// K split into `splits` slices (only with EPI_PARTIAL, slice z written to
// Cf + z M ldc); returns the number of slices launched in *slices.
template <int EPI>
hipError_t gemm(GemmArgs g, hipStream_t s, int splits = 1, int* slices = nullptr) {
  splits = std::max(1, splits);
  g.kslice = std::max(TK, ((g.K + splits - 1) / splits + TK - 1) / TK * TK);
  const int z = std::max(1, (g.K + g.kslice - 1) / g.kslice);
  if (slices) *slices = z;
  const int64_t t128 = (int64_t)((g.N + 127) / 128) * ((g.M + 127) / 128) * z;
  if (t128 >= 512) {
    const dim3 grid((g.N + 127) / 128, (g.M + 127) / 128, z);
    hipLaunchKernelGGL((gemm_kernel<128, 128, EPI, 32>), grid, dim3(256), 0, s, g);
  } else {
    // 64 x 64 tiles take K in steps of 64 (half the global round trips of
    // steps of 32; 36 KB of LDS)
    const dim3 grid((g.N + 63) / 64, (g.M + 63) / 64, z);
    hipLaunchKernelGGL((gemm_kernel<64, 64, EPI, 64>), grid, dim3(256), 0, s, g);
  }
  return hipGetLastError();
}

// weight-gradient slices added in slice order: out[i] = sum_z part[z][i]
__global__ void slice_sum_kernel(const float* __restrict__ part, int Z, int64_t n, float* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = 0.f;
  for (int z = 0; z < Z; ++z) s += part[(int64_t)z * n + i];
  out[i] = s;
}

__global__ void to_bf16_kernel(const float* x, uint16_t* y, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) y[i] = f2bf(x[i]);
}

// network input: fp32 [B][n_in] -> bf16 [B][kin] (zero-padded columns) and bf16 [n_in][B]
__global__ void prep_input_kernel(const float* x, int B, int n_in, int kin, uint16_t* xb, uint16_t* xt) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= (int64_t)B * kin) return;
  const int row = (int)(i / kin), c = (int)(i % kin);
  const uint16_t v = c < n_in ? f2bf(x[(int64_t)row * n_in + c]) : (uint16_t)0;
  xb[i] = v;
  if (c < n_in) xt[(int64_t)c * B + row] = v;
}

// gradient at the output: fp32 [B][N] -> bf16 [B][N] and bf16 [N][B]
__global__ void prep_grad_kernel(const float* d, int B, int N, uint16_t* db, uint16_t* dt) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= (int64_t)B * N) return;
  const uint16_t v = f2bf(d[i]);
  db[i] = v;
  dt[(int64_t)(i % N) * B + i / N] = v;
}

// bf16 W^T of one layer: wt[c][r] = bf16(w[r][c]) for r < din (columns din..dinp
// of wt stay zero)
__global__ void transpose_bf16_kernel(const float* w, int din, int dout, int dinp, uint16_t* wt) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= (int64_t)din * dout) return;
  const int r = (int)(i / dout), c = (int)(i % dout);
  wt[(int64_t)c * dinp + r] = f2bf(w[i]);
}

// Column sums of an M x N fp32 matrix (bias gradients) in a fixed order, two
// passes: blocks of CS_ROWS rows x 64 columns write partial sums, then one
// thread per column adds the partials in row-block order.
constexpr int CS_ROWS = 256;
__global__ __launch_bounds__(256) void colsum_partial_kernel(const float* __restrict__ x, int M, int N,
                                                            float* __restrict__ part) {
  __shared__ float red[4][64];
  const int c = threadIdx.x & 63, sl = threadIdx.x >> 6;
  const int n = blockIdx.x * 64 + c;
  const int m0 = blockIdx.y * CS_ROWS;
  const int m1 = min(M, m0 + CS_ROWS);
  float s = 0.f;
  if (n < N) {
#pragma unroll 8
    for (int m = m0 + sl; m < m1; m += 4) s += x[(int64_t)m * N + n];
  }
  red[sl][c] = s;
  __syncthreads();
  if (sl == 0 && n < N) part[(int64_t)blockIdx.y * N + n] = (red[0][c] + red[1][c]) + (red[2][c] + red[3][c]);
}

__global__ void colsum_final_kernel(const float* __restrict__ part, int nrb, int N, float* __restrict__ out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int r = 0; r < nrb; ++r) s += part[(int64_t)r * N + n];
  out[n] = s;
}

// Update of one layer inside the training step, right after its gradient
// products: the weight gradient's K slices summed in slice order and the
// bias gradient's column-sum partials in row-block order (the same sums as
// slice_sum_kernel and colsum_final_kernel), Adam on the fp32 master weights
// (step scalars sc as set by set_scalars_kernel), and the layer's bf16
// copies, as stored and transposed for the forward product (to_bf16_kernel,
// transpose_bf16_kernel).
// Pointers are the layer's: w, g, m, v, wb at its weights (biases follow).
__global__ void layer_update_kernel(float* w, float* g, float* m, float* v, uint16_t* wb, uint16_t* wt,
                                    const float* __restrict__ kpart, int Z, const float* __restrict__ csum,
                                    int nrb, int din, int dout, int dinp, const float* sc, float b1, float b2,
                                    float eps) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t nw = (int64_t)din * dout;
  if (i >= nw + dout) return;
  float gi = 0.f;
  if (i < nw) {
    for (int z = 0; z < Z; ++z) gi += kpart[(int64_t)z * nw + i];
  } else {
    const int c = (int)(i - nw);
    for (int r = 0; r < nrb; ++r) gi += csum[(int64_t)r * dout + c];
  }
  g[i] = gi;
  const float lr = sc[0], c1 = sc[1], c2 = sc[2];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  w[i] = wi;
  const uint16_t bw = f2bf(wi);
  wb[i] = bw;
  if (i < nw) wt[(int64_t)(i % dout) * dinp + i / dout] = bw;
}

// MSE over B x N: dy = 2 (y - t) / (B N) as fp32, bf16 and transposed bf16; per-block loss partials
__global__ void mse_kernel(const float* y, const float* t, int B, int N, float scale, float* dyf, uint16_t* dyb,
                           uint16_t* dyt, float* partial) {
  __shared__ float red[256];
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  float l = 0.f;
  if (i < (int64_t)B * N) {
    const float d = y[i] - t[i];
    l = d * d;
    const float g = 2.f * d * scale;
    const uint16_t gb = f2bf(g);
    dyf[i] = g;
    dyb[i] = gb;
    dyt[(int64_t)(i % N) * B + i / N] = gb;
  }
  red[threadIdx.x] = l;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Adam's moment decay rates and epsilon for the weight update.
constexpr float ADAM_B1 = 0.9f, ADAM_B2 = 0.999f, ADAM_EPS = 1e-8f;

// The Adam step's learning rate and bias corrections come from device memory
// (sc = {lr, 1 - b1^t, 1 - b2^t}), so that a captured training step replays
// with each step's values.
__global__ void set_scalars_kernel(float* sc, float lr, float c1, float c2) {
  if (threadIdx.x == 0) {
    sc[0] = lr;
    sc[1] = c1;
    sc[2] = c2;
  }
}
// Surrogate Poisson deviance per row with Gaussian input priors, and dL/dy:
// mu = exp(y std + mean), L = sum [mu - n + n ln(n/mu)] + 1/2 sum w_j (x_j - xbar_j)^2
__global__ void surrogate_nll_kernel(const float* y, const float* nobs, const float* mean, const float* stdv,
                                     int N, const float* x, const float* xbar, const float* xw, int Nin,
                                     float* dyf, uint16_t* dyb, float* dxp, float* nll) {
  __shared__ float red[256];
  const int row = blockIdx.x;
  float l = 0.f;
  for (int j = threadIdx.x; j < N; j += blockDim.x) {
    const int64_t o = (int64_t)row * N + j;
    const float lm = y[o] * stdv[j] + mean[j];
    const float mu = expf(lm);
    const float n = nobs[o];
    l += n > 0.f ? (mu - n + n * (logf(n) - lm)) : mu;
    const float g = (mu - n) * stdv[j];
    dyf[o] = g;
    dyb[o] = f2bf(g);
  }
  for (int j = threadIdx.x; j < Nin; j += blockDim.x) {
    const int64_t o = (int64_t)row * Nin + j;
    const float d = x[o] - xbar[j];
    l += 0.5f * xw[j] * d * d;
    dxp[o] = xw[j] * d;
  }
  red[threadIdx.x] = l;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) nll[row] = red[0];
}

// Adam on the inputs of every row (warm start), gradient = MLP input gradient + prior term
__global__ void input_adam_kernel(float* x, const float* dx, const float* dxp, float* m, float* v, int64_t n,
                                  float lr, float c1, float c2) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float g = dx[i] + dxp[i];
  const float mi = 0.9f * m[i] + 0.1f * g;
  const float vi = 0.999f * v[i] + 0.001f * g * g;
  m[i] = mi;
  v[i] = vi;
  x[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

}  // namespace nufold

using namespace nufold;

namespace {

template <typename T>
T* dalloc(size_t n) {
  T* p = nullptr;
  if (n && hipMalloc(&p, n * sizeof(T)) != hipSuccess) throw std::bad_alloc();
  return p;
}

constexpr int MAX_SPLITS = 32;  // batch slices of one weight-gradient product

}  // namespace

struct nf_mlp {
  std::string err;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int n_in = 0, kin = 0, width = 0, depth = 0, n_out = 0, max_batch = 0;
  int L = 0;                          // number of weight layers = depth + 1
  std::vector<int> din, dout, dinp;   // per layer; dinp: contraction length of the forward product
  std::vector<int64_t> woff, boff;    // offsets into the flat parameter vector
  std::vector<int64_t> toff;          // offsets of each layer's W^T in wbt
  int64_t nparam = 0, nwt = 0, maxdw = 0;
  float *w = nullptr, *g = nullptr, *am = nullptr, *av = nullptr;  // master params, grads, Adam moments
  uint16_t* wb = nullptr;             // bf16 copy of the parameter vector (W as stored: input gradient)
  uint16_t* wbt = nullptr;            // bf16 W^T per layer, [dout][dinp] (forward)
  float* xf = nullptr;                // B x n_in staging (fp32)
  uint16_t* xb = nullptr;             // B x kin bf16 (zero-padded)
  uint16_t* xt = nullptr;             // n_in x B bf16
  std::vector<float*> Z;              // pre-activations per hidden layer (B x width)
  std::vector<uint16_t*> H, HT;       // activations bf16, B x width and width x B
  float* Y = nullptr;                 // B x n_out
  float* T = nullptr;                 // targets B x n_out
  float *dYf = nullptr, *dZf = nullptr;        // B x max(width, n_out): back-propagated gradients (ping-pong)
  uint16_t *dYb = nullptr, *dZb = nullptr;     // the same in bf16
  uint16_t *dYt = nullptr, *dZt = nullptr;     // the same transposed, max(width, n_out) x B
  float* dX = nullptr;                // B x n_in
  float* partial = nullptr;           // loss partials
  float* csum = nullptr;              // column-sum partials
  float* kpart = nullptr;             // weight-gradient slices, MAX_SPLITS x maxdw
  float* scal = nullptr;              // learning rate and Adam bias corrections of the current step
  int adam_t = 0;
  // one training step of batch graph_B captured as a HIP graph (inputs and
  // step scalars are written before each replay)
  bool use_graph = true;
  int graph_B = 0;
  hipGraphExec_t step_graph = nullptr;
  ~nf_mlp() {
    for (void* p : {(void*)w, (void*)g, (void*)am, (void*)av, (void*)wb, (void*)wbt, (void*)xf, (void*)xb,
                    (void*)xt, (void*)Y, (void*)T, (void*)dYf, (void*)dZf, (void*)dYb, (void*)dZb, (void*)dYt,
                    (void*)dZt, (void*)dX, (void*)partial, (void*)csum, (void*)kpart, (void*)scal})
      if (p) (void)hipFree(p);
    for (auto* p : Z) (void)hipFree(p);
    for (auto* p : H) (void)hipFree(p);
    for (auto* p : HT) (void)hipFree(p);
    if (step_graph) (void)hipGraphExecDestroy(step_graph);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }
};

namespace {

thread_local std::string g_mlp_create_error;

struct MlpError : std::runtime_error {
  int code;
  MlpError(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void mck(hipError_t e, const char* what) {
  if (e != hipSuccess) throw MlpError(NF_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

template <typename F>
int mguard(nf_mlp* n, F&& f) {
  if (!n) return NF_EINVAL;
  try {
    n->err.clear();
    return f();
  } catch (const MlpError& e) {
    n->err = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    n->err = "device allocation failed";
    return NF_ENOMEM;
  }
}

inline dim3 blocks(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

// x (fp32, B x n_in, already in n->xf) -> bf16 operand copies
void prep_input(nf_mlp* n, int B) {
  hipLaunchKernelGGL(prep_input_kernel, blocks((int64_t)B * n->kin), dim3(256), 0, n->stream, n->xf, B, n->n_in,
                     n->kin, n->xb, n->xt);
}

void copy_x(nf_mlp* n, int B, const float* x, int on_device) {
  mck(hipMemcpyAsync(n->xf, x, sizeof(float) * B * n->n_in, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                     n->stream), "x copy");
}
void upload_x(nf_mlp* n, int B, const float* x, int on_device) {
  copy_x(n, B, x, on_device);
  prep_input(n, B);
}

void refresh_bf16(nf_mlp* n) {
  hipLaunchKernelGGL(to_bf16_kernel, blocks(n->nparam), dim3(256), 0, n->stream, n->w, n->wb, n->nparam);
  for (int l = 0; l < n->L; ++l)
    hipLaunchKernelGGL(transpose_bf16_kernel, blocks((int64_t)n->din[l] * n->dout[l]), dim3(256), 0, n->stream,
                       n->w + n->woff[l], n->din[l], n->dout[l], n->dinp[l], n->wbt + n->toff[l]);
}

// forward pass of B rows already in n->xb; output fp32 in n->Y. keep_t: also
// write the transposed activations that the weight gradient needs.
void forward(nf_mlp* n, int B, bool keep_t) {
  const uint16_t* in = n->xb;
  for (int l = 0; l < n->L; ++l) {
    GemmArgs a{};
    a.M = B; a.N = n->dout[l]; a.K = n->dinp[l];
    a.A = in; a.lda = n->dinp[l];
    a.B = n->wbt + n->toff[l]; a.ldb = n->dinp[l];
    a.ldc = n->dout[l];
    a.bias = n->w + n->boff[l];
    if (l < n->L - 1) {
      a.Cf = n->Z[l];
      a.Cb = n->H[l];
      a.Ct = keep_t ? n->HT[l] : nullptr;
      a.ldt = B;
      mck(gemm<EPI_BIAS_GELU>(a, n->stream), "gemm");
      in = n->H[l];
    } else {
      a.Cf = n->Y;
      mck(gemm<EPI_BIAS_F32>(a, n->stream), "gemm");
    }
  }
}

// backward from the output gradient (fp32 n->dYf, bf16 n->dYb and, when
// want_dw, transposed bf16 n->dYt, B x n_out): parameter gradients into n->g
// when want_dw; input gradient into n->dX when want_dx. update: the training
// step's form -- each layer's input gradient first (with the layer's weights
// before the step), then its parameter gradients and, in one kernel, its
// Adam step and bf16 copies (step scalars in n->scal).
void backward(nf_mlp* n, int B, bool want_dx, bool want_dw, bool update = false) {
  float* cf = n->dYf;
  uint16_t* cb = n->dYb;
  uint16_t* ct = n->dYt;
  for (int l = n->L - 1; l >= 0; --l) {
    float* nf = (cf == n->dZf) ? n->dYf : n->dZf;
    uint16_t* nb = (cb == n->dZb) ? n->dYb : n->dZb;
    uint16_t* nt = (ct == n->dZt) ? n->dYt : n->dZt;
    auto input_grad = [&] {
      // d(inp) = dcur W_l^T (B x din): W_l as stored is [din][dout], k = dout contiguous
      GemmArgs gd{};
      gd.M = B; gd.N = n->din[l]; gd.K = n->dout[l];
      gd.A = cb; gd.lda = n->dout[l];
      gd.B = n->wb + n->woff[l]; gd.ldb = n->dout[l];
      gd.ldc = n->din[l];
      if (l > 0) {
        gd.Cf = nf; gd.Cb = nb; gd.Ct = want_dw ? nt : nullptr; gd.ldt = B; gd.Zin = n->Z[l - 1];
        mck(gemm<EPI_DGELU>(gd, n->stream), "gemm dH");
      } else {
        gd.Cf = n->dX;
        mck(gemm<EPI_F32>(gd, n->stream), "gemm dX");
      }
    };
    const bool want_in = l > 0 || want_dx;
    if (update && want_in) input_grad();
    if (want_dw) {
      // dW_l = inp^T dcur (din x dout), contraction over the batch in slices
      GemmArgs gw{};
      gw.M = n->din[l]; gw.N = n->dout[l]; gw.K = B;
      gw.A = l == 0 ? n->xt : n->HT[l - 1]; gw.lda = B;
      gw.B = ct; gw.ldb = B;
      gw.Cf = n->kpart; gw.ldc = n->dout[l];
      const int tiles = ((gw.M + 127) / 128) * ((gw.N + 127) / 128);
      const int splits = std::min(MAX_SPLITS, std::max(1, std::min(512 / tiles, B / 256)));
      int zs = 1;
      mck(gemm<EPI_PARTIAL>(gw, n->stream, splits, &zs), "gemm dW");
      const int64_t mn = (int64_t)gw.M * gw.N;
      // db_l = column sums of dcur
      const int nrb = (B + CS_ROWS - 1) / CS_ROWS;
      hipLaunchKernelGGL(colsum_partial_kernel, dim3((n->dout[l] + 63) / 64, nrb), dim3(256), 0, n->stream, cf, B,
                         n->dout[l], n->csum);
      if (update) {
        const int64_t o = n->woff[l];
        hipLaunchKernelGGL(layer_update_kernel, blocks(mn + n->dout[l]), dim3(256), 0, n->stream, n->w + o, n->g + o,
                           n->am + o, n->av + o, n->wb + o, n->wbt + n->toff[l], (const float*)n->kpart, zs,
                           (const float*)n->csum, nrb, n->din[l], n->dout[l], n->dinp[l], (const float*)n->scal,
                           ADAM_B1, ADAM_B2, ADAM_EPS);
      } else {
        hipLaunchKernelGGL(slice_sum_kernel, blocks(mn), dim3(256), 0, n->stream, n->kpart, zs, mn,
                           n->g + n->woff[l]);
        hipLaunchKernelGGL(colsum_final_kernel, blocks(n->dout[l]), dim3(256), 0, n->stream, n->csum, nrb,
                           n->dout[l], n->g + n->boff[l]);
      }
    }
    if (!want_in) break;
    if (!update) input_grad();
    if (l > 0) {
      cf = nf;
      cb = nb;
      ct = nt;
    }
  }
}

}  // namespace

extern "C" {

int nf_mlp_create(nf_mlp** out, int n_in, int width, int depth, int n_out, int max_batch, void* hip_stream) {
  if (!out) return NF_EINVAL;
  *out = nullptr;
  g_mlp_create_error.clear();
  if (n_in < 1 || width < 1 || depth < 1 || n_out < 1 || max_batch < 1 || depth > 64) {
    g_mlp_create_error = "invalid MLP shape";
    return NF_EINVAL;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    g_mlp_create_error = "no HIP device available";
    return NF_EDEVICE;
  }
  nf_mlp* n = new nf_mlp();
  try {
    n->n_in = n_in; n->width = width; n->depth = depth; n->n_out = n_out; n->max_batch = max_batch;
    n->kin = (n_in + 7) / 8 * 8;
    n->L = depth + 1;
    int64_t off = 0, toff = 0;
    for (int l = 0; l < n->L; ++l) {
      const int a = l == 0 ? n_in : width, b = l == n->L - 1 ? n_out : width;
      const int ap = l == 0 ? n->kin : width;
      n->din.push_back(a);
      n->dout.push_back(b);
      n->dinp.push_back(ap);
      n->woff.push_back(off);
      off += (int64_t)a * b;
      n->boff.push_back(off);
      off += b;
      n->toff.push_back(toff);
      toff += (int64_t)b * ap;
      n->maxdw = std::max<int64_t>(n->maxdw, (int64_t)a * b);
    }
    n->nparam = off;
    n->nwt = toff;
    if (hip_stream) n->stream = (hipStream_t)hip_stream;
    else {
      mck(hipStreamCreateWithFlags(&n->stream, hipStreamNonBlocking), "hipStreamCreate");
      n->own_stream = true;
    }
    const size_t B = max_batch, wmax = std::max(width, n_out);
    n->w = dalloc<float>(off); n->g = dalloc<float>(off); n->am = dalloc<float>(off); n->av = dalloc<float>(off);
    n->wb = dalloc<uint16_t>(off);
    n->wbt = dalloc<uint16_t>(toff);
    n->xf = dalloc<float>(B * n_in); n->xb = dalloc<uint16_t>(B * n->kin); n->xt = dalloc<uint16_t>(B * n_in);
    for (int l = 0; l < depth; ++l) {
      n->Z.push_back(dalloc<float>(B * width));
      n->H.push_back(dalloc<uint16_t>(B * width));
      n->HT.push_back(dalloc<uint16_t>(B * width));
    }
    n->Y = dalloc<float>(B * n_out); n->T = dalloc<float>(B * n_out);
    n->dYf = dalloc<float>(B * wmax); n->dZf = dalloc<float>(B * wmax);
    n->dYb = dalloc<uint16_t>(B * wmax); n->dZb = dalloc<uint16_t>(B * wmax);
    n->dYt = dalloc<uint16_t>(B * wmax); n->dZt = dalloc<uint16_t>(B * wmax);
    n->dX = dalloc<float>(B * n_in);
    n->partial = dalloc<float>((B * n_out + 255) / 256 + 1);
    n->csum = dalloc<float>(((B + CS_ROWS - 1) / CS_ROWS) * wmax);
    n->kpart = dalloc<float>((size_t)MAX_SPLITS * n->maxdw);
    n->scal = dalloc<float>(4);
    mck(hipMemsetAsync(n->w, 0, sizeof(float) * off, n->stream), "memset");
    mck(hipMemsetAsync(n->am, 0, sizeof(float) * off, n->stream), "memset");
    mck(hipMemsetAsync(n->av, 0, sizeof(float) * off, n->stream), "memset");
    mck(hipMemsetAsync(n->wbt, 0, sizeof(uint16_t) * toff, n->stream), "memset");  // padding columns stay zero
    refresh_bf16(n);
    mck(hipStreamSynchronize(n->stream), "sync");
  } catch (const std::exception& e) {
    g_mlp_create_error = e.what();
    delete n;
    return NF_ENOMEM;
  }
  *out = n;
  return NF_OK;
}

void nf_mlp_destroy(nf_mlp* n) {
  if (!n) return;
  if (n->stream) (void)hipStreamSynchronize(n->stream);
  delete n;
}

const char* nf_mlp_last_error(const nf_mlp* n) { return n ? n->err.c_str() : g_mlp_create_error.c_str(); }

int64_t nf_mlp_num_params(const nf_mlp* n) { return n ? n->nparam : NF_EINVAL; }

int nf_mlp_set_params(nf_mlp* n, const float* params) {
  return mguard(n, [&] {
    if (!params) throw MlpError(NF_EINVAL, "params is null");
    mck(hipMemcpyAsync(n->w, params, sizeof(float) * n->nparam, hipMemcpyHostToDevice, n->stream), "H2D");
    mck(hipMemsetAsync(n->am, 0, sizeof(float) * n->nparam, n->stream), "memset");
    mck(hipMemsetAsync(n->av, 0, sizeof(float) * n->nparam, n->stream), "memset");
    n->adam_t = 0;
    refresh_bf16(n);
    mck(hipStreamSynchronize(n->stream), "sync");
    return NF_OK;
  });
}

int nf_mlp_get_params(nf_mlp* n, float* params) {
  return mguard(n, [&] {
    if (!params) throw MlpError(NF_EINVAL, "params is null");
    mck(hipMemcpyAsync(params, n->w, sizeof(float) * n->nparam, hipMemcpyDeviceToHost, n->stream), "D2H");
    mck(hipStreamSynchronize(n->stream), "sync");
    return NF_OK;
  });
}

int nf_mlp_forward(nf_mlp* n, int B, const float* x, float* y, int on_device) {
  return mguard(n, [&] {
    if (B < 1 || B > n->max_batch || !x || !y) throw MlpError(NF_EINVAL, "bad batch or null pointer");
    upload_x(n, B, x, on_device);
    forward(n, B, false);
    mck(hipMemcpyAsync(y, n->Y, sizeof(float) * B * n->n_out,
                       on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, n->stream), "y copy");
    mck(hipStreamSynchronize(n->stream), "sync");
    return NF_OK;
  });
}

int nf_mlp_grad(nf_mlp* n, int B, const float* x, const float* dy, float* grad, float* dx, int on_device) {
  return mguard(n, [&] {
    if (B < 1 || B > n->max_batch || !x || !dy) throw MlpError(NF_EINVAL, "bad batch or null pointer");
    const hipMemcpyKind k_in = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    const hipMemcpyKind k_out = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    upload_x(n, B, x, on_device);
    forward(n, B, true);
    const int64_t cnt = (int64_t)B * n->n_out;
    mck(hipMemcpyAsync(n->dYf, dy, sizeof(float) * cnt, k_in, n->stream), "dy copy");
    hipLaunchKernelGGL(prep_grad_kernel, blocks(cnt), dim3(256), 0, n->stream, n->dYf, B, n->n_out, n->dYb, n->dYt);
    backward(n, B, dx != nullptr, true);
    if (grad) mck(hipMemcpyAsync(grad, n->g, sizeof(float) * n->nparam, k_out, n->stream), "grad copy");
    if (dx) mck(hipMemcpyAsync(dx, n->dX, sizeof(float) * B * n->n_in, k_out, n->stream), "dx copy");
    mck(hipStreamSynchronize(n->stream), "sync");
    return NF_OK;
  });
}

int nf_mlp_train_step(nf_mlp* n, int B, const float* x, const float* t, float lr, float* loss, int on_device) {
  return mguard(n, [&] {
    if (B < 1 || B > n->max_batch || !x || !t || !(lr > 0.f)) throw MlpError(NF_EINVAL, "bad arguments");
    const int64_t cnt = (int64_t)B * n->n_out;
    const int nb = (int)((cnt + 255) / 256);
    // inputs and the step's scalars, then the step itself: input conversion,
    // forward, loss and its gradient, backward, Adam, bf16 refresh -- as
    // launches, or as one replay of the step captured for this batch size
    copy_x(n, B, x, on_device);
    mck(hipMemcpyAsync(n->T, t, sizeof(float) * cnt, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                       n->stream), "t copy");
    n->adam_t += 1;
    const float c1 = 1.f - std::pow(ADAM_B1, (float)n->adam_t), c2 = 1.f - std::pow(ADAM_B2, (float)n->adam_t);
    hipLaunchKernelGGL(set_scalars_kernel, dim3(1), dim3(64), 0, n->stream, n->scal, lr, c1, c2);
    auto body = [&] {
      prep_input(n, B);
      forward(n, B, true);
      hipLaunchKernelGGL(mse_kernel, dim3(nb), dim3(256), 0, n->stream, n->Y, n->T, B, n->n_out,
                         1.0f / (float)cnt, n->dYf, n->dYb, n->dYt, n->partial);
      backward(n, B, false, true, true);  // Adam and the bf16 copies per layer
    };
    if (!n->use_graph) {
      body();
    } else {
      if (n->step_graph && n->graph_B != B) {
        (void)hipGraphExecDestroy(n->step_graph);
        n->step_graph = nullptr;
      }
      if (!n->step_graph) {
        mck(hipStreamBeginCapture(n->stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
        try {
          body();
        } catch (...) {
          hipGraph_t g = nullptr;
          (void)hipStreamEndCapture(n->stream, &g);
          if (g) (void)hipGraphDestroy(g);
          throw;
        }
        hipGraph_t g = nullptr;
        mck(hipStreamEndCapture(n->stream, &g), "hipStreamEndCapture");
        const hipError_t e = hipGraphInstantiate(&n->step_graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        mck(e, "hipGraphInstantiate");
        n->graph_B = B;
      }
      mck(hipGraphLaunch(n->step_graph, n->stream), "hipGraphLaunch");
    }
    if (loss) {
      std::vector<float> part(nb);
      mck(hipMemcpyAsync(part.data(), n->partial, sizeof(float) * nb, hipMemcpyDeviceToHost, n->stream), "D2H");
      mck(hipStreamSynchronize(n->stream), "sync");
      double s = 0.0;
      for (float v : part) s += v;
      *loss = (float)(s / (double)cnt);
    } else if (!on_device) {
      mck(hipStreamSynchronize(n->stream), "sync");
    }
    return NF_OK;
  });
}

int nf_mlp_use_graphs(nf_mlp* n, int on) {
  return mguard(n, [&] {
    n->use_graph = on != 0;
    if (!n->use_graph && n->step_graph) {
      mck(hipStreamSynchronize(n->stream), "sync");
      (void)hipGraphExecDestroy(n->step_graph);
      n->step_graph = nullptr;
      n->graph_B = 0;
    }
    return NF_OK;
  });
}

int nf_mlp_fit_inputs(nf_mlp* n, int B, float* x, const float* nobs, const float* out_mean, const float* out_std,
                      const float* x_prior, const float* x_weight, int iters, float lr, float* nll) {
  return mguard(n, [&] {
    if (B < 1 || B > n->max_batch || !x || !nobs || !out_mean || !out_std || !x_prior || !x_weight || iters < 1)
      throw MlpError(NF_EINVAL, "bad arguments");
    const int Ni = n->n_in, No = n->n_out;
    float* mom = dalloc<float>((size_t)B * Ni * 3);  // m, v, prior gradient
    float* aux = dalloc<float>((size_t)No * 2 + (size_t)Ni * 2 + B);
    float* nd = dalloc<float>((size_t)B * No);
    struct Free {
      std::vector<void*> p;
      ~Free() { for (void* q : p) (void)hipFree(q); }
    } fr{{mom, aux, nd}};
    float *mean = aux, *sd = aux + No, *xbar = aux + 2 * No, *xw = xbar + Ni, *nllv = xw + Ni;
    float* xd = n->xf;  // the inputs being fitted live in the network's input staging buffer
    mck(hipMemcpyAsync(xd, x, sizeof(float) * B * Ni, hipMemcpyHostToDevice, n->stream), "H2D");
    mck(hipMemcpyAsync(nd, nobs, sizeof(float) * B * No, hipMemcpyHostToDevice, n->stream), "H2D");
    mck(hipMemcpyAsync(mean, out_mean, sizeof(float) * No, hipMemcpyHostToDevice, n->stream), "H2D");
    mck(hipMemcpyAsync(sd, out_std, sizeof(float) * No, hipMemcpyHostToDevice, n->stream), "H2D");
    mck(hipMemcpyAsync(xbar, x_prior, sizeof(float) * Ni, hipMemcpyHostToDevice, n->stream), "H2D");
    mck(hipMemcpyAsync(xw, x_weight, sizeof(float) * Ni, hipMemcpyHostToDevice, n->stream), "H2D");
    mck(hipMemsetAsync(mom, 0, sizeof(float) * B * Ni * 2, n->stream), "memset");
    const int64_t cx = (int64_t)B * Ni;
    for (int it = 1; it <= iters; ++it) {
      prep_input(n, B);
      forward(n, B, false);
      hipLaunchKernelGGL(surrogate_nll_kernel, dim3(B), dim3(256), 0, n->stream, n->Y, nd, mean, sd, No, xd, xbar, xw,
                         Ni, n->dYf, n->dYb, mom + 2 * cx, nllv);
      backward(n, B, true, false);
      const float c1 = 1.f - std::pow(0.9f, (float)it), c2 = 1.f - std::pow(0.999f, (float)it);
      hipLaunchKernelGGL(input_adam_kernel, blocks(cx), dim3(256), 0, n->stream, xd, n->dX, mom + 2 * cx, mom,
                         mom + cx, cx, lr, c1, c2);
    }
    // final NLL at the returned inputs
    prep_input(n, B);
    forward(n, B, false);
    hipLaunchKernelGGL(surrogate_nll_kernel, dim3(B), dim3(256), 0, n->stream, n->Y, nd, mean, sd, No, xd, xbar, xw, Ni,
                       n->dYf, n->dYb, mom + 2 * cx, nllv);
    mck(hipMemcpyAsync(x, xd, sizeof(float) * B * Ni, hipMemcpyDeviceToHost, n->stream), "D2H");
    if (nll) mck(hipMemcpyAsync(nll, nllv, sizeof(float) * B, hipMemcpyDeviceToHost, n->stream), "D2H");
    mck(hipStreamSynchronize(n->stream), "sync");
    return NF_OK;
  });
}

}  // extern "C"

namespace nufold {
// Shape of a network, for the engine's warm starts.
int mlp_shape(const nf_mlp* n, int* n_in, int* n_out, int* max_batch) {
  if (!n) return NF_EINVAL;
  *n_in = n->n_in;
  *n_out = n->n_out;
  *max_batch = n->max_batch;
  return NF_OK;
}
}  // namespace nufold
