// Learned coarse-grid correction: a three-layer width-3 convolution over the
// coarse time steps, run and trained on gfx950 with bfloat16 MFMA products
// and FP32 accumulation.  The network and its contract: include/pitmg.h.
//
// Every layer, forward and backward, is one GEMM on the matrix cores,
//     C[m][n] = sum_k A(m,k) B(k,n),
// whose operands are read through small loaders that do the im2col of the
// width-3 convolution on the fly (rows of node-major activations are
// contiguous in time, so row t's receptive field is rows t-1, t, t+1):
//   forward    A = im2col(input)            B = W as [out][(d,c)]
//   weights    A = (layer output grad)^T    B = im2col(input)        (K = rows)
//   inputs     A = im2col(grad, reversed)   B = W as [in][(d,out)]
// The K range is split over work-groups when M x N has few tiles (inference
// has M = T = 8 rows); the partial sums are added in a fixed order by the
// epilogue kernels, which also apply bias, tanh and its derivative, so the
// results do not depend on scheduling.
#include "pitmg_internal.h"
#include "pitmg_device.h"
#include "../../include/pitmg.h"

#include <algorithm>
#include <cmath>
#include <string>

using namespace pitmg;

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t bf16_t;   // raw bfloat16 bits

constexpr int kWidth = 3;
constexpr int kBM = 32, kBN = 32, kBK = 32;
constexpr int kGemmThreads = 256;
constexpr int kEpiThreads = 256;

// Round to nearest, ties to even (no NaN inputs reach this).
__device__ __forceinline__ bf16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (bf16_t)(u >> 16);
}

// ---------------------------------------------------------------------------
// operand loaders: get(row, col) -> bfloat16 bits, zero outside the matrix
// ---------------------------------------------------------------------------

// im2col of node-major activations [samples][T][Cin]: row r = (s, t),
// column (d, c) -> act[s][t + dir (d - 1)][c], zero outside 0 <= t' < T.
struct Im2col {
  const bf16_t* bf = nullptr;   // bfloat16 source, or
  const float* f32 = nullptr;   // FP32 source rounded on load
  const int* idx = nullptr;     // optional sample gather (entries < count)
  int count = 0;
  int T = 0, Cin = 0, rows = 0, dir = 1;
  __device__ bf16_t get(int r, int col) const {
    if (r >= rows || col >= kWidth * Cin) return 0;
    const int s = r / T, t = r - s * T;
    const int d = col / Cin, c = col - d * Cin;
    const int tt = t + dir * (d - 1);
    if (tt < 0 || tt >= T) return 0;
    long long smp = s;
    if (idx) {
      smp = idx[s];
      if (smp < 0 || smp >= count) return 0;   // invalid index: zero row
    }
    const long long off = (smp * T + tt) * Cin + c;
    return bf ? bf[off] : to_bf16(f32[off]);
  }
};

// Row-major [n][ld] matrix read as B(k, n) = P[n*ld + k].
struct RowsAsCols {
  const bf16_t* P;
  int ld, nk, nn;
  __device__ bf16_t get(int k, int n) const {
    return (k < nk && n < nn) ? P[(long long)n * ld + k] : (bf16_t)0;
  }
};

// Row-major [k][ld] matrix read transposed as A(m, k) = P[k*ld + m].
struct Transposed {
  const bf16_t* P;
  int ld, nm, nk;
  __device__ bf16_t get(int m, int k) const {
    return (m < nm && k < nk) ? P[(long long)k * ld + m] : (bf16_t)0;
  }
};

// One 32x32 output tile per work-group, four waves of 16x16; K in steps of
// 32 through LDS, one v_mfma_f32_16x16x32_bf16 per wave and step.  Lane l
// supplies A[l%16][8(l/16) .. +7] and B[8(l/16) .. +7][l%16] and receives
// D[4(l/16) + i][l%16], i < 4.  blockIdx.z selects the K range
// [z*kchunk, (z+1)*kchunk); results go to part[z][M][N].
template <class SA, class SB>
__global__ __launch_bounds__(kGemmThreads) void k_gemm(SA a, SB b, int M, int N, int K,
                                                        int kchunk, float* __restrict__ part) {
  __shared__ __attribute__((aligned(16))) __bf16 As[kBM][kBK + 8];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[kBN][kBK + 8];
  const int tid = threadIdx.x, w = tid / kWave, lane = tid % kWave;
  const int m0 = blockIdx.y * kBM, n0 = blockIdx.x * kBN;
  const int kb = blockIdx.z * kchunk;
  const int ke = min(K, kb + kchunk);
  const int wm = (w >> 1) * 16, wn = (w & 1) * 16;
  const int fr = tid >> 3, fc = (tid & 7) * 4;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = kb; k0 < ke; k0 += kBK) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int k = k0 + fc + e;
      const bool in = k < ke;
      As[fr][fc + e] = __builtin_bit_cast(__bf16, in ? a.get(m0 + fr, k) : (bf16_t)0);
      Bs[fr][fc + e] = __builtin_bit_cast(__bf16, in ? b.get(k, n0 + fr) : (bf16_t)0);
    }
    __syncthreads();
    const int r = lane & 15, kq = (lane >> 4) * 8;
    const bf16x8 fa = *reinterpret_cast<const bf16x8*>(&As[wm + r][kq]);
    const bf16x8 fb = *reinterpret_cast<const bf16x8*>(&Bs[wn + r][kq]);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, fb, acc, 0, 0, 0);
    __syncthreads();
  }
  float* P = part + (size_t)blockIdx.z * M * N;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = m0 + wm + 4 * (lane >> 4) + i, n = n0 + wn + (lane & 15);
    if (m < M && n < N) P[(size_t)m * N + n] = acc[i];
  }
}

__device__ __forceinline__ float sum_parts(const float* part, int splits, long long MN,
                                           long long i) {
  float s = 0.f;
  for (int z = 0; z < splits; ++z) s += part[z * MN + i];
  return s;
}

// h = tanh(sum + bias): FP32 copy for the backward pass, bf16 for the next layer.
__global__ void k_epi_tanh(const float* __restrict__ part, int splits, int M, int N,
                           const float* __restrict__ bias, float* __restrict__ hf,
                           bf16_t* __restrict__ hb) {
  const long long MN = (long long)M * N;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < MN;
       i += (long long)gridDim.x * blockDim.x) {
    const float v = tanhf(sum_parts(part, splits, MN, i) + bias[i % N]);
    hf[i] = v;
    hb[i] = to_bf16(v);
  }
}

// y = sum + bias (network output, FP32).
__global__ void k_epi_out(const float* __restrict__ part, int splits, int M, int N,
                          const float* __restrict__ bias, float* __restrict__ y) {
  const long long MN = (long long)M * N;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < MN;
       i += (long long)gridDim.x * blockDim.x)
    y[i] = sum_parts(part, splits, MN, i) + bias[i % N];
}

// g = bf16(sum * (1 - h^2)): gradient at the pre-activation of a tanh layer.
__global__ void k_epi_tanh_grad(const float* __restrict__ part, int splits, int M, int N,
                                const float* __restrict__ h, bf16_t* __restrict__ g) {
  const long long MN = (long long)M * N;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < MN;
       i += (long long)gridDim.x * blockDim.x) {
    const float hv = h[i];
    g[i] = to_bf16(sum_parts(part, splits, MN, i) * (1.f - hv * hv));
  }
}

// Weight gradient: part is [Cout][(d, c)] -> grad W[o][c][d].
__global__ void k_epi_dw(const float* __restrict__ part, int splits, int Cout, int Cin,
                         float* __restrict__ gW) {
  const long long MN = (long long)Cout * kWidth * Cin;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < MN;
       i += (long long)gridDim.x * blockDim.x) {
    const int o = (int)(i / (kWidth * Cin));
    const int col = (int)(i % (kWidth * Cin));
    const int d = col / Cin, c = col % Cin;
    gW[((long long)o * Cin + c) * kWidth + d] = sum_parts(part, splits, MN, i);
  }
}

// Bias gradient: db[o] = sum over rows of g[r][o] (fixed order).
__global__ void k_colsum(const bf16_t* __restrict__ g, int rows, int N, float* __restrict__ db) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= N) return;
  float s = 0.f;
  for (int r = 0; r < rows; ++r) s += __uint_as_float((uint32_t)g[(long long)r * N + o] << 16);
  db[o] = s;
}

// Mean squared error: g = bf16(2 (y - target) / count), per-work-group
// partial sums of (y - target)^2 in FP64.
__global__ void k_mse(const float* __restrict__ y, const float* __restrict__ Y,
                      const int* __restrict__ idx, int count, int batch, int TC,
                      bf16_t* __restrict__ g, double* __restrict__ partial) {
  __shared__ double red[kEpiThreads / kWave];
  const long long total = (long long)batch * TC;
  const float scale = 2.f / (float)total;
  double acc = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    const long long s = i / TC, e = i % TC;
    const long long smp = idx ? idx[s] : s;
    const bool ok = smp >= 0 && smp < count;
    const float d = y[i] - (ok ? Y[smp * TC + e] : 0.f);
    g[i] = to_bf16(scale * d);
    acc += (double)d * (double)d;
  }
  acc = wave_sum(acc);
  if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kEpiThreads / kWave; ++w) s += red[w];
    partial[blockIdx.x] = s;
  }
}

__global__ void k_sum_partials(const double* __restrict__ partial, int n, double scale,
                               double* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += partial[i];
    *out = s * scale;
  }
}

// dy given in FP32 -> bf16 output gradient.
__global__ void k_round(const float* __restrict__ x, long long n, bf16_t* __restrict__ out) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    out[i] = to_bf16(x[i]);
}

__global__ void k_adam(float* __restrict__ theta, const float* __restrict__ g,
                       float* __restrict__ m, float* __restrict__ v, long long n, float lr,
                       float b1, float b2, float eps, float bc1, float bc2) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    theta[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
  }
}

// bf16 weight layouts from the FP32 master W[o][c][d] (Cout x Cin):
// fwd[o][d*Cin + c] (B of the forward GEMM), bwd[c][d*Cout + o] (B of the
// input-gradient GEMM; NULL to skip).
__global__ void k_prep_weights(const float* __restrict__ W, int Cout, int Cin,
                               bf16_t* __restrict__ fwd, bf16_t* __restrict__ bwd) {
  const long long n = (long long)Cout * Cin * kWidth;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const int d = (int)(i % kWidth);
    const int c = (int)((i / kWidth) % Cin);
    const int o = (int)(i / ((long long)kWidth * Cin));
    const bf16_t b = to_bf16(W[i]);
    fwd[(long long)o * kWidth * Cin + (long long)d * Cin + c] = b;
    if (bwd) bwd[(long long)c * kWidth * Cout + (long long)d * Cout + o] = b;
  }
}

// Offset in a type-major coarse vector of node-major entry (t, ch).
__device__ __forceinline__ long long type_index(int t, int ch, int p, int q, int T) {
  const long long Tp = (long long)T * p, Tq = (long long)T * q;
  if (ch < p) return (long long)t * p + ch;
  if (ch < 2 * p) return Tp + (long long)t * p + (ch - p);
  if (ch < 2 * p + q) return 2 * Tp + (long long)t * q + (ch - 2 * p);
  if (ch < 3 * p + q) return 2 * Tp + Tq + (long long)t * p + (ch - 2 * p - q);
  return 3 * Tp + Tq + (long long)t * p + (ch - 3 * p - q);
}

constexpr int kPackThreads = 1024;

// One work-group per sample: s = rms(r); x = node-major r / s (and, for
// training pairs, y = node-major e / s).  s = 0 gives zeros.  s_out: the
// scale of sample 0 (inference).
__global__ __launch_bounds__(kPackThreads) void k_pack(const double* __restrict__ r,
                                                       const double* __restrict__ e, int p,
                                                       int q, int T, float* __restrict__ x,
                                                       float* __restrict__ y,
                                                       double* __restrict__ s_out) {
  __shared__ double red[kPackThreads / kWave];
  __shared__ double sc;
  const int C = 4 * p + q;
  const long long len = (long long)C * T;
  const double* rs = r + blockIdx.x * len;
  double acc = 0.0;
  for (long long i = threadIdx.x; i < len; i += kPackThreads) acc += rs[i] * rs[i];
  acc = wave_sum(acc);
  if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kPackThreads / kWave; ++w) s += red[w];
    sc = sqrt(s / (double)len);
    if (s_out && blockIdx.x == 0) *s_out = sc;
  }
  __syncthreads();
  const double s = sc;
  const double inv = s > 0.0 ? 1.0 / s : 0.0;
  for (long long i = threadIdx.x; i < len; i += kPackThreads) {
    const int t = (int)(i / C), ch = (int)(i % C);
    const long long ti = type_index(t, ch, p, q, T);
    x[blockIdx.x * len + i] = (float)(rs[ti] * inv);
    if (e) y[blockIdx.x * len + i] = (float)(e[blockIdx.x * len + ti] * inv);
  }
}

// Inference output: e_type = s * (sum + b3), scattered to type-major order.
__global__ void k_epi_coarse(const float* __restrict__ part, int splits, int T, int C,
                             const float* __restrict__ bias, const double* __restrict__ s_in,
                             int p, int q, double* __restrict__ e) {
  const long long MN = (long long)T * C;
  const double s = *s_in;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < MN;
       i += (long long)gridDim.x * blockDim.x) {
    const int t = (int)(i / C), ch = (int)(i % C);
    const float yv = sum_parts(part, splits, MN, i) + bias[ch];
    e[type_index(t, ch, p, q, T)] = s * (double)yv;
  }
}

int grid_1d(long long n, int threads) {
  long long g = (n + threads - 1) / threads;
  return (int)std::max<long long>(1, std::min<long long>(g, 4096));
}

struct Split {
  int splits, kchunk;
};

// K split so that the launch has about 256 work-groups.
Split split_k(int M, int N, int K) {
  const int tiles = ((M + kBM - 1) / kBM) * ((N + kBN - 1) / kBN);
  const int kch = (K + kBK - 1) / kBK;
  int s = std::max(1, std::min(kch, (256 + tiles - 1) / tiles));
  const int per = (kch + s - 1) / s;
  Split r;
  r.kchunk = per * kBK;
  r.splits = (K + r.kchunk - 1) / r.kchunk;
  return r;
}

size_t part_floats(int M, int N, int K) {
  const Split s = split_k(M, N, K);
  return (size_t)s.splits * M * N;
}

}  // namespace

struct pitmg_net {
  hipStream_t stream = nullptr;
  int C = 0, T = 0, H = 0, maxB = 0;
  long long P = 0;
  long long oW1 = 0, ob1 = 0, oW2 = 0, ob2 = 0, oW3 = 0, ob3 = 0;
  float *theta = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
  int t_adam = 0;
  bf16_t *W1f = nullptr, *W2f = nullptr, *W3f = nullptr, *W2b = nullptr, *W3b = nullptr;
  float *h1f = nullptr, *h2f = nullptr, *y = nullptr, *xin = nullptr;
  bf16_t *h1b = nullptr, *h2b = nullptr, *g1 = nullptr, *g2 = nullptr, *g3 = nullptr;
  float* part = nullptr;
  size_t part_cap = 0;
  double *lossp = nullptr, *loss = nullptr, *scale = nullptr;
  std::string err;
};

namespace {

int net_err(pitmg_net* n, int code, const std::string& msg) {
  if (n) n->err = msg;
  return code;
}

#define NETCHK(n, call)                                                             \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess)                                                           \
      return net_err(n, PITMG_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <class SA, class SB>
hipError_t gemm(pitmg_net* n, const SA& a, const SB& b, int M, int N, int K, Split* used,
                hipStream_t s) {
  const Split sp = split_k(M, N, K);
  if ((size_t)sp.splits * M * N > n->part_cap) return hipErrorInvalidValue;
  dim3 grid((N + kBN - 1) / kBN, (M + kBM - 1) / kBM, sp.splits);
  hipLaunchKernelGGL((k_gemm<SA, SB>), grid, dim3(kGemmThreads), 0, s, a, b, M, N, K,
                     sp.kchunk, n->part);
  *used = sp;
  return hipGetLastError();
}

Im2col conv_rows(const bf16_t* bf, const float* f32, const int* idx, int T, int Cin, int rows,
                 int dir, int count = 0) {
  Im2col a;
  a.bf = bf;
  a.f32 = f32;
  a.idx = idx;
  a.count = count;
  a.T = T;
  a.Cin = Cin;
  a.rows = rows;
  a.dir = dir;
  return a;
}

hipError_t prep_weights(pitmg_net* n, hipStream_t s) {
  const int C = n->C, H = n->H;
  hipLaunchKernelGGL(k_prep_weights, dim3(grid_1d((long long)H * C * kWidth, 256)), dim3(256), 0,
                     s, n->theta + n->oW1, H, C, n->W1f, (bf16_t*)nullptr);
  hipLaunchKernelGGL(k_prep_weights, dim3(grid_1d((long long)H * H * kWidth, 256)), dim3(256), 0,
                     s, n->theta + n->oW2, H, H, n->W2f, n->W2b);
  hipLaunchKernelGGL(k_prep_weights, dim3(grid_1d((long long)C * H * kWidth, 256)), dim3(256), 0,
                     s, n->theta + n->oW3, C, H, n->W3f, n->W3b);
  return hipGetLastError();
}

// Forward over `batch` samples of x (FP32, optional gather): leaves h1f/h1b,
// h2f/h2b in the network's buffers and the output either in y_out (FP32
// [batch][T][C]) or, when e_type is given, scattered to a type-major FP64
// coarse vector times *scale.
hipError_t forward(pitmg_net* n, int batch, const float* x, const int* idx, int count,
                   float* y_out, double* e_type, int p, int q, hipStream_t s) {
  const int T = n->T, C = n->C, H = n->H, R = batch * T;
  Split sp;
  hipError_t e;
  RowsAsCols w1{n->W1f, kWidth * C, kWidth * C, H};
  if ((e = gemm(n, conv_rows(nullptr, x, idx, T, C, R, 1, count), w1, R, H, kWidth * C, &sp, s)))
    return e;
  hipLaunchKernelGGL(k_epi_tanh, dim3(grid_1d((long long)R * H, kEpiThreads)), dim3(kEpiThreads),
                     0, s, n->part, sp.splits, R, H, n->theta + n->ob1, n->h1f, n->h1b);
  RowsAsCols w2{n->W2f, kWidth * H, kWidth * H, H};
  if ((e = gemm(n, conv_rows(n->h1b, nullptr, nullptr, T, H, R, 1), w2, R, H, kWidth * H, &sp,
                s)))
    return e;
  hipLaunchKernelGGL(k_epi_tanh, dim3(grid_1d((long long)R * H, kEpiThreads)), dim3(kEpiThreads),
                     0, s, n->part, sp.splits, R, H, n->theta + n->ob2, n->h2f, n->h2b);
  RowsAsCols w3{n->W3f, kWidth * H, kWidth * H, C};
  if ((e = gemm(n, conv_rows(n->h2b, nullptr, nullptr, T, H, R, 1), w3, R, C, kWidth * H, &sp,
                s)))
    return e;
  if (e_type) {
    hipLaunchKernelGGL(k_epi_coarse, dim3(grid_1d((long long)T * C, kEpiThreads)),
                       dim3(kEpiThreads), 0, s, n->part, sp.splits, T, C, n->theta + n->ob3,
                       n->scale, p, q, e_type);
  } else {
    hipLaunchKernelGGL(k_epi_out, dim3(grid_1d((long long)R * C, kEpiThreads)),
                       dim3(kEpiThreads), 0, s, n->part, sp.splits, R, C, n->theta + n->ob3,
                       y_out);
  }
  return hipGetLastError();
}

// Backward from the bf16 output gradient in g3 (rows R = batch*T) to the
// parameter gradient in n->grad; the forward activations must be in place.
hipError_t backward(pitmg_net* n, int batch, const float* x, const int* idx, int count,
                    hipStream_t s) {
  const int T = n->T, C = n->C, H = n->H, R = batch * T;
  float* gr = n->grad;
  Split sp;
  hipError_t e;
  const int eg = kEpiThreads;
  // layer 3: dW3 = g3^T im2col(h2), db3, dh2 = im2col_rev(g3) W3
  if ((e = gemm(n, Transposed{n->g3, C, C, R}, conv_rows(n->h2b, nullptr, nullptr, T, H, R, 1),
                C, kWidth * H, R, &sp, s)))
    return e;
  hipLaunchKernelGGL(k_epi_dw, dim3(grid_1d((long long)C * kWidth * H, eg)), dim3(eg), 0, s,
                     n->part, sp.splits, C, H, gr + n->oW3);
  hipLaunchKernelGGL(k_colsum, dim3((C + 255) / 256), dim3(256), 0, s, n->g3, R, C, gr + n->ob3);
  if ((e = gemm(n, conv_rows(n->g3, nullptr, nullptr, T, C, R, -1),
                RowsAsCols{n->W3b, kWidth * C, kWidth * C, H}, R, H, kWidth * C, &sp, s)))
    return e;
  hipLaunchKernelGGL(k_epi_tanh_grad, dim3(grid_1d((long long)R * H, eg)), dim3(eg), 0, s,
                     n->part, sp.splits, R, H, n->h2f, n->g2);
  // layer 2
  if ((e = gemm(n, Transposed{n->g2, H, H, R}, conv_rows(n->h1b, nullptr, nullptr, T, H, R, 1),
                H, kWidth * H, R, &sp, s)))
    return e;
  hipLaunchKernelGGL(k_epi_dw, dim3(grid_1d((long long)H * kWidth * H, eg)), dim3(eg), 0, s,
                     n->part, sp.splits, H, H, gr + n->oW2);
  hipLaunchKernelGGL(k_colsum, dim3((H + 255) / 256), dim3(256), 0, s, n->g2, R, H, gr + n->ob2);
  if ((e = gemm(n, conv_rows(n->g2, nullptr, nullptr, T, H, R, -1),
                RowsAsCols{n->W2b, kWidth * H, kWidth * H, H}, R, H, kWidth * H, &sp, s)))
    return e;
  hipLaunchKernelGGL(k_epi_tanh_grad, dim3(grid_1d((long long)R * H, eg)), dim3(eg), 0, s,
                     n->part, sp.splits, R, H, n->h1f, n->g1);
  // layer 1 (no input gradient needed)
  if ((e = gemm(n, Transposed{n->g1, H, H, R}, conv_rows(nullptr, x, idx, T, C, R, 1, count), H,
                kWidth * C, R, &sp, s)))
    return e;
  hipLaunchKernelGGL(k_epi_dw, dim3(grid_1d((long long)H * kWidth * C, eg)), dim3(eg), 0, s,
                     n->part, sp.splits, H, C, gr + n->oW1);
  hipLaunchKernelGGL(k_colsum, dim3((H + 255) / 256), dim3(256), 0, s, n->g1, R, H, gr + n->ob1);
  return hipGetLastError();
}

hipError_t adam(pitmg_net* n, const float* g, float lr, hipStream_t s) {
  n->t_adam += 1;
  const double b1 = 0.9, b2 = 0.999;
  const float bc1 = (float)(1.0 - std::pow(b1, n->t_adam));
  const float bc2 = (float)(1.0 - std::pow(b2, n->t_adam));
  hipLaunchKernelGGL(k_adam, dim3(grid_1d(n->P, 256)), dim3(256), 0, s, n->theta, g, n->m, n->v,
                     n->P, lr, (float)b1, (float)b2, 1e-8f, bc1, bc2);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return prep_weights(n, s);
}

int check_batch(pitmg_net* n, int batch) {
  if (batch < 1 || batch > n->maxB)
    return net_err(n, PITMG_ERR_INVALID, "batch must be in [1, max_batch]");
  return PITMG_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// internal entry for the solver's coarse level
// ---------------------------------------------------------------------------

namespace pitmg {

bool net_matches(const pitmg_net* n, int C, int T) { return n && n->C == C && n->T == T; }

// e_type = s * net(r / s) for one type-major coarse vector, on stream s.
hipError_t net_coarse_correction(pitmg_net* n, const double* r, double* e, int p, int q,
                                 hipStream_t s) {
  hipLaunchKernelGGL(k_pack, dim3(1), dim3(kPackThreads), 0, s, r, (const double*)nullptr, p, q,
                     n->T, n->xin, (float*)nullptr, n->scale);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  return forward(n, 1, n->xin, nullptr, 0, nullptr, e, p, q, s);
}

}  // namespace pitmg

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" {

long long pitmg_net_param_count(int C, int H) {
  if (C < 1 || H < 1) return 0;
  return (long long)H * C * kWidth + H + (long long)H * H * kWidth + H +
         (long long)C * H * kWidth + C;
}

void pitmg_net_destroy(pitmg_net* n) {
  if (!n) return;
  void* ptrs[] = {n->theta, n->m,   n->v,   n->grad, n->W1f,  n->W2f, n->W3f, n->W2b,
                  n->W3b,   n->h1f, n->h2f, n->y,    n->xin,  n->h1b, n->h2b, n->g1,
                  n->g2,    n->g3,  n->part, n->lossp, n->loss, n->scale};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete n;
}

int pitmg_net_create(pitmg_net** out, int C, int T, int H, int max_batch, void* stream) {
  if (!out) return PITMG_ERR_INVALID;
  *out = nullptr;
  if (C < 1 || T < 1 || H < 1 || max_batch < 1) return PITMG_ERR_INVALID;
  if ((long long)max_batch * T * std::max(C, H) > (1LL << 30)) return PITMG_ERR_UNSUPPORTED;
  pitmg_net* n = new pitmg_net;
  n->stream = (hipStream_t)stream;
  n->C = C;
  n->T = T;
  n->H = H;
  n->maxB = max_batch;
  n->P = pitmg_net_param_count(C, H);
  n->oW1 = 0;
  n->ob1 = n->oW1 + (long long)H * C * kWidth;
  n->oW2 = n->ob1 + H;
  n->ob2 = n->oW2 + (long long)H * H * kWidth;
  n->oW3 = n->ob2 + H;
  n->ob3 = n->oW3 + (long long)C * H * kWidth;
  const long long R = (long long)max_batch * T;
  const int K1 = kWidth * C, K2 = kWidth * H;
  size_t pc = 0;
  for (int rows : {(int)R, T}) {
    pc = std::max(pc, part_floats(rows, H, K1));
    pc = std::max(pc, part_floats(rows, H, K2));
    pc = std::max(pc, part_floats(rows, C, K2));
  }
  pc = std::max(pc, part_floats(C, K2, (int)R));
  pc = std::max(pc, part_floats(H, K2, (int)R));
  pc = std::max(pc, part_floats(H, K1, (int)R));
  pc = std::max(pc, part_floats((int)R, H, K1));
  // a smaller batch has fewer tiles and so more K splits: with at most 256
  // tiles, splits * M * N stays below (256 + tiles) * kBM * kBN
  pc = std::max(pc, (size_t)512 * kBM * kBN);
  n->part_cap = pc;
  const size_t pb = (size_t)n->P * 4;
  struct A {
    void** p;
    size_t bytes;
  } allocs[] = {
      {(void**)&n->theta, pb},                 {(void**)&n->m, pb},
      {(void**)&n->v, pb},                     {(void**)&n->grad, pb},
      {(void**)&n->W1f, (size_t)H * K1 * 2},   {(void**)&n->W2f, (size_t)H * K2 * 2},
      {(void**)&n->W3f, (size_t)C * K2 * 2},   {(void**)&n->W2b, (size_t)H * K2 * 2},
      {(void**)&n->W3b, (size_t)H * K1 * 2},   {(void**)&n->h1f, (size_t)R * H * 4},
      {(void**)&n->h2f, (size_t)R * H * 4},    {(void**)&n->y, (size_t)R * C * 4},
      {(void**)&n->xin, (size_t)T * C * 4},    {(void**)&n->h1b, (size_t)R * H * 2},
      {(void**)&n->h2b, (size_t)R * H * 2},    {(void**)&n->g1, (size_t)R * H * 2},
      {(void**)&n->g2, (size_t)R * H * 2},     {(void**)&n->g3, (size_t)R * C * 2},
      {(void**)&n->part, pc * 4},              {(void**)&n->lossp, 4096 * 8},
      {(void**)&n->loss, 8},                   {(void**)&n->scale, 8},
  };
  for (auto& a : allocs) {
    if (hipMalloc(a.p, a.bytes) != hipSuccess) {
      *a.p = nullptr;
      pitmg_net_destroy(n);
      return PITMG_ERR_OOM;
    }
  }
  hipError_t e = hipMemsetAsync(n->theta, 0, n->P * 4, n->stream);
  if (e == hipSuccess) e = hipMemsetAsync(n->m, 0, n->P * 4, n->stream);
  if (e == hipSuccess) e = hipMemsetAsync(n->v, 0, n->P * 4, n->stream);
  if (e == hipSuccess) e = prep_weights(n, n->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
  if (e != hipSuccess) {
    pitmg_net_destroy(n);
    return PITMG_ERR_HIP;
  }
  *out = n;
  return PITMG_OK;
}

int pitmg_net_set_params(pitmg_net* n, const float* theta, int on_device) {
  if (!n || !theta) return PITMG_ERR_INVALID;
  NETCHK(n, hipMemcpyAsync(n->theta, theta, n->P * 4,
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                           n->stream));
  NETCHK(n, hipMemsetAsync(n->m, 0, n->P * 4, n->stream));
  NETCHK(n, hipMemsetAsync(n->v, 0, n->P * 4, n->stream));
  n->t_adam = 0;
  NETCHK(n, prep_weights(n, n->stream));
  NETCHK(n, hipStreamSynchronize(n->stream));
  return PITMG_OK;
}

int pitmg_net_get_params(pitmg_net* n, float* theta_host) {
  if (!n || !theta_host) return PITMG_ERR_INVALID;
  NETCHK(n, hipMemcpyAsync(theta_host, n->theta, n->P * 4, hipMemcpyDeviceToHost, n->stream));
  NETCHK(n, hipStreamSynchronize(n->stream));
  return PITMG_OK;
}

int pitmg_net_forward(pitmg_net* n, int batch, const float* x, float* y) {
  if (!n || !x || !y) return PITMG_ERR_INVALID;
  if (int rc = check_batch(n, batch)) return rc;
  NETCHK(n, forward(n, batch, x, nullptr, 0, y, nullptr, 0, 0, n->stream));
  NETCHK(n, hipStreamSynchronize(n->stream));
  return PITMG_OK;
}

int pitmg_net_backward(pitmg_net* n, int batch, const float* x, const float* dy, float* grad) {
  if (!n || !x || !dy || !grad) return PITMG_ERR_INVALID;
  if (int rc = check_batch(n, batch)) return rc;
  const long long RC = (long long)batch * n->T * n->C;
  NETCHK(n, forward(n, batch, x, nullptr, 0, n->y, nullptr, 0, 0, n->stream));
  hipLaunchKernelGGL(k_round, dim3(grid_1d(RC, 256)), dim3(256), 0, n->stream, dy, RC, n->g3);
  NETCHK(n, hipGetLastError());
  NETCHK(n, backward(n, batch, x, nullptr, 0, n->stream));
  NETCHK(n, hipMemcpyAsync(grad, n->grad, n->P * 4, hipMemcpyDeviceToDevice, n->stream));
  NETCHK(n, hipStreamSynchronize(n->stream));
  return PITMG_OK;
}

int pitmg_net_adam(pitmg_net* n, const float* grad, float lr) {
  if (!n || !grad) return PITMG_ERR_INVALID;
  NETCHK(n, adam(n, grad, lr, n->stream));
  NETCHK(n, hipStreamSynchronize(n->stream));
  return PITMG_OK;
}

int pitmg_net_train_step(pitmg_net* n, int batch, const int* idx, int count, const float* X,
                         const float* Y, float lr, double* loss) {
  if (!n || !idx || !X || !Y || count < 1) return PITMG_ERR_INVALID;
  if (int rc = check_batch(n, batch)) return rc;
  hipStream_t s = n->stream;
  const int TC = n->T * n->C;
  NETCHK(n, forward(n, batch, X, idx, count, n->y, nullptr, 0, 0, s));
  const int g = std::min(grid_1d((long long)batch * TC, kEpiThreads), 4096);
  hipLaunchKernelGGL(k_mse, dim3(g), dim3(kEpiThreads), 0, s, n->y, Y, idx, count, batch, TC,
                     n->g3, n->lossp);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64), 0, s, n->lossp, g,
                     1.0 / ((double)batch * TC), n->loss);
  NETCHK(n, hipGetLastError());
  NETCHK(n, backward(n, batch, X, idx, count, s));
  NETCHK(n, adam(n, n->grad, lr, s));
  if (loss) {
    NETCHK(n, hipMemcpyAsync(loss, n->loss, 8, hipMemcpyDeviceToHost, s));
  }
  NETCHK(n, hipStreamSynchronize(s));
  return PITMG_OK;
}

int pitmg_net_make_samples(pitmg_net* n, int count, int p, int q, const double* r,
                           const double* e, float* X, float* Y) {
  if (!n || !r || !e || !X || !Y || count < 0) return PITMG_ERR_INVALID;
  if (p < 1 || q < 1 || 4 * p + q != n->C)
    return net_err(n, PITMG_ERR_INVALID, "4p+q must equal the network's channel count");
  if (count == 0) return PITMG_OK;
  hipLaunchKernelGGL(k_pack, dim3(count), dim3(kPackThreads), 0, n->stream, r, e, p, q, n->T, X,
                     Y, (double*)nullptr);
  NETCHK(n, hipGetLastError());
  NETCHK(n, hipStreamSynchronize(n->stream));
  return PITMG_OK;
}

const char* pitmg_net_last_error(const pitmg_net* n) { return n ? n->err.c_str() : ""; }

}  // extern "C"
