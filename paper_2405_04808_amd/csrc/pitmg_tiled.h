// Register-tiled solve of one time-step block D_k x = r for p = q = 32*RT =
// 16*CT with 512 threads (8 waves).
//
// Thread (a, b) = (tid / 16, tid % 16) owns rows [RT a, RT a + RT) and the
// CT columns 2b + 32c + e (c < CT/2, e < 2) of N_k and of the inverse
// Cholesky factor G_k^{-1}, so each 16-byte load instruction of a wave reads
// four fully used 256-byte row segments.  Both tiles stay in registers, so
// every entry is read once and
// serves the row products (t = N r_u + ..., s = G^{-1} t) and the column
// products (lambda = G^{-T} s, N^T lambda).  Row sums reduce over the 16
// lanes that share a; column sums over the 4 row groups of a wave (lane xor
// 16, 32) and then over the 8 waves through LDS, in a fixed order.  V_k and
// Z~_k are read in the same tile shape (from L2 when shared by every step).
// Block algebra: the Schur form documented in pitmg_kernels.hip.
#pragma once
#include "pitmg_internal.h"
#include "pitmg_device.h"

namespace pitmg {

constexpr int kTiledThreads = 512;
constexpr int kTiledWaves = kTiledThreads / kWave;

// Column of the thread's c-th tile entry (c < CT): 2b + 32 (c / 2) + c % 2.
__device__ __forceinline__ int tile_col(int c) { return 2 * (threadIdx.x % 16) + 32 * (c >> 1) + (c & 1); }

// Load the thread's CT entries of one row (row points at the row start).
template <int CT>
__device__ __forceinline__ void tile_load_row(const double* __restrict__ row, double (&dst)[CT]) {
  const double* src = row + 2 * (threadIdx.x % 16);
#pragma unroll
  for (int c = 0; c < CT; c += 2) {
    const double2 v = *reinterpret_cast<const double2*>(src + 16 * c);
    dst[c] = v.x;
    dst[c + 1] = v.y;
  }
}

// Same for a lower-triangular row i: pairs wholly above the diagonal are
// zero in memory and are not loaded.
template <int CT>
__device__ __forceinline__ void tile_load_row_lower(const double* __restrict__ row, int i,
                                                    double (&dst)[CT]) {
  const int j0 = 2 * (threadIdx.x % 16);
  const double* src = row + j0;
#pragma unroll
  for (int c = 0; c < CT; c += 2) {
    if (j0 + 16 * c <= i) {
      const double2 v = *reinterpret_cast<const double2*>(src + 16 * c);
      dst[c] = v.x;
      dst[c + 1] = v.y;
    } else {
      dst[c] = 0.0;
      dst[c + 1] = 0.0;
    }
  }
}

__device__ __forceinline__ double tile_sum16(double v) {
  v += __shfl_xor(v, 8, kWave);
  v += __shfl_xor(v, 4, kWave);
  v += __shfl_xor(v, 2, kWave);
  v += __shfl_xor(v, 1, kWave);
  return v;
}

template <int RT, int CT>
struct TiledSolve {
  static constexpr int P = 32 * RT;
  static_assert(P == 16 * CT, "tile shape");
  static constexpr int kThreads = kTiledThreads;

  struct Regs {
    double nt[RT][CT];
    double gt[RT][CT];
  };
  // LDS scratch (doubles): t, s, then three [waves][P] reduction slabs.
  static constexpr size_t kScratch = 2 * P + 3 * kTiledWaves * P;

  // Issue the loads of the N_k and G_k^{-1} tiles of step kk (0-based).
  __device__ __forceinline__ static void load(const LevelView& L, long long kk, Regs& R) {
    load_n(L, kk, R);
    load_g(L, kk, R);
  }

  __device__ __forceinline__ static void load_n(const LevelView& L, long long kk, Regs& R) {
    const int r0 = RT * (threadIdx.x / 16);
    const double* __restrict__ Nk = L.N + kk * L.sN;
#pragma unroll
    for (int r = 0; r < RT; ++r) tile_load_row<CT>(Nk + (long long)(r0 + r) * P, R.nt[r]);
  }

  __device__ __forceinline__ static void load_g(const LevelView& L, long long kk, Regs& R) {
    const int r0 = RT * (threadIdx.x / 16);
    const double* __restrict__ Gk = L.Gi + kk * (long long)P * P;
#pragma unroll
    for (int r = 0; r < RT; ++r)
      tile_load_row_lower<CT>(Gk + (long long)(r0 + r) * P, r0 + r, R.gt[r]);
  }

  // Column partials of one thread -> per-wave slot of red (lanes 0..15).
  __device__ __forceinline__ static void col_partial(double (&v)[CT], double* red) {
    const int tid = threadIdx.x, lane = tid % kWave, w = tid / kWave;
#pragma unroll
    for (int c = 0; c < CT; ++c) {
      v[c] += __shfl_xor(v[c], 16, kWave);
      v[c] += __shfl_xor(v[c], 32, kWave);
    }
    if (lane < 16) {
#pragma unroll
      for (int c = 0; c < CT; ++c) red[w * P + tile_col(c)] = v[c];
    }
  }

  __device__ __forceinline__ static double col_total(const double* red, int j) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kTiledWaves; ++w) s += red[w * P + j];
    return s;
  }

  // Solve with the right-hand side in LDS (r_v, r_u, r_z, r_l, r_m; r_v and
  // r_m unused when !hv).  Results: lambda in ol; N^T lambda, Z^T lambda and
  // V^T lambda are left in the reduction slabs and combined by finish().
  __device__ __forceinline__ static void solve(const LevelView& L, long long kk, bool hv,
                                               const Regs& R, const double* sru,
                                               const double* srz, const double* srm,
                                               const double* srl, double* ol, double* scr) {
    const int tid = threadIdx.x, a = tid / 16, bq = tid % 16;
    const int r0 = RT * a;
    double* st = scr;
    double* ss = scr + P;
    double* red = scr + 2 * P;
    const double* __restrict__ Vk = L.V + kk * L.sV;
    const double* __restrict__ Zk = L.Z + kk * L.sZ;
    // t = N r_u + Z r_z - V r_m - r_l
    double acc[RT];
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      double s = 0.0;
#pragma unroll
      for (int c = 0; c < CT; ++c) s += R.nt[r][c] * sru[tile_col(c)];
      double zr[CT];
      tile_load_row<CT>(Zk + (long long)(r0 + r) * P, zr);
#pragma unroll
      for (int c = 0; c < CT; ++c) s += zr[c] * srz[tile_col(c)];
      if (hv) {
        double vr[CT];
        tile_load_row<CT>(Vk + (long long)(r0 + r) * P, vr);
#pragma unroll
        for (int c = 0; c < CT; ++c) s -= vr[c] * srm[tile_col(c)];
      }
      acc[r] = tile_sum16(s);
    }
    if (bq == 0) {
#pragma unroll
      for (int r = 0; r < RT; ++r) st[r0 + r] = acc[r] - srl[r0 + r];
    }
    __syncthreads();
    // s = G^{-1} t
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      double s = 0.0;
#pragma unroll
      for (int c = 0; c < CT; ++c) s += R.gt[r][c] * st[tile_col(c)];
      acc[r] = tile_sum16(s);
    }
    if (bq == 0) {
#pragma unroll
      for (int r = 0; r < RT; ++r) ss[r0 + r] = acc[r];
    }
    __syncthreads();
    // lambda = G^{-T} s
    double cacc[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) {
      double s = 0.0;
#pragma unroll
      for (int r = 0; r < RT; ++r) s += R.gt[r][c] * ss[r0 + r];
      cacc[c] = s;
    }
    col_partial(cacc, red);
    __syncthreads();
    for (int j = tid; j < P; j += kThreads) ol[j] = col_total(red, j);
    __syncthreads();
    // N^T lambda, Z^T lambda, V^T lambda -> slabs 0, 1, 2
#pragma unroll
    for (int c = 0; c < CT; ++c) {
      double s = 0.0;
#pragma unroll
      for (int r = 0; r < RT; ++r) s += R.nt[r][c] * ol[r0 + r];
      cacc[c] = s;
    }
    col_partial(cacc, red);
    {
      double zacc[CT];
#pragma unroll
      for (int c = 0; c < CT; ++c) zacc[c] = 0.0;
#pragma unroll
      for (int r = 0; r < RT; ++r) {
        double zr[CT];
        tile_load_row<CT>(Zk + (long long)(r0 + r) * P, zr);
#pragma unroll
        for (int c = 0; c < CT; ++c) zacc[c] += zr[c] * ol[r0 + r];
      }
      col_partial(zacc, red + kTiledWaves * P);
    }
    if (hv) {
      double vacc[CT];
#pragma unroll
      for (int c = 0; c < CT; ++c) vacc[c] = 0.0;
#pragma unroll
      for (int r = 0; r < RT; ++r) {
        double vr[CT];
        tile_load_row<CT>(Vk + (long long)(r0 + r) * P, vr);
#pragma unroll
        for (int c = 0; c < CT; ++c) vacc[c] += vr[c] * ol[r0 + r];
      }
      col_partial(vacc, red + 2 * kTiledWaves * P);
    }
    __syncthreads();
  }

  // Component i of the solution after solve():
  //   u = r_u - N^T lambda, z = r_z - Z^T lambda, mu = V^T lambda - r_m - r_v,
  //   v = -r_m   (lambda is ol[i]).
  __device__ __forceinline__ static double u_of(const double* scr, const double* sru, int i) {
    return sru[i] - col_total(scr + 2 * P, i);
  }
  __device__ __forceinline__ static double z_of(const double* scr, const double* srz, int i) {
    return srz[i] - col_total(scr + 2 * P + kTiledWaves * P, i);
  }
  __device__ __forceinline__ static double mu_of(const double* scr, const double* srm,
                                                 const double* srv, int i) {
    return col_total(scr + 2 * P + 2 * kTiledWaves * P, i) - srm[i] - srv[i];
  }
};

}  // namespace pitmg
