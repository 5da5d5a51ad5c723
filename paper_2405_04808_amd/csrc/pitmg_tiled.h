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

// 16-byte vector of the tile element type.
template <class T>
struct Vec16;
template <>
struct Vec16<double> {
  using type = double2;
  static constexpr int n = 2;
  __device__ static void put(const type& v, double* d) {
    d[0] = v.x;
    d[1] = v.y;
  }
};
template <>
struct Vec16<float> {
  using type = float4;
  static constexpr int n = 4;
  __device__ static void put(const type& v, float* d) {
    d[0] = v.x;
    d[1] = v.y;
    d[2] = v.z;
    d[3] = v.w;
  }
};

// Column of the thread's c-th tile entry (c < CT), with E = 16/sizeof(T)
// elements per load: E b + 16 E (c / E) + c % E.
template <class T>
__device__ __forceinline__ int tile_col(int c) {
  constexpr int E = Vec16<T>::n;
  return E * (threadIdx.x % 16) + 16 * E * (c / E) + c % E;
}

// Load the thread's CT entries of one row (row points at the row start).
template <int CT, class T>
__device__ __forceinline__ void tile_load_row(const T* __restrict__ row, T (&dst)[CT]) {
  constexpr int E = Vec16<T>::n;
  const T* src = row + E * (threadIdx.x % 16);
#pragma unroll
  for (int c = 0; c < CT; c += E)
    Vec16<T>::put(*reinterpret_cast<const typename Vec16<T>::type*>(src + 16 * c), dst + c);
}

// Same for a lower-triangular row i: vectors wholly above the diagonal are
// zero in memory and are not fetched.  Every lane still issues every load
// (such a lane re-reads its first vector, a line it has just requested, and
// zeroes the result), so the loads are straight-line code: the compiler can
// then wait for loads issued before the tile without waiting for the tile.
template <int CT, class T>
__device__ __forceinline__ void tile_load_row_lower(const T* __restrict__ row, int i,
                                                    T (&dst)[CT]) {
  constexpr int E = Vec16<T>::n;
  const int j0 = E * (threadIdx.x % 16);
  const T* src = row + j0;
#pragma unroll
  for (int c = 0; c < CT; c += E) {
    const bool in = j0 + 16 * c <= i;
    const T* a = in ? src + 16 * c : src;
    T v[E];
    Vec16<T>::put(*reinterpret_cast<const typename Vec16<T>::type*>(a), v);
#pragma unroll
    for (int e = 0; e < E; ++e) dst[c + e] = in ? v[e] : T(0);
  }
}

// tile_load_row_lower as straight-line code: every lane issues every load,
// and a vector wholly above the diagonal is read from `zeros` (16 zero bytes
// in device memory, a line every such lane shares, so no block bytes are
// fetched for it).  With no branch around the loads the compiler can wait
// for loads issued before the tile without waiting for the tile.
template <int CT, class T>
__device__ __forceinline__ void tile_load_row_lower_z(const T* __restrict__ row, int i,
                                                      const T* __restrict__ zeros,
                                                      T (&dst)[CT]) {
  constexpr int E = Vec16<T>::n;
  const int j0 = E * (threadIdx.x % 16);
  const T* src = row + j0;
#pragma unroll
  for (int c = 0; c < CT; c += E) {
    const T* a = j0 + 16 * c <= i ? src + 16 * c : zeros;
    Vec16<T>::put(*reinterpret_cast<const typename Vec16<T>::type*>(a), dst + c);
  }
}

template <class T>
__device__ __forceinline__ T tile_sum16(T v) {
  return row_sum16(v);
}

template <int RT, int CT, class T = double>
struct TiledSolve {
  static constexpr int P = 32 * RT;
  static_assert(P == 16 * CT, "tile shape");
  static constexpr int kThreads = kTiledThreads;

  struct Regs {
    T nt[RT][CT];
    T gt[RT][CT];
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
    const T* __restrict__ Nk = Mats<T>::N(L) + kk * L.sN;
#pragma unroll
    for (int r = 0; r < RT; ++r) tile_load_row<CT, T>(Nk + (long long)(r0 + r) * P, R.nt[r]);
  }

  __device__ __forceinline__ static void load_g(const LevelView& L, long long kk, Regs& R) {
    const int r0 = RT * (threadIdx.x / 16);
    const T* __restrict__ Gk = Mats<T>::Gi(L) + kk * (long long)P * P;
#pragma unroll
    for (int r = 0; r < RT; ++r)
      tile_load_row_lower<CT, T>(Gk + (long long)(r0 + r) * P, r0 + r, R.gt[r]);
  }

  // The one-step kernels' tiles: W_k = G_k^{-1} N_k (gn, levels whose L.GiN
  // is set) or N_k, and G_k^{-1} with its zeros from L.zeros.
  __device__ __forceinline__ static void load_straight(const LevelView& L, long long kk, bool gn,
                                                       Regs& R) {
    const int r0 = RT * (threadIdx.x / 16);
    const T* __restrict__ Nk =
        gn ? Mats<T>::GiN(L) + kk * (long long)P * P : Mats<T>::N(L) + kk * L.sN;
#pragma unroll
    for (int r = 0; r < RT; ++r) tile_load_row<CT, T>(Nk + (long long)(r0 + r) * P, R.nt[r]);
    const T* __restrict__ Gk = Mats<T>::Gi(L) + kk * (long long)P * P;
    const T* __restrict__ z = reinterpret_cast<const T*>(L.zeros);
#pragma unroll
    for (int r = 0; r < RT; ++r)
      tile_load_row_lower_z<CT, T>(Gk + (long long)(r0 + r) * P, r0 + r, z, R.gt[r]);
  }

  // Column partials of one thread -> per-wave slot of red (lanes 0..15).
  __device__ __forceinline__ static void col_partial(T (&v)[CT], T* red) {
    const int tid = threadIdx.x, lane = tid % kWave, w = tid / kWave;
#pragma unroll
    for (int c = 0; c < CT; ++c) {
      v[c] = xor32_sum(xor16_sum(v[c]));
    }
    if (lane < 16) {
#pragma unroll
      for (int c = 0; c < CT; ++c) red[w * P + tile_col<T>(c)] = v[c];
    }
  }

  // Column partials of two arrays at once, va -> per-wave slots of redA and
  // vb -> redB: each swap of pair16_sum / pair32_sum serves a value of both,
  // so lane (row rho) of the wave ends with the total of array rho & 1 for
  // column c + (rho >> 1) CT/2, and every lane stores CT/2 values.  Same sums
  // in the same order as two col_partial calls.
  __device__ __forceinline__ static void col_partial_pair(T (&va)[CT], T (&vb)[CT], T* redA,
                                                          T* redB) {
    static_assert(CT % 2 == 0, "columns in pairs");
    const int tid = threadIdx.x, lane = tid % kWave, w = tid / kWave, rho = lane / 16;
    T a[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) a[c] = pair16_sum(va[c], vb[c]);
    T* red = (rho & 1) ? redB : redA;
    const int off = (rho >> 1) * (CT / 2);
#pragma unroll
    for (int c = 0; c < CT / 2; ++c) {
      const T v = pair32_sum(a[c], a[c + CT / 2]);
      red[w * P + tile_col<T>(c + off)] = v;
    }
  }

  __device__ __forceinline__ static T col_total(const T* red, int j) {
    T s = 0;
#pragma unroll
    for (int w = 0; w < kTiledWaves; ++w) s += red[w * P + j];
    return s;
  }

  // Solve with the right-hand side in LDS (r_v, r_u, r_z, r_l, r_m; r_v and
  // r_m unused when !hv).  Results: lambda in ol; N^T lambda, Z^T lambda and
  // V^T lambda are left in the reduction slabs and combined by finish().
  __device__ __forceinline__ static void solve(const LevelView& L, long long kk, bool hv,
                                               const Regs& R, const T* sru,
                                               const T* srz, const T* srm,
                                               const T* srl, T* ol, T* scr) {
    const int tid = threadIdx.x, a = tid / 16, bq = tid % 16;
    const int r0 = RT * a;
    T* st = scr;
    T* ss = scr + P;
    T* red = scr + 2 * P;
    const T* __restrict__ Vk = Mats<T>::V(L) + kk * L.sV;
    const T* __restrict__ Zk = Mats<T>::Z(L) + kk * L.sZ;
    const bool dg = L.vz_diag != 0;                      // diagonal shared V, Z~
    const T* __restrict__ Vd = Mats<T>::Vd(L);
    const T* __restrict__ Zd = Mats<T>::Zd(L);
    // t = N r_u + Z r_z - V r_m - r_l
    T acc[RT];
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      T s = 0;
#pragma unroll
      for (int c = 0; c < CT; ++c) s += R.nt[r][c] * sru[tile_col<T>(c)];
      if (!dg) {
        T zr[CT];
        tile_load_row<CT, T>(Zk + (long long)(r0 + r) * P, zr);
#pragma unroll
        for (int c = 0; c < CT; ++c) s += zr[c] * srz[tile_col<T>(c)];
        if (hv) {
          T vr[CT];
          tile_load_row<CT, T>(Vk + (long long)(r0 + r) * P, vr);
#pragma unroll
          for (int c = 0; c < CT; ++c) s -= vr[c] * srm[tile_col<T>(c)];
        }
      }
      acc[r] = tile_sum16(s);
    }
    if (bq == 0) {
#pragma unroll
      for (int r = 0; r < RT; ++r) {
        const int i = r0 + r;
        T d = 0;
        if (dg) d = Zd[i] * srz[i] - (hv ? Vd[i] * srm[i] : T(0));
        st[i] = acc[r] + d - srl[i];
      }
    }
    __syncthreads();
    // s = G^{-1} t
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      T s = 0;
#pragma unroll
      for (int c = 0; c < CT; ++c) s += R.gt[r][c] * st[tile_col<T>(c)];
      acc[r] = tile_sum16(s);
    }
    if (bq == 0) {
#pragma unroll
      for (int r = 0; r < RT; ++r) ss[r0 + r] = acc[r];
    }
    __syncthreads();
    // lambda = G^{-T} s
    T cacc[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) {
      T s = 0;
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
      T s = 0;
#pragma unroll
      for (int r = 0; r < RT; ++r) s += R.nt[r][c] * ol[r0 + r];
      cacc[c] = s;
    }
    col_partial(cacc, red);
    if (!dg) {
      T zacc[CT];
#pragma unroll
      for (int c = 0; c < CT; ++c) zacc[c] = 0;
#pragma unroll
      for (int r = 0; r < RT; ++r) {
        T zr[CT];
        tile_load_row<CT, T>(Zk + (long long)(r0 + r) * P, zr);
#pragma unroll
        for (int c = 0; c < CT; ++c) zacc[c] += zr[c] * ol[r0 + r];
      }
      col_partial(zacc, red + kTiledWaves * P);
    }
    if (hv && !dg) {
      T vacc[CT];
#pragma unroll
      for (int c = 0; c < CT; ++c) vacc[c] = 0;
#pragma unroll
      for (int r = 0; r < RT; ++r) {
        T vr[CT];
        tile_load_row<CT, T>(Vk + (long long)(r0 + r) * P, vr);
#pragma unroll
        for (int c = 0; c < CT; ++c) vacc[c] += vr[c] * ol[r0 + r];
      }
      col_partial(vacc, red + 2 * kTiledWaves * P);
    }
    __syncthreads();
  }

  // Entries i of the diagonals of Z~ and V when they are diagonal (else 0),
  // read once by the thread that owns entry i of the block's vectors.
  struct Diag {
    T zd = 0, vd = 0;
  };
  __device__ __forceinline__ static Diag diag_at(const LevelView& L, int i) {
    Diag g;
    if (L.vz_diag) {
      g.zd = Mats<T>::Zd(L)[i];
      g.vd = Mats<T>::Vd(L)[i];
    }
    return g;
  }

  // Entry i of d = Z~ r_z - V r_mu - r_l when V and Z~ are diagonal (r_mu = 0
  // in the first block, which has no mu row).
  __device__ __forceinline__ static T d_of(const Diag& g, const T* srz, const T* srm,
                                           const T* srl, int i) {
    return g.zd * srz[i] - g.vd * srm[i] - srl[i];
  }

  // The same solve with W = G^{-1} N in the N tile (R from load_gn) and V,
  // Z~ diagonal, d = Z~ r_z - V r_mu - r_l in srd.  With t = N r_u + d,
  //     s = G^{-1} t = W r_u + G^{-1} d,   lambda = G^{-T} s,
  //     N^T lambda = N^T G^{-T} s = W^T s,
  // so one pass of row products and one of column products (two barriers)
  // replace the four dependent phases of solve().  Results as for solve():
  // lambda in ol, N^T lambda in slab 0; ol[j] is written by thread j only
  // (no barrier after it: each thread reads back its own entries).
  __device__ __forceinline__ static void solve_gn(const Regs& R, const T* sru, const T* srd,
                                                  T* ol, T* scr) {
    const int tid = threadIdx.x, a = tid / 16, bq = tid % 16;
    const int r0 = RT * a;
    T* ss = scr + P;
    T* red = scr + 2 * P;
    // s = W r_u + G^{-1} d
    T acc[RT];
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      T s = 0;
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        const int j = tile_col<T>(c);
        s += R.nt[r][c] * sru[j] + R.gt[r][c] * srd[j];
      }
      acc[r] = tile_sum16(s);
    }
    if (bq == 0) {
#pragma unroll
      for (int r = 0; r < RT; ++r) ss[r0 + r] = acc[r];
    }
    __syncthreads();
    // W^T s -> slab 0, lambda = G^{-T} s -> slab 1
    T wacc[CT], lacc[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) {
      T sw = 0, sl = 0;
#pragma unroll
      for (int r = 0; r < RT; ++r) {
        const T sv = ss[r0 + r];
        sw += R.nt[r][c] * sv;
        sl += R.gt[r][c] * sv;
      }
      wacc[c] = sw;
      lacc[c] = sl;
    }
    col_partial_pair(wacc, lacc, red, red + kTiledWaves * P);
    __syncthreads();
    for (int j = tid; j < P; j += kThreads) ol[j] = col_total(red + kTiledWaves * P, j);
  }

  // Component i of the solution after solve():
  //   u = r_u - N^T lambda, z = r_z - Z^T lambda, mu = V^T lambda - r_m - r_v,
  //   v = -r_m   (lambda is ol[i]; with diagonal V, Z~ their products with
  //   lambda are elementwise, g from diag_at).
  __device__ __forceinline__ static T u_of(const T* scr, const T* sru, int i) {
    return sru[i] - col_total(scr + 2 * P, i);
  }
  __device__ __forceinline__ static T z_of(const LevelView& L, const Diag& g, const T* scr,
                                           const T* srz, const T* ol, int i) {
    if (L.vz_diag) return srz[i] - g.zd * ol[i];
    return srz[i] - col_total(scr + 2 * P + kTiledWaves * P, i);
  }
  __device__ __forceinline__ static T mu_of(const LevelView& L, const Diag& g, const T* scr,
                                            const T* srm, const T* srv, const T* ol, int i) {
    if (L.vz_diag) return g.vd * ol[i] - srm[i] - srv[i];
    return col_total(scr + 2 * P + 2 * kTiledWaves * P, i) - srm[i] - srv[i];
  }
};

}  // namespace pitmg
