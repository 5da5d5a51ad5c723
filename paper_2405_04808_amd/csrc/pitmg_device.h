// Small device helpers shared by the kernel translation units.
#pragma once
#include "pitmg_internal.h"

namespace pitmg {

// Cross-lane sums that stay in the vector ALU (no trip through the LDS
// crossbar): DPP row rotations inside each row of 16 lanes, and the gfx950
// permlane swaps between rows (lane ^ 16) and between the two halves of the
// wave (lane ^ 32).  Every lane ends with the sum.  All lanes of the wave
// must be active.
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// sum over the 16 lanes of each row (DPP row_ror 8, 4, 2, 1)
template <class T>
__device__ __forceinline__ T row_sum16(T v) {
  v += dpp_move<0x128>(v);
  v += dpp_move<0x124>(v);
  v += dpp_move<0x122>(v);
  v += dpp_move<0x121>(v);
  return v;
}

// v + v[lane ^ 16]: the swap leaves rows (0,0,2,2) in one register and
// rows (1,1,3,3) in the other
__device__ __forceinline__ float xor16_sum(float v) {
  const unsigned b = __float_as_uint(v);
  const auto r = __builtin_amdgcn_permlane16_swap(b, b, false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ double xor16_sum(double v) {
  const unsigned lo = (unsigned)__double2loint(v), hi = (unsigned)__double2hiint(v);
  const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  return __hiloint2double((int)h[0], (int)l[0]) + __hiloint2double((int)h[1], (int)l[1]);
}

// v + v[lane ^ 32] (halves of the wave)
__device__ __forceinline__ float xor32_sum(float v) {
  const unsigned b = __float_as_uint(v);
  const auto r = __builtin_amdgcn_permlane32_swap(b, b, false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ double xor32_sum(double v) {
  const unsigned lo = (unsigned)__double2loint(v), hi = (unsigned)__double2hiint(v);
  const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  return __hiloint2double((int)h[0], (int)l[0]) + __hiloint2double((int)h[1], (int)l[1]);
}

// Two sums for one swap: x + x[lane ^ 16] in the even rows (0, 2) and
// y + y[lane ^ 16] in the odd rows (1, 3).  The swap exchanges the odd rows
// of its first operand with the even rows of its second, so each register
// it returns holds one value of each pair.
__device__ __forceinline__ float pair16_sum(float x, float y) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false,
                                                  false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ double pair16_sum(double x, double y) {
  const auto l = __builtin_amdgcn_permlane16_swap((unsigned)__double2loint(x),
                                                  (unsigned)__double2loint(y), false, false);
  const auto h = __builtin_amdgcn_permlane16_swap((unsigned)__double2hiint(x),
                                                  (unsigned)__double2hiint(y), false, false);
  return __hiloint2double((int)h[0], (int)l[0]) + __hiloint2double((int)h[1], (int)l[1]);
}

// x + x[lane ^ 32] in lanes 0..31 and y + y[lane ^ 32] in lanes 32..63
// (the swap exchanges the upper half of its first operand with the lower
// half of its second).
__device__ __forceinline__ float pair32_sum(float x, float y) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false,
                                                  false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ double pair32_sum(double x, double y) {
  const auto l = __builtin_amdgcn_permlane32_swap((unsigned)__double2loint(x),
                                                  (unsigned)__double2loint(y), false, false);
  const auto h = __builtin_amdgcn_permlane32_swap((unsigned)__double2hiint(x),
                                                  (unsigned)__double2hiint(y), false, false);
  return __hiloint2double((int)h[0], (int)l[0]) + __hiloint2double((int)h[1], (int)l[1]);
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
  return xor32_sum(xor16_sum(row_sum16(v)));
}

// Value of the interpolated coarse vector (one node-type segment of nc coarse
// steps, width p) at fine step k (1-based), component i.  Variant 0 follows
// the printed transfer: fine step 2m-1 takes coarse step m, fine step 2m the
// mean of coarse steps m and m+1, with the missing step nc+1 replaced by nc.
// Variant 1 aligns coarse step m with fine step 2m and averages m-1, m into
// fine step 2m-1 (coarse step 0 is zero).
__device__ __forceinline__ double interp_node(const double* __restrict__ seg, int nc, int p,
                                              int k, int i, int variant) {
  if (variant == 0) {
    if (k & 1) return seg[(long long)((k + 1) / 2 - 1) * p + i];
    const int m = k / 2, m2 = m < nc ? m + 1 : nc;
    return 0.5 * (seg[(long long)(m - 1) * p + i] + seg[(long long)(m2 - 1) * p + i]);
  }
  if (!(k & 1)) return seg[(long long)(k / 2 - 1) * p + i];
  const int m = (k + 1) / 2;
  const double a = seg[(long long)(m - 1) * p + i];
  const double b = m >= 2 ? seg[(long long)(m - 2) * p + i] : 0.0;
  return 0.5 * (a + b);
}

// Stores and loads of values that another work-group of the same launch
// reads or wrote: agent-scope atomics, which gfx950 performs at the device's
// coherence point (the sc1 bit), past the non-coherent L2 of each XCD.
__device__ __forceinline__ void coherent_store(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double coherent_load(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The loads behind one entry of PrevIterate::at, issued together by
// PrevIterate::fetch and combined by PrevIterate::value (same arithmetic as
// at()), so that a kernel can request several entries before it needs any.
struct PrevFetch {
  double y = 0.0, a = 0.0, b = 0.0;
};

// The iterate a sweep starts from: yold (NULL = 0) plus, in the first
// post-smoothing sweep, the interpolated coarse correction P ec (NULL = 0),
// whose mu block carries mu_scale and whose control is constant over the
// two fine steps of a coarse step.  type: 0 u, 1 v, 2 z, 3 lambda, 4 mu.
struct PrevIterate {
  const double* yold;
  const double* ec;
  int p, q, n, variant;
  double mu_scale;
  // ec (yold) is written by other work-groups of the same launch: read it
  // with coherent loads
  bool ec_coherent = false;
  bool yold_coherent = false;
  __device__ __forceinline__ double ec_at(long long idx) const {
    return ec_coherent ? coherent_load(ec + idx) : ec[idx];
  }
  __device__ __forceinline__ double yold_at(long long idx) const {
    return yold_coherent ? coherent_load(yold + idx) : yold[idx];
  }
  __device__ double at(int type, int k, int i) const {
    const TypeMajor Tm(p, q, n);
    const long long seg[5] = {Tm.u, Tm.v, Tm.z, Tm.l, Tm.m};
    const int w = type == 2 ? q : p;
    double v = yold ? yold_at(seg[type] + (long long)(k - 1) * w + i) : 0.0;
    if (ec) {
      const int nc = n / 2;
      const TypeMajor Tc(p, q, nc > 0 ? nc : 1);
      if (type == 2) {
        v += ec_at(Tc.z + (long long)((k + 1) / 2 - 1) * q + i);
      } else {
        const long long sc[5] = {Tc.u, Tc.v, Tc.z, Tc.l, Tc.m};
        double e;
        if (ec_coherent) {
          int ma, mb, two;
          node_terms(nc, k, variant, &ma, &mb, &two);
          const double a = ec_at(sc[type] + (long long)(ma - 1) * p + i);
          const double b2 = ec_at(sc[type] + (long long)(mb - 1) * p + i);
          e = two == 0 ? a : 0.5 * (a + (two == 1 ? b2 : 0.0));
        } else {
          e = interp_node(ec + sc[type], nc, p, k, i, variant);
        }
        v += type == 4 ? mu_scale * e : e;
      }
    }
    return v;
  }

  // Coarse steps (1-based) of the one or two terms interp_node averages for
  // fine step k; *two = 0 when there is one term (then mb = ma).
  __device__ __forceinline__ static void node_terms(int nc, int k, int variant, int* ma,
                                                    int* mb, int* two) {
    if (variant == 0) {
      if (k & 1) {
        *ma = *mb = (k + 1) / 2;
        *two = 0;
      } else {
        const int m = k / 2;
        *ma = m;
        *mb = m < nc ? m + 1 : nc;
        *two = 1;
      }
    } else if (!(k & 1)) {
      *ma = *mb = k / 2;
      *two = 0;
    } else {
      const int m = (k + 1) / 2;
      *ma = m;
      *mb = m >= 2 ? m - 1 : m;                 // coarse step 0 is zero
      *two = m >= 2 ? 1 : 2;                    // 2: the second term is 0
    }
  }

  __device__ __forceinline__ PrevFetch fetch(int type, int k, int i) const {
    PrevFetch f;
    const TypeMajor Tm(p, q, n);
    const long long seg[5] = {Tm.u, Tm.v, Tm.z, Tm.l, Tm.m};
    const int w = type == 2 ? q : p;
    if (yold) f.y = yold_at(seg[type] + (long long)(k - 1) * w + i);
    if (ec) {
      const int nc = n / 2;
      const TypeMajor Tc(p, q, nc > 0 ? nc : 1);
      if (type == 2) {
        f.a = ec_at(Tc.z + (long long)((k + 1) / 2 - 1) * q + i);
      } else {
        const long long sc[5] = {Tc.u, Tc.v, Tc.z, Tc.l, Tc.m};
        int ma, mb, two;
        node_terms(nc, k, variant, &ma, &mb, &two);
        f.a = ec_at(sc[type] + (long long)(ma - 1) * p + i);
        f.b = ec_at(sc[type] + (long long)(mb - 1) * p + i);
      }
    }
    return f;
  }

  __device__ __forceinline__ double value(const PrevFetch& f, int type, int k) const {
    double v = yold ? f.y : 0.0;
    if (ec) {
      if (type == 2) {
        v += f.a;
      } else {
        int ma, mb, two;
        node_terms(n / 2, k, variant, &ma, &mb, &two);
        const double e = two == 0 ? f.a : 0.5 * (f.a + (two == 1 ? f.b : 0.0));
        v += type == 4 ? mu_scale * e : e;
      }
    }
    return v;
  }
};

// Weighted sweep output (1 - omega) y_prev + omega y_hat; omega = 1 reads
// nothing.
__device__ __forceinline__ double weigh(double omega, double yhat, const PrevIterate& prev,
                                        int type, int k, int i) {
  if (omega == 1.0) return yhat;
  return omega * yhat + (1.0 - omega) * prev.at(type, k, i);
}

}  // namespace pitmg
