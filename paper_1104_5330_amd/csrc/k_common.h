// Device helpers shared by the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "sp6_internal.h"

#define SP6_DEV __device__ __forceinline__

// Apply a centro-(anti)symmetric L x L matrix to a line held in registers, in
// even/odd form (tables built by even_odd() on the host: A then B, h x h each).
// On entry v holds the line; on exit v[j] = e_j = v_j + v_{L-1-j} and
// v[L-1-j] = o_j = v_j - v_{L-1-j} (j < h).  Output pairs i0 .. i0 + NPAIR - 1 are
// produced: emit(i, (Dv)_i) and emit(L-1-i, (Dv)_{L-1-i}).  i0 must be uniform
// across the wavefront so that the table reads become scalar loads.
template <int L, typename T>
SP6_DEV void eo_split(T (&v)[L]) {
  constexpr int h = L / 2;
#pragma unroll
  for (int j = 0; j < h; ++j) {
    T a = v[j], b = v[L - 1 - j];
    v[j] = a + b;
    v[L - 1 - j] = a - b;
  }
}

template <int L, int NPAIR, bool ANTI, typename T, typename TT, typename Emit>
SP6_DEV void eo_pairs(const TT* __restrict__ tab, int i0, const T (&v)[L], Emit&& emit) {
  constexpr int h = L / 2;
#pragma unroll
  for (int ii = 0; ii < NPAIR; ++ii) {
    const int i = i0 + ii;
    const TT* __restrict__ A = tab + i * h;
    const TT* __restrict__ B = tab + h * h + i * h;
    T p = T(0), q = T(0);
#pragma unroll
    for (int j = 0; j < h; ++j) {
      p = fma(T(A[j]), v[j], p);
      q = fma(T(B[j]), v[L - 1 - j], q);
    }
    emit(i, p + q);
    emit(L - 1 - i, ANTI ? (q - p) : (p - q));
  }
}

SP6_DEV int wave_uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

// inflow node test (Sect. 4.2): r_in with cos(Theta) > 0, r_out with cos(Theta) < 0
SP6_DEV bool is_inflow(const KDims& d, const KTab& t, int j, int iTh) {
  if (!d.bc) return false;
  double c = t.cos_Th[iTh];
  return (j == 0 && c > 0.0) || (j == d.n_r - 1 && c < 0.0);
}
