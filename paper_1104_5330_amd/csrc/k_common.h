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
// p advanced by b bytes (a 32-bit lane offset added to a wave-uniform pointer)
template <typename T>
SP6_DEV T* byte_off(T* p, uint32_t b) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(p) + b);
}
template <typename T>
SP6_DEV const T* byte_off(const T* p, uint32_t b) {
  return reinterpret_cast<const T*>(reinterpret_cast<const char*>(p) + b);
}
// x, opaque to the optimiser (no instruction): keeps a lane offset from being
// folded into a 64-bit lane address hoisted out of a loop, so that a uniform row
// pointer plus this 32-bit offset is formed at the access
SP6_DEV uint32_t lane_opaque(uint32_t x) {
  asm volatile("" : "+v"(x));
  return x;
}

// Streaming access: data read or written once per pass.  SP6_NT selects which
// global accesses carry the nontemporal hint (bits below).  Measured on the
// 33 x 16 x 32 x 16 x 32 grid: on the loads and stores of the plane pass it takes
// the pass from 4.66 to 5.03 TB/s; on the radial pass's T loads and stores from
// 4.84 to 5.0 TB/s, and on its stage-input loads from 331 to 318 us (the next
// plane pass, which reads that input again, loses 6 us of it; with the plane
// lines streamed from LDS it had lost all of it); on the theta-phi pass
// (partial-line stores) it costs 12 %, so that pass has none; the adjoint plane
// pass streams all its operands with it.
#ifndef SP6_NT
#define SP6_NT 1999
#endif
template <int BIT, typename T>
SP6_DEV T ld_stream(const T* p) {
  if constexpr ((SP6_NT & BIT) != 0)
    return __builtin_nontemporal_load(p);
  else
    return *p;
}
template <int BIT, typename T>
SP6_DEV void st_stream(T* p, T v) {
  if constexpr ((SP6_NT & BIT) != 0)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}
// plane pass: 1 stage input and T loads, 2 next-stage state (or output) stores,
// 64 accumulator and y loads, 128 accumulator stores; radial pass: 4 stage input
// loads, 256 T loads, 8 T stores; adjoint plane pass: 512 loads, 1024 stores
enum {
  NT_PLANE_LD = 1, NT_PLANE_ST = 2, NT_RAD_LD = 4, NT_RAD_ST = 8, NT_SPH_LD = 16, NT_SPH_ST = 32,
  NT_PLANE_LDA = 64, NT_PLANE_STA = 128, NT_RAD_LDT = 256, NT_ADJ_LD = 512, NT_ADJ_ST = 1024
};

// Line-operator tables in constant memory.  The Fourier derivative and the
// filter on an L-point periodic line depend on L only, so one copy per L serves
// every handle.  Kind 0: derivative, kind 1: filter; each in even/odd form
// (A then B, h x h, h = L/2), line lengths 4, 8, 16, 32, 64 back to back.
// Uniform indices let the compiler read them with scalar loads.
constexpr int line_tab_offset(int L) {
  return L == 4 ? 0 : L == 8 ? 8 : L == 16 ? 40 : L == 32 ? 168 : L == 64 ? 680 : -1;
}
constexpr int LINE_TAB_SIZE = 2728;  // sum of 2 (L/2)^2 over L = 4 .. 64
constexpr int LINE_TAB_KINDS = 4;
// 0: derivative, 1: filter, 2 and 3: the same transposed (entries of consecutive
// output pairs at one input index j contiguous)
enum { LT_DERIV = 0, LT_FILTER = 1, LT_DERIV_T = 2, LT_FILTER_T = 3 };

// Output pairs i0 .. i0 + NPAIR - 1 of a centro-(anti)symmetric L x L matrix
// applied to a line that is read element by element (from LDS): ldA(j) returns
// element j and ldB(j) element L - 1 - j of the line, j < L / 2.  The line is
// streamed once (e_j, o_j formed on the fly) and only the 2 NPAIR accumulators
// stay live.  tabT is the transposed even/odd table.
template <int L, int NPAIR, bool ANTI, typename T, int U = 4, typename TT, typename LoadA, typename LoadB,
          typename Emit>
SP6_DEV void eo_pairs_stream2(const TT* __restrict__ tabT, int i0, LoadA&& ldA, LoadB&& ldB, Emit&& emit) {
  constexpr int h = L / 2;
  T p[NPAIR], q[NPAIR];
#pragma unroll
  for (int ii = 0; ii < NPAIR; ++ii) p[ii] = q[ii] = T(0);
  // partial unrolling (U) bounds the number of line elements and table entries
  // the compiler hoists into registers
#pragma unroll U
  for (int j = 0; j < h; ++j) {
    const T a = ldA(j), b = ldB(j);
    const T e = a + b, o = a - b;
    const TT* __restrict__ At = tabT + j * h + i0;
    const TT* __restrict__ Bt = tabT + h * h + j * h + i0;
#pragma unroll
    for (int ii = 0; ii < NPAIR; ++ii) {
      p[ii] = fma(T(At[ii]), e, p[ii]);
      q[ii] = fma(T(Bt[ii]), o, q[ii]);
    }
  }
#pragma unroll
  for (int ii = 0; ii < NPAIR; ++ii) {
    emit(i0 + ii, p[ii] + q[ii]);
    emit(L - 1 - (i0 + ii), ANTI ? (q[ii] - p[ii]) : (p[ii] - q[ii]));
  }
}

// the same with one loader ld(q) for every element q of the line
template <int L, int NPAIR, bool ANTI, typename T, int U = 4, typename TT, typename Load, typename Emit>
SP6_DEV void eo_pairs_stream(const TT* __restrict__ tabT, int i0, Load&& ld, Emit&& emit) {
  eo_pairs_stream2<L, NPAIR, ANTI, T, U>(
      tabT, i0, [&](int j) { return ld(j); }, [&](int j) { return ld(L - 1 - j); }, emit);
}

// inflow node test (Sect. 4.2): r_in with cos(Theta) > 0, r_out with cos(Theta) < 0
SP6_DEV bool is_inflow(const KDims& d, const KTab& t, int j, int iTh) {
  if (!d.bc) return false;
  double c = t.cos_Th[iTh];
  return (j == 0 && c > 0.0) || (j == d.n_r - 1 && c < 0.0);
}
