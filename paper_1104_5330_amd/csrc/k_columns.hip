// Column passes: the theta, phi and r terms of the Liouville operator.
//
// Data layout [eps][r][theta][phi][Theta][Phi]: every (Theta, Phi) plane is a
// contiguous run, and lines along r, theta and phi cross planes at a fixed
// in-plane index ("column").  Each thread owns one column of one line and holds
// the whole line in registers, so consecutive threads read consecutive
// addresses of every plane they touch (fully coalesced).
//
//   phi   : Fourier line of n_phi points; term (sin Theta sin Phi / (r sin theta)) d/dphi
//   theta : double-Fourier-sphere line of 2 n_theta points built from the column
//           (phi_k, Phi_m) and, reversed, its partner (phi_k + pi, Phi_m + pi),
//           since (-theta, phi, Theta, Phi) is the point (theta, phi + pi, Theta,
//           Phi + pi); term (sin Theta cos Phi / r) d/dtheta
//   r     : Chebyshev-Gauss-Lobatto line of n_r points on FP64 MFMA
//           (v_mfma_f64_16x16x4f64), term cos(Theta) d/dr
// (Eq. Liouvsph).  Both angular coefficients are constant along their lines, and
// the angular matrices are antisymmetric, so the transposed theta and phi passes
// are the forward passes with the coefficient negated; the transposed radial pass
// uses D_r^T.
#include "k_common.h"

namespace {

constexpr int CB = 256;  // threads per block of the column kernels

// ---------------------------------------------------------------------------
// phi lines

template <int L>
__global__ __launch_bounds__(CB) void k_phi(KDims d, KTab t, const double* __restrict__ Y,
                                            double* __restrict__ T, int accum, double coef_sign,
                                            int mask_in, double in_scale) {
  const int64_t gid = int64_t(blockIdx.x) * CB + threadIdx.x;
  const int64_t nouter = int64_t(d.n_eps) * d.n_r * d.n_th;
  if (gid >= nouter * d.plane) return;
  const int c = int(gid % d.plane);
  const int64_t o = gid / d.plane;
  const int l = int(o % d.n_th);
  const int j = int((o / d.n_th) % d.n_r);
  const int iTh = c / d.n_Ph, m = c % d.n_Ph;
  const int64_t stride = d.plane;
  const int64_t base = o * (int64_t(L) * stride) + c;

  double s_in = in_scale;
  if (mask_in && is_inflow(d, t, j, iTh)) s_in = 0.0;
  double v[L];
#pragma unroll
  for (int k = 0; k < L; ++k) v[k] = Y[base + k * stride] * s_in;
  double tv[L];
  if (accum) {
#pragma unroll
    for (int k = 0; k < L; ++k) tv[k] = T[base + k * stride];
  }
  const double s = coef_sign * t.sin_Th[iTh] * t.sin_Ph[m] * t.inv_r[j] * t.inv_sin_th[l];
  eo_split<L>(v);
  eo_pairs<L, L / 2, true>(t.eo_ph, 0, v, [&](int k, double z) {
    const double val = s * z;
    T[base + k * stride] = accum ? tv[k] + val : val;
  });
}

// ---------------------------------------------------------------------------
// theta DFS lines: thread = (eps, r, k < n_phi/2, column c); it owns the orbit
// {(k, c), (k + n_phi/2, c')} with c' the column at Phi_m + pi.

template <int NTH>
__global__ __launch_bounds__(CB) void k_theta(KDims d, KTab t, const double* __restrict__ Y,
                                              double* __restrict__ T, int accum, double coef_sign,
                                              int mask_in, double in_scale) {
  constexpr int L = 2 * NTH;
  const int hph = d.n_ph / 2;
  const int64_t gid = int64_t(blockIdx.x) * CB + threadIdx.x;
  const int64_t total = int64_t(d.n_eps) * d.n_r * hph * d.plane;
  if (gid >= total) return;
  const int c = int(gid % d.plane);
  const int64_t rest = gid / d.plane;
  const int k = int(rest % hph);
  const int64_t ej = rest / hph;
  const int j = int(ej % d.n_r);
  const int kp = k + hph;
  const int iTh = c / d.n_Ph, m = c % d.n_Ph;
  const int mp = (m + d.n_Ph / 2) % d.n_Ph;
  const int cp = iTh * d.n_Ph + mp;
  const int64_t rowstride = int64_t(d.n_ph) * d.plane;
  const int64_t base = ej * (int64_t(NTH) * rowstride);
  const int64_t ba = base + int64_t(k) * d.plane + c;
  const int64_t bb = base + int64_t(kp) * d.plane + cp;

  double s_in = in_scale;
  if (mask_in && is_inflow(d, t, j, iTh)) s_in = 0.0;
  double v[L];
#pragma unroll
  for (int l = 0; l < NTH; ++l) {
    v[l] = Y[ba + l * rowstride] * s_in;
    v[L - 1 - l] = Y[bb + l * rowstride] * s_in;
  }
  double tv[L];
  if (accum) {
#pragma unroll
    for (int l = 0; l < NTH; ++l) {
      tv[l] = T[ba + l * rowstride];
      tv[L - 1 - l] = T[bb + l * rowstride];
    }
  }
  // partner coefficient is -s (cos(Phi + pi) = -cos Phi) and the partner
  // derivative is -z[L-1-l]; both signs cancel.
  const double s = coef_sign * t.sin_Th[iTh] * t.cos_Ph[m] * t.inv_r[j];
  eo_split<L>(v);
  eo_pairs<L, NTH, true>(t.eo_th, 0, v, [&](int q, double z) {
    const double val = s * z;
    const int64_t a = (q < NTH) ? ba + q * rowstride : bb + (L - 1 - q) * rowstride;
    T[a] = accum ? tv[q] + val : val;
  });
}

// ---------------------------------------------------------------------------
// radial lines on FP64 MFMA.  Per wavefront: 16 columns x all r as one
// (NRP x KP) * (KP x 16) product, NRP = 16 NRT rows, KP = 4 KS.
// Operand layouts of v_mfma_f64_16x16x4f64 (lane l):
//   A (16 x 4): A[l % 16][l / 16];  B (4 x 16): B[l / 16][l % 16];
//   C (16 x 16): register v holds C[l / 16 + 4 v][l % 16] (rows interleaved).

typedef double v4d __attribute__((ext_vector_type(4)));

template <int KS>
__global__ __launch_bounds__(CB) void k_radial(KDims d, KTab t, const double* __restrict__ Y,
                                               double* __restrict__ T, int accum, int transpose,
                                               int mask_in, double in_scale) {
  constexpr int NRT = (KS + 3) / 4;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const double* __restrict__ Dp = transpose ? t.DpadT : t.Dpad;
  double a[NRT][KS];
#pragma unroll
  for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
    for (int s = 0; s < KS; ++s) a[rt][s] = Dp[(16 * rt + lr) * t.KP + 4 * s + lk];

  const int64_t gpe = d.M / 16;  // column groups per energy group
  const int64_t ngroups = gpe * d.n_eps;
  const int nw = CB / 64;
  for (int64_t g = int64_t(blockIdx.x) * nw + wave; g < ngroups; g += int64_t(gridDim.x) * nw) {
    const int64_t e = g / gpe;
    const int64_t col = (g % gpe) * 16 + lr;
    const int64_t ebase = e * d.n_r * d.M + col;
    const int iTh = int((col / d.n_Ph) % d.n_Th);
    double b[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int row = 4 * s + lk;
      double val = 0.0;
      if (row < d.n_r) {
        val = Y[ebase + row * d.M] * in_scale;
        if (mask_in && is_inflow(d, t, row, iTh)) val = 0.0;
      }
      b[s] = val;
    }
    v4d acc[NRT];
#pragma unroll
    for (int rt = 0; rt < NRT; ++rt) {
      acc[rt] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < KS; ++s) acc[rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rt][s], b[s], acc[rt], 0, 0, 0);
    }
    const double cT = t.cos_Th[iTh];
#pragma unroll
    for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * rt + lk + 4 * v;
        if (row < d.n_r) {
          const int64_t ad = ebase + row * d.M;
          const double val = cT * acc[rt][v];
          T[ad] = accum ? T[ad] + val : val;
        }
      }
  }
}

// ---------------------------------------------------------------------------
// filter of theta and phi lines (in place; centro-symmetric matrices)

template <int L>
__global__ __launch_bounds__(CB) void k_filter_phi(KDims d, KTab t, double* __restrict__ F) {
  const int64_t gid = int64_t(blockIdx.x) * CB + threadIdx.x;
  const int64_t nouter = int64_t(d.n_eps) * d.n_r * d.n_th;
  if (gid >= nouter * d.plane) return;
  const int c = int(gid % d.plane);
  const int64_t o = gid / d.plane;
  const int64_t stride = d.plane;
  const int64_t base = o * (int64_t(L) * stride) + c;
  double v[L];
#pragma unroll
  for (int k = 0; k < L; ++k) v[k] = F[base + k * stride];
  eo_split<L>(v);
  eo_pairs<L, L / 2, false>(t.fl_ph, 0, v, [&](int k, double z) { F[base + k * stride] = z; });
}

template <int NTH>
__global__ __launch_bounds__(CB) void k_filter_theta(KDims d, KTab t, double* __restrict__ F) {
  constexpr int L = 2 * NTH;
  const int hph = d.n_ph / 2;
  const int64_t gid = int64_t(blockIdx.x) * CB + threadIdx.x;
  const int64_t total = int64_t(d.n_eps) * d.n_r * hph * d.plane;
  if (gid >= total) return;
  const int c = int(gid % d.plane);
  const int64_t rest = gid / d.plane;
  const int k = int(rest % hph);
  const int64_t ej = rest / hph;
  const int iTh = c / d.n_Ph, m = c % d.n_Ph;
  const int cp = iTh * d.n_Ph + (m + d.n_Ph / 2) % d.n_Ph;
  const int64_t rowstride = int64_t(d.n_ph) * d.plane;
  const int64_t base = ej * (int64_t(NTH) * rowstride);
  const int64_t ba = base + int64_t(k) * d.plane + c;
  const int64_t bb = base + int64_t(k + hph) * d.plane + cp;
  double v[L];
#pragma unroll
  for (int l = 0; l < NTH; ++l) {
    v[l] = F[ba + l * rowstride];
    v[L - 1 - l] = F[bb + l * rowstride];
  }
  eo_split<L>(v);
  eo_pairs<L, NTH, false>(t.fl_th, 0, v, [&](int q, double z) {
    const int64_t a = (q < NTH) ? ba + q * rowstride : bb + (L - 1 - q) * rowstride;
    F[a] = z;
  });
}

unsigned grid_for(int64_t threads) { return unsigned((threads + CB - 1) / CB); }

}  // namespace

hipError_t launch_phi(const KDims& d, const KTab& t, const double* Y, double* T, bool accum,
                      double coef_sign, bool mask_in, double in_scale, hipStream_t s) {
  const unsigned g = grid_for(int64_t(d.n_eps) * d.n_r * d.n_th * d.plane);
  switch (d.n_ph) {
#define CASE(N) \
  case N: k_phi<N><<<g, CB, 0, s>>>(d, t, Y, T, accum, coef_sign, mask_in, in_scale); break;
    CASE(4) CASE(8) CASE(16) CASE(32) CASE(64)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_theta(const KDims& d, const KTab& t, const double* Y, double* T, bool accum,
                        double coef_sign, bool mask_in, double in_scale, hipStream_t s) {
  const unsigned g = grid_for(int64_t(d.n_eps) * d.n_r * (d.n_ph / 2) * d.plane);
  switch (d.n_th) {
#define CASE(N) \
  case N: k_theta<N><<<g, CB, 0, s>>>(d, t, Y, T, accum, coef_sign, mask_in, in_scale); break;
    CASE(2) CASE(4) CASE(8) CASE(16) CASE(32)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_radial(const KDims& d, const KTab& t, const double* Y, double* T, bool accum,
                         bool transpose, bool mask_in, double in_scale, hipStream_t s) {
  const int64_t ngroups = (d.M / 16) * d.n_eps;
  int64_t blocks = (ngroups + 3) / 4;
  if (blocks > 4096) blocks = 4096;
  const unsigned g = unsigned(blocks);
  const int KS = t.KP / 4;
  switch (KS) {
#define CASE(N) \
  case N: k_radial<N><<<g, CB, 0, s>>>(d, t, Y, T, accum, transpose, mask_in, in_scale); break;
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10)
    CASE(11) CASE(12) CASE(13) CASE(14) CASE(15) CASE(16) CASE(17) CASE(18) CASE(19) CASE(20)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_filter_columns(const KDims& d, const KTab& t, double* F, hipStream_t s) {
  const unsigned gt = grid_for(int64_t(d.n_eps) * d.n_r * (d.n_ph / 2) * d.plane);
  switch (d.n_th) {
#define CASE(N) \
  case N: k_filter_theta<N><<<gt, CB, 0, s>>>(d, t, F); break;
    CASE(2) CASE(4) CASE(8) CASE(16) CASE(32)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const unsigned gp = grid_for(int64_t(d.n_eps) * d.n_r * d.n_th * d.plane);
  switch (d.n_ph) {
#define CASE(N) \
  case N: k_filter_phi<N><<<gp, CB, 0, s>>>(d, t, F); break;
    CASE(4) CASE(8) CASE(16) CASE(32) CASE(64)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
