// Fokker-Planck energy coupling (Sect. 3.2, Eq. Transpfp): with the coupling on,
// the energy groups are the Chebyshev-Gauss-Lobatto nodes gamma_k of
// [gamma_min, gamma_max] and each right-hand side gains, per (eps, r, theta, phi)
// plane, the isotropic source sigma S(gamma),
//
//   S = (1/4pi) d/dgamma [alpha gamma^2 dM0/dgamma + (gamma^2 - 2 alpha gamma) M0]
//       + 3/(128 pi^2) dQ/dgamma,
//   M0 = int F dw,  Q = int int (1 - mu + mu^2 - mu^3) F(w') F(w'') dw' dw''
//                     = M0^2 - M1.M1 + M2:M2 - M3:.M3  (moments Mk of rank k),
//
// sigma standing for n sigma_Th.  The sign is the one for which the energy
// diffusion is forward in time and the Bose distribution (Eq. Bose) is a steady
// state (the printed Eq. Kompa has the opposite overall sign, the printed
// induced term of Eq. Transpfp the opposite sign of that term).
//
// Two passes per right-hand side, ahead of the plane pass, which then takes
// eta + sigma S as its emissivity (the moment pass reads the FP64 state or the
// mixed path's FP32 stage copy; everything after it is FP64):
//   k_fp_moments: each plane reduced to (M0, Q): lane = column of the plane,
//     20 moments summed over its rows, then reduced over the plane's lanes
//     (8 bytes read per point, 16 written per plane);
//   k_fp_source: one workgroup per position (r, theta, phi), thread k for group
//     k: the two collocation products in gamma across the groups of that
//     position, then eta_eff = eta + sigma S for each group's plane.
#include "k_common.h"

namespace {

constexpr int FP_THREADS = 256;
constexpr int FP_MAXG = 64;  // largest number of energy groups with the coupling on

// contraction weight of moment k in Q = M0^2 - M1.M1 + M2:M2 - M3:.M3 (each
// off-diagonal component of a symmetric tensor counts once per index order)
SP6_DEV double q_weight(int k) {
  if (k == 0) return 1.0;
  if (k <= 3) return -1.0;
  if (k <= 6) return 1.0;
  if (k <= 9) return 2.0;
  if (k <= 12) return -1.0;
  if (k <= 18) return -3.0;
  if (k == 19) return -6.0;
  return 0.0;
}

// one step of the transposed reduction: a lane keeps the half of its C values
// selected by bit O of its lane index and receives the partner's share of it
template <int O, int C>
SP6_DEV void tr_step(double (&v)[32], int lane) {
  if constexpr (C == 1) {
    v[0] += __shfl_xor(v[0], O, 64);
  } else {
    constexpr int H = C / 2;
    const bool up = (lane & O) != 0;
#pragma unroll
    for (int j = 0; j < H; ++j) {
      const double send = up ? v[j] : v[H + j];
      const double keep = up ? v[H + j] : v[j];
      v[j] = keep + __shfl_xor(send, O, 64);
    }
  }
}

// Lanes take the columns (Phi nodes) of 64 / NP planes; each lane sums the 20
// moments over the Theta rows of its column, then the lanes of a plane reduce
// them.  For NP >= 32 the reduction is transposed: at each butterfly step a lane
// keeps one half of its values and trades the other half with its partner, so
// that after the steps lane l of the plane holds moment l (NP = 32) or l / 2
// (NP = 64) summed over the plane (31 or 32 exchanges instead of 20 log2 NP);
// Q is then a weighted sum of squares over those lanes.
template <int NP, typename TI>
__global__ __launch_bounds__(FP_THREADS) void k_fp_moments(KDims d, KTab t, const TI* __restrict__ Y,
                                                           double* __restrict__ mq) {
  __shared__ double sW[32], sCT[32], sST[32];
  const int tid = threadIdx.x;
  if (tid < d.n_Th) {
    sW[tid] = 4.0 * M_PI * t.wmean[tid];  // w_i (2 pi / n_Phi)
    sCT[tid] = t.cos_Th[tid];
    sST[tid] = t.sin_Th[tid];
  }
  __syncthreads();
  constexpr int PPW = 64 / NP;  // planes per wavefront
  const int lane = tid & 63, nT = d.n_Th;
  const int pl = lane / NP, m = lane % NP;  // plane within the group, column
  const double cP = t.cos_Ph[m], sP = t.sin_Ph[m];
  const int64_t ngroups = (d.nplanes + PPW - 1) / PPW;
  const int64_t wstep = int64_t(gridDim.x) * (FP_THREADS / 64);
  for (int64_t gi = int64_t(blockIdx.x) * (FP_THREADS / 64) + (tid >> 6); gi < ngroups; gi += wstep) {
    const int64_t pid = gi * PPW + pl;
    const bool ok = pid < d.nplanes;
    double v[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) v[k] = 0.0;
    if (ok) {
      const TI* __restrict__ col = Y + pid * d.plane + m;
      for (int i = 0; i < nT; ++i) {
        const double f = sW[i] * double(col[i * NP]);
        const double x = sCT[i], y = sST[i] * cP, z = sST[i] * sP;
        const double fx = f * x, fy = f * y, fz = f * z;
        v[0] += f;
        v[1] += fx;
        v[2] += fy;
        v[3] += fz;
        v[4] += fx * x;
        v[5] += fy * y;
        v[6] += fz * z;
        v[7] += fx * y;
        v[8] += fx * z;
        v[9] += fy * z;
        v[10] += fx * x * x;
        v[11] += fy * y * y;
        v[12] += fz * z * z;
        v[13] += fx * x * y;
        v[14] += fx * x * z;
        v[15] += fx * y * y;
        v[16] += fy * y * z;
        v[17] += fx * z * z;
        v[18] += fy * z * z;
        v[19] += fx * y * z;
      }
    }
    double M0, Q = 0.0;
    if constexpr (NP >= 32) {
      if constexpr (NP == 64) tr_step<32, 32>(v, lane);
      constexpr int C0 = NP == 64 ? 16 : 32;  // values held before the offset-16 step
      tr_step<16, C0>(v, lane);
      tr_step<8, C0 / 2>(v, lane);
      tr_step<4, C0 / 4>(v, lane);
      tr_step<2, C0 / 8>(v, lane);
      tr_step<1, C0 / 16>(v, lane);
      const int k = NP == 64 ? (lane >> 1) & 31 : lane & 31;
      const bool own = NP == 32 || (lane & 1) == 0;  // one lane per moment
      double q = own ? q_weight(k) * v[0] * v[0] : 0.0;
#pragma unroll
      for (int o = 1; o < NP; o <<= 1) q += __shfl_xor(q, o, 64);
      Q = q;
      M0 = v[0];  // the plane's first lane holds moment 0
    } else {
#pragma unroll
      for (int k = 0; k < 20; ++k)
#pragma unroll
        for (int o = 1; o < NP; o <<= 1) v[k] += __shfl_xor(v[k], o, 64);
      M0 = v[0];
#pragma unroll
      for (int k = 0; k < 20; ++k) Q += q_weight(k) * v[k] * v[k];
    }
    if (ok && m == 0) {
      mq[2 * pid] = M0;
      mq[2 * pid + 1] = Q;
    }
  }
}

__global__ __launch_bounds__(FP_MAXG) void k_fp_source(KDims d, const double* __restrict__ D, const double* __restrict__ gam,
                                                       double alpha, const double* __restrict__ mq,
                                                       const double* __restrict__ eta, const double* __restrict__ sigma,
                                                       double* __restrict__ eta_eff) {
  __shared__ double sM[FP_MAXG], sQ[FP_MAXG], sF[FP_MAXG];
  const int k = threadIdx.x, n = d.n_eps;
  const int64_t per = d.nplanes / n;  // planes of one energy group
  const int64_t pid = int64_t(k) * per + blockIdx.x;
  if (k < n) {
    sM[k] = mq[2 * pid];
    sQ[k] = mq[2 * pid + 1];
  }
  __syncthreads();
  if (k < n) {
    const double* __restrict__ Dk = D + size_t(k) * n;
    double dM = 0.0;
    for (int j = 0; j < n; ++j) dM += Dk[j] * sM[j];
    const double g = gam[k];
    sF[k] = alpha * g * g * dM + (g * g - 2.0 * alpha * g) * sM[k];
  }
  __syncthreads();
  if (k < n) {
    const double* __restrict__ Dk = D + size_t(k) * n;
    double dF = 0.0, dQ = 0.0;
    for (int j = 0; j < n; ++j) {
      dF += Dk[j] * sF[j];
      dQ += Dk[j] * sQ[j];
    }
    const double S = dF / (4.0 * M_PI) + 3.0 / (128.0 * M_PI * M_PI) * dQ;
    eta_eff[pid] = eta[pid] + sigma[pid] * S;
  }
}

}  // namespace

hipError_t launch_fp_source(const KDims& d, const KTab& t, const void* Y, bool y_f32, const double* D,
                            const double* gam, double alpha, double* mq, const double* eta, const double* sigma,
                            double* eta_eff, hipStream_t s) {
  if (d.n_eps > FP_MAXG || d.n_Th > 32 || d.n_Ph > 64 || (d.n_Ph & (d.n_Ph - 1))) return hipErrorInvalidValue;
  const int64_t ngroups = (d.nplanes + 64 / d.n_Ph - 1) / (64 / d.n_Ph);
  int64_t blocks = (ngroups + FP_THREADS / 64 - 1) / (FP_THREADS / 64);
  const int64_t cap = int64_t(d.ncu) * 8;
  if (blocks > cap) blocks = cap;
  const unsigned nb = unsigned(blocks);
  const double* Yd = static_cast<const double*>(Y);
  const float* Yf = static_cast<const float*>(Y);
#define FP_CASE(N)                                                    \
  case N:                                                             \
    if (y_f32)                                                        \
      k_fp_moments<N, float><<<nb, FP_THREADS, 0, s>>>(d, t, Yf, mq);  \
    else                                                              \
      k_fp_moments<N, double><<<nb, FP_THREADS, 0, s>>>(d, t, Yd, mq); \
    break;
  switch (d.n_Ph) {
    FP_CASE(4) FP_CASE(8) FP_CASE(16) FP_CASE(32) FP_CASE(64)
    default: return hipErrorInvalidValue;
  }
#undef FP_CASE
  const int64_t per = d.nplanes / d.n_eps;
  k_fp_source<<<unsigned(per), FP_MAXG, 0, s>>>(d, D, gam, alpha, mq, eta, sigma, eta_eff);
  return hipGetLastError();
}
