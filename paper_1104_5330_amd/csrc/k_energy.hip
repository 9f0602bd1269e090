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
// eta + sigma S as its emissivity:
//   k_fp_moments: one workgroup per plane reduces the plane to (M0, Q): 20
//     moments summed per thread from the coalesced plane, reduced over the
//     wavefront and then over the wavefronts in a fixed order (8 bytes read per
//     point, 16 written per plane);
//   k_fp_source: one workgroup per position (r, theta, phi), thread k for group
//     k: the two collocation products in gamma across the groups of that
//     position, then eta_eff = eta + sigma S for each group's plane.
#include "k_common.h"

namespace {

constexpr int FP_THREADS = 256;
constexpr int FP_MAXG = 64;  // largest number of energy groups with the coupling on

__global__ __launch_bounds__(FP_THREADS) void k_fp_moments(KDims d, KTab t, const double* __restrict__ Y,
                                                           double* __restrict__ mq) {
  __shared__ double sW[32], sCT[32], sST[32], sCP[64], sSP[64];
  __shared__ double sRed[FP_THREADS / 64][20];
  const int tid = threadIdx.x;
  if (tid < d.n_Th) {
    sW[tid] = 4.0 * M_PI * t.wmean[tid];  // w_i (2 pi / n_Phi)
    sCT[tid] = t.cos_Th[tid];
    sST[tid] = t.sin_Th[tid];
  }
  if (tid < d.n_Ph) {
    sCP[tid] = t.cos_Ph[tid];
    sSP[tid] = t.sin_Ph[tid];
  }
  __syncthreads();
  const int64_t pid = blockIdx.x;
  const double* __restrict__ P = Y + pid * d.plane;
  const int sh = __builtin_ctz(d.n_Ph), mk = d.n_Ph - 1;
  // moments: 0; x y z; xx yy zz xy xz yz; xxx yyy zzz xxy xxz xyy yyz xzz yzz xyz
  double m[20];
#pragma unroll
  for (int k = 0; k < 20; ++k) m[k] = 0.0;
  for (int p = tid; p < d.plane; p += FP_THREADS) {
    const int i = p >> sh, j = p & mk;
    const double f = sW[i] * P[p];
    const double x = sCT[i], y = sST[i] * sCP[j], z = sST[i] * sSP[j];
    const double fx = f * x, fy = f * y, fz = f * z;
    m[0] += f;
    m[1] += fx;
    m[2] += fy;
    m[3] += fz;
    m[4] += fx * x;
    m[5] += fy * y;
    m[6] += fz * z;
    m[7] += fx * y;
    m[8] += fx * z;
    m[9] += fy * z;
    m[10] += fx * x * x;
    m[11] += fy * y * y;
    m[12] += fz * z * z;
    m[13] += fx * x * y;
    m[14] += fx * x * z;
    m[15] += fx * y * y;
    m[16] += fy * y * z;
    m[17] += fx * z * z;
    m[18] += fy * z * z;
    m[19] += fx * y * z;
  }
#pragma unroll
  for (int k = 0; k < 20; ++k) {
    double v = m[k];
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
    if ((tid & 63) == 0) sRed[tid >> 6][k] = v;
  }
  __syncthreads();
  if (tid == 0) {
    double M[20];
#pragma unroll
    for (int k = 0; k < 20; ++k) {
      double s = 0.0;
#pragma unroll
      for (int w = 0; w < FP_THREADS / 64; ++w) s += sRed[w][k];
      M[k] = s;
    }
    // full contractions: each off-diagonal component of a symmetric tensor
    // stands for as many entries as it has index permutations
    const double m1 = M[1] * M[1] + M[2] * M[2] + M[3] * M[3];
    const double m2 = M[4] * M[4] + M[5] * M[5] + M[6] * M[6] + 2.0 * (M[7] * M[7] + M[8] * M[8] + M[9] * M[9]);
    const double m3 = M[10] * M[10] + M[11] * M[11] + M[12] * M[12] +
                      3.0 * (M[13] * M[13] + M[14] * M[14] + M[15] * M[15] + M[16] * M[16] + M[17] * M[17] +
                             M[18] * M[18]) +
                      6.0 * M[19] * M[19];
    mq[2 * pid] = M[0];
    mq[2 * pid + 1] = M[0] * M[0] - m1 + m2 - m3;
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

hipError_t launch_fp_source(const KDims& d, const KTab& t, const double* Y, const double* D, const double* gam,
                            double alpha, double* mq, const double* eta, const double* sigma, double* eta_eff,
                            hipStream_t s) {
  if (d.n_eps > FP_MAXG || d.n_Th > 32 || d.n_Ph > 64) return hipErrorInvalidValue;
  k_fp_moments<<<unsigned(d.nplanes), FP_THREADS, 0, s>>>(d, t, Y, mq);
  const int64_t per = d.nplanes / d.n_eps;
  k_fp_source<<<unsigned(per), FP_MAXG, 0, s>>>(d, D, gam, alpha, mq, eta, sigma, eta_eff);
  return hipGetLastError();
}
