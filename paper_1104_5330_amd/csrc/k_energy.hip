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

// adds f times the 20 monomials of the direction (x, y, z) to v[0..19]:
// 1; x y z; xx yy zz xy xz yz; xxx yyy zzz xxy xxz xyy yyz xzz yzz xyz
SP6_DEV void add_moments(double (&v)[32], double f, double x, double y, double z) {
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

// the 20 monomials of (x, y, z) in the order of add_moments, dotted with c
SP6_DEV double eval_monomials(const double* c, double x, double y, double z) {
  return c[0] + c[1] * x + c[2] * y + c[3] * z + c[4] * x * x + c[5] * y * y + c[6] * z * z + c[7] * x * y +
         c[8] * x * z + c[9] * y * z + c[10] * x * x * x + c[11] * y * y * y + c[12] * z * z * z + c[13] * x * x * y +
         c[14] * x * x * z + c[15] * x * y * y + c[16] * y * y * z + c[17] * x * z * z + c[18] * y * z * z +
         c[19] * x * y * z;
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
      // the column's rows in batches of eight loads in flight
      const TI* __restrict__ col = Y + pid * d.plane + m;
      for (int i0 = 0; i0 < nT; i0 += 8) {
        double f[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) f[u] = i0 + u < nT ? double(col[(i0 + u) * NP]) : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int i = i0 + u;
          if (i < nT) add_moments(v, sW[i] * f[u], sCT[i], sST[i] * cP, sST[i] * sP);
        }
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

// ---------------------------------------------------------------------------
// adjoint: the transpose of the linearisation at the stage input Y of
// F -> M sigma S(F), applied to X = xs x (M: inflow mask):
//   u = sigma sum_w M X (per plane);  a0 = L1^T u,  aQ = 3/(128 pi^2) D^T u,
//   L1 = (1/4pi) D [diag(alpha gamma^2) D + diag(gamma^2 - 2 alpha gamma)];
//   result(w) = wq(w) sum_k C_k phi_k(w),  C_k = a0 [k = 0] + 2 aQ q_k M_k
// (phi_k the monomials of add_moments, M_k the moments of Y, q_k the weights
// of Q = sum_k q_k M_k^2); sigma's gradient gains S(Y) sum_w M X.

// per plane: the 20 moments of Y and sum_w M X into mom[plane][21]
template <int NP>
__global__ __launch_bounds__(FP_THREADS) void k_fp_adj_moments(KDims d, KTab t, const double* __restrict__ Y,
                                                               const double* __restrict__ X, double xs,
                                                               double* __restrict__ mom) {
  __shared__ double sW[32], sCT[32], sST[32];
  const int tid = threadIdx.x;
  if (tid < d.n_Th) {
    sW[tid] = 4.0 * M_PI * t.wmean[tid];
    sCT[tid] = t.cos_Th[tid];
    sST[tid] = t.sin_Th[tid];
  }
  __syncthreads();
  constexpr int PPW = 64 / NP;
  const int lane = tid & 63, nT = d.n_Th;
  const int pl = lane / NP, m = lane % NP;
  const double cP = t.cos_Ph[m], sP = t.sin_Ph[m];
  const int sh_ph = __builtin_ctz(d.n_ph), sh_th = __builtin_ctz(d.n_th);
  const int64_t ngroups = (d.nplanes + PPW - 1) / PPW;
  const int64_t wstep = int64_t(gridDim.x) * (FP_THREADS / 64);
  for (int64_t gi = int64_t(blockIdx.x) * (FP_THREADS / 64) + (tid >> 6); gi < ngroups; gi += wstep) {
    const int64_t pid = gi * PPW + pl;
    const bool ok = pid < d.nplanes;
    double v[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) v[k] = 0.0;
    if (ok) {
      const int j = int(pid >> (sh_ph + sh_th)) % d.n_r;  // radial index of the plane
      const double* __restrict__ yc = Y + pid * d.plane + m;
      const double* __restrict__ xc = X + pid * d.plane + m;
      for (int i0 = 0; i0 < nT; i0 += 8) {
        double fy[8], fx[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          fy[u] = i0 + u < nT ? yc[(i0 + u) * NP] : 0.0;
          fx[u] = i0 + u < nT ? xc[(i0 + u) * NP] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int i = i0 + u;
          if (i >= nT) continue;
          add_moments(v, sW[i] * fy[u], sCT[i], sST[i] * cP, sST[i] * sP);
          const bool held = d.bc && ((j == 0 && sCT[i] > 0.0) || (j == d.n_r - 1 && sCT[i] < 0.0));
          v[20] += held ? 0.0 : xs * fx[u];
        }
      }
    }
    if constexpr (NP >= 32) {
      if constexpr (NP == 64) tr_step<32, 32>(v, lane);
      constexpr int C0 = NP == 64 ? 16 : 32;
      tr_step<16, C0>(v, lane);
      tr_step<8, C0 / 2>(v, lane);
      tr_step<4, C0 / 4>(v, lane);
      tr_step<2, C0 / 8>(v, lane);
      tr_step<1, C0 / 16>(v, lane);
      const int k = NP == 64 ? (lane >> 1) & 31 : lane & 31;
      const bool own = NP == 32 || (lane & 1) == 0;
      if (ok && own && k <= 20) mom[21 * pid + k] = v[0];
    } else {
#pragma unroll
      for (int k = 0; k <= 20; ++k)
#pragma unroll
        for (int o = 1; o < NP; o <<= 1) v[k] += __shfl_xor(v[k], o, 64);
      if (ok && m == 0)
#pragma unroll
        for (int k = 0; k <= 20; ++k) mom[21 * pid + k] = v[k];
    }
  }
}

// per position, thread k for group k: C[plane][20] and sigma's gradient
__global__ __launch_bounds__(FP_MAXG) void k_fp_adj_source(KDims d, const double* __restrict__ D,
                                                           const double* __restrict__ gam, double alpha,
                                                           const double* __restrict__ mom,
                                                           const double* __restrict__ sigma,
                                                           double* __restrict__ C, double* __restrict__ gs) {
  __shared__ double sM[FP_MAXG], sQ[FP_MAXG], sU[FP_MAXG], sF[FP_MAXG], sW[FP_MAXG], sA[FP_MAXG];
  const int k = threadIdx.x, n = d.n_eps;
  const int64_t per = d.nplanes / n;
  const int64_t pid = int64_t(k) * per + blockIdx.x;
  double g = 0.0;
  if (k < n) {
    const double* mk = mom + 21 * pid;
    double q = 0.0;
#pragma unroll
    for (int j = 0; j < 20; ++j) q += q_weight(j) * mk[j] * mk[j];
    sM[k] = mk[0];
    sQ[k] = q;
    sU[k] = sigma[pid] * mk[20];
    g = gam[k];
  }
  __syncthreads();
  if (k < n) {
    double dM = 0.0, w = 0.0;
    for (int j = 0; j < n; ++j) {
      dM += D[size_t(k) * n + j] * sM[j];
      w += D[size_t(j) * n + k] * sU[j];  // (D^T u)_k
    }
    sF[k] = alpha * g * g * dM + (g * g - 2.0 * alpha * g) * sM[k];  // forward flux at Y
    sW[k] = w;
    sA[k] = alpha * g * g * w;
  }
  __syncthreads();
  if (k < n) {
    double dF = 0.0, dQ = 0.0, dA = 0.0;
    for (int j = 0; j < n; ++j) {
      const double Dkj = D[size_t(k) * n + j];
      dF += Dkj * sF[j];
      dQ += Dkj * sQ[j];
      dA += D[size_t(j) * n + k] * sA[j];  // (D^T diag(alpha gamma^2) D^T u)_k
    }
    const double cq = 3.0 / (128.0 * M_PI * M_PI);
    const double a0 = (dA + (g * g - 2.0 * alpha * g) * sW[k]) / (4.0 * M_PI);
    const double aQ = cq * sW[k];
    const double* mk = mom + 21 * pid;
    double* ck = C + 20 * pid;
#pragma unroll
    for (int j = 0; j < 20; ++j) ck[j] = 2.0 * aQ * q_weight(j) * mk[j];
    ck[0] += a0;
    if (gs) {
      const double S = dF / (4.0 * M_PI) + cq * dQ;
      gs[pid] += S * mk[20];
    }
  }
}

// adds wq(w) sum_k C_k phi_k(w) to lacc and kb * that to kbnext (if given);
// lane = column of a plane, as in the moment pass
template <int NP>
__global__ __launch_bounds__(FP_THREADS) void k_fp_adj_apply(KDims d, KTab t, const double* __restrict__ C,
                                                             double* __restrict__ lacc, double* __restrict__ kbnext,
                                                             double kb) {
  __shared__ double sW[32], sCT[32], sST[32];
  const int tid = threadIdx.x;
  if (tid < d.n_Th) {
    sW[tid] = 4.0 * M_PI * t.wmean[tid];
    sCT[tid] = t.cos_Th[tid];
    sST[tid] = t.sin_Th[tid];
  }
  __syncthreads();
  constexpr int PPW = 64 / NP;
  const int lane = tid & 63, nT = d.n_Th;
  const int pl = lane / NP, m = lane % NP;
  const double cP = t.cos_Ph[m], sP = t.sin_Ph[m];
  const int64_t ngroups = (d.nplanes + PPW - 1) / PPW;
  const int64_t wstep = int64_t(gridDim.x) * (FP_THREADS / 64);
  for (int64_t gi = int64_t(blockIdx.x) * (FP_THREADS / 64) + (tid >> 6); gi < ngroups; gi += wstep) {
    const int64_t pid = gi * PPW + pl;
    if (pid >= d.nplanes) continue;
    double c[20];
#pragma unroll
    for (int k = 0; k < 20; ++k) c[k] = C[20 * pid + k];
    const int64_t base = pid * d.plane + m;
    for (int i = 0; i < nT; ++i) {
      const double v = sW[i] * eval_monomials(c, sCT[i], sST[i] * cP, sST[i] * sP);
      const int64_t p = base + int64_t(i) * NP;
      lacc[p] += v;
      if (kbnext) kbnext[p] += kb * v;
    }
  }
}

}  // namespace

hipError_t launch_fp_adj(const KDims& d, const KTab& t, const double* Y, const double* X, double xs, const double* D,
                         const double* gam, double alpha, double* mom, const double* sigma, double* C, double* gs,
                         hipStream_t s) {
  if (d.n_eps > FP_MAXG || d.n_Th > 32 || d.n_Ph > 64 || (d.n_Ph & (d.n_Ph - 1))) return hipErrorInvalidValue;
  const int64_t ngroups = (d.nplanes + 64 / d.n_Ph - 1) / (64 / d.n_Ph);
  int64_t blocks = (ngroups + FP_THREADS / 64 - 1) / (FP_THREADS / 64);
  const int64_t cap = int64_t(d.ncu) * 8;
  if (blocks > cap) blocks = cap;
  const unsigned nb = unsigned(blocks);
  switch (d.n_Ph) {
    case 4: k_fp_adj_moments<4><<<nb, FP_THREADS, 0, s>>>(d, t, Y, X, xs, mom); break;
    case 8: k_fp_adj_moments<8><<<nb, FP_THREADS, 0, s>>>(d, t, Y, X, xs, mom); break;
    case 16: k_fp_adj_moments<16><<<nb, FP_THREADS, 0, s>>>(d, t, Y, X, xs, mom); break;
    case 32: k_fp_adj_moments<32><<<nb, FP_THREADS, 0, s>>>(d, t, Y, X, xs, mom); break;
    case 64: k_fp_adj_moments<64><<<nb, FP_THREADS, 0, s>>>(d, t, Y, X, xs, mom); break;
    default: return hipErrorInvalidValue;
  }
  const int64_t per = d.nplanes / d.n_eps;
  k_fp_adj_source<<<unsigned(per), FP_MAXG, 0, s>>>(d, D, gam, alpha, mom, sigma, C, gs);
  return hipGetLastError();
}

hipError_t launch_fp_adj_apply(const KDims& d, const KTab& t, const double* C, double* lacc, double* kbnext, double kb,
                               hipStream_t s) {
  if (d.n_Th > 32 || d.n_Ph > 64 || (d.n_Ph & (d.n_Ph - 1))) return hipErrorInvalidValue;
  const int64_t ngroups = (d.nplanes + 64 / d.n_Ph - 1) / (64 / d.n_Ph);
  int64_t blocks = (ngroups + FP_THREADS / 64 - 1) / (FP_THREADS / 64);
  const int64_t cap = int64_t(d.ncu) * 8;
  if (blocks > cap) blocks = cap;
  const unsigned nb = unsigned(blocks);
  switch (d.n_Ph) {
    case 4: k_fp_adj_apply<4><<<nb, FP_THREADS, 0, s>>>(d, t, C, lacc, kbnext, kb); break;
    case 8: k_fp_adj_apply<8><<<nb, FP_THREADS, 0, s>>>(d, t, C, lacc, kbnext, kb); break;
    case 16: k_fp_adj_apply<16><<<nb, FP_THREADS, 0, s>>>(d, t, C, lacc, kbnext, kb); break;
    case 32: k_fp_adj_apply<32><<<nb, FP_THREADS, 0, s>>>(d, t, C, lacc, kbnext, kb); break;
    case 64: k_fp_adj_apply<64><<<nb, FP_THREADS, 0, s>>>(d, t, C, lacc, kbnext, kb); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

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
