// Inflow projection, filter driver, particle number / boundary fluxes
// (App. A, Eqs. Npho and Flux) and the outgoing-flux map.
#include "k_common.h"

hipError_t launch_filter_columns(const KDims& d, const KTab& t, double* F, hipStream_t s);
hipError_t launch_filter_plane(const KDims& d, const KTab& t, double* F, hipStream_t s);

namespace {

// F := g at the inflow nodes: r_in with cos Theta > 0 (g_in), r_out with
// cos Theta < 0 (g_out); a null plane means zero.
__global__ __launch_bounds__(256) void k_project(KDims d, KTab t, KCoef c, double* __restrict__ F) {
  const int64_t per_e = int64_t(d.n_th) * d.n_ph * d.plane;
  const int64_t gid = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (gid >= 2 * per_e * d.n_eps) return;
  const int side = int(gid / (per_e * d.n_eps));  // 0: r_in, 1: r_out
  const int64_t rest = gid % (per_e * d.n_eps);
  const int64_t e = rest / per_e, w = rest % per_e;
  const int iTh = int((w % d.plane) / d.n_Ph);
  const double cT = t.cos_Th[iTh];
  const bool inflow = side == 0 ? cT > 0.0 : cT < 0.0;
  if (!inflow) return;
  const double* g = side == 0 ? c.g_in : c.g_out;
  const int j = side == 0 ? 0 : d.n_r - 1;
  F[(e * d.n_r + j) * d.M + w] = g ? g[rest] : 0.0;
}

// Block (eps, r, theta): weighted sums over its n_phi * plane points, reduced in a
// fixed order (deterministic).  partial[blk][0] = particle-number sum,
// [1] flux sum at r_in (j = 0 blocks), [2] flux sum at r_out.
constexpr int DB = 256;
__global__ __launch_bounds__(DB) void k_diag_partial(KDims d, KTab t, const double* __restrict__ F,
                                                     double* __restrict__ partial) {
  __shared__ double red[3][DB];
  const int64_t blk = blockIdx.x;  // = (e * n_r + j) * n_th + l
  const int l = int(blk % d.n_th);
  const int j = int((blk / d.n_th) % d.n_r);
  const int64_t n = int64_t(d.n_ph) * d.plane;
  const double* __restrict__ src = F + blk * n;
  double sN = 0.0, sJ = 0.0;
  for (int64_t p = threadIdx.x; p < n; p += DB) {
    const int iTh = int((p % d.plane) / d.n_Ph);
    const double f = src[p];
    sN += t.qN[(int64_t(j) * d.n_th + l) * d.n_Th + iTh] * f;
    sJ += t.qJ[int64_t(l) * d.n_Th + iTh] * f;
  }
  red[0][threadIdx.x] = sN;
  red[1][threadIdx.x] = (j == 0) ? sJ : 0.0;
  red[2][threadIdx.x] = (j == d.n_r - 1) ? sJ : 0.0;
  __syncthreads();
  for (int w = DB / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int q = 0; q < 3; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 3) partial[blk * 3 + threadIdx.x] = red[threadIdx.x][0];
}

// One block per energy group: fixed-order sum of its n_r * n_th partials.
__global__ __launch_bounds__(DB) void k_diag_final(KDims d, const double* __restrict__ partial,
                                                   double r_in2, double r_out2, double* __restrict__ out3) {
  __shared__ double red[3][DB];
  const int e = blockIdx.x;
  const int64_t nb = int64_t(d.n_r) * d.n_th;
  double s[3] = {0.0, 0.0, 0.0};
  for (int64_t b = threadIdx.x; b < nb; b += DB)
    for (int q = 0; q < 3; ++q) s[q] += partial[(e * nb + b) * 3 + q];
  for (int q = 0; q < 3; ++q) red[q][threadIdx.x] = s[q];
  __syncthreads();
  for (int w = DB / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int q = 0; q < 3; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out3[e * 3 + 0] = red[0][0];
    out3[e * 3 + 1] = r_in2 * red[1][0];
    out3[e * 3 + 2] = r_out2 * red[2][0];
  }
}

// One wavefront per (eps, theta, phi): j = sum_{i, m} wflux_i F(r_out, i, m).
__global__ __launch_bounds__(256) void k_outflux(KDims d, KTab t, const double* __restrict__ F,
                                                 double* __restrict__ jmap) {
  const int64_t w = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t nmap = int64_t(d.n_eps) * d.n_th * d.n_ph;
  if (w >= nmap) return;
  const int64_t e = w / (int64_t(d.n_th) * d.n_ph), lk = w % (int64_t(d.n_th) * d.n_ph);
  const double* __restrict__ src = F + (e * d.n_r + (d.n_r - 1)) * d.M + lk * d.plane;
  double s = 0.0;
  for (int p = lane; p < d.plane; p += 64) s += t.wflux[p / d.n_Ph] * src[p];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) jmap[w] = s;
}

// Transpose of k_outflux: out = 0 except at r_out, where
// out(eps, theta, phi, Theta_i, Phi_m) = jbar(eps, theta, phi) * wflux_i.
__global__ __launch_bounds__(256) void k_outflux_T(KDims d, KTab t, const double* __restrict__ jbar,
                                                   double* __restrict__ out) {
  const int64_t gid = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (gid >= d.P) return;
  const int64_t e = gid / (d.n_r * d.M);
  const int64_t rest = gid % (d.n_r * d.M);
  const int j = int(rest / d.M);
  const int64_t w = rest % d.M;  // (theta, phi, Theta, Phi)
  double v = 0.0;
  if (j == d.n_r - 1) {
    const int iTh = int((w % d.plane) / d.n_Ph);
    v = jbar[e * (d.M / d.plane) + w / d.plane] * t.wflux[iTh];
  }
  out[gid] = v;
}

}  // namespace

hipError_t launch_outflux_T(const KDims& d, const KTab& t, const double* jbar, double* out, hipStream_t s) {
  k_outflux_T<<<unsigned((d.P + 255) / 256), 256, 0, s>>>(d, t, jbar, out);
  return hipGetLastError();
}

hipError_t launch_project(const KDims& d, const KTab& t, const KCoef& c, double* F, hipStream_t s) {
  const int64_t n = 2 * int64_t(d.n_eps) * d.n_th * d.n_ph * d.plane;
  k_project<<<unsigned((n + 255) / 256), 256, 0, s>>>(d, t, c, F);
  return hipGetLastError();
}

hipError_t launch_filter(const KDims& d, const KTab& t, double* F, int radial, hipStream_t s) {
  hipError_t e = launch_filter_columns(d, t, F, s);
  if (e == hipSuccess) e = launch_filter_plane(d, t, F, s);
  if (e == hipSuccess && radial) e = launch_filter_radial(d, t, F, radial == 2, s);
  return e;
}

size_t diag_partial_count(const KDims& d) { return size_t(d.n_eps) * d.n_r * d.n_th * 3; }

hipError_t launch_diag(const KDims& d, const KTab& t, const double* F, double* partial, double r_in2,
                       double r_out2, double* out3, hipStream_t s) {
  const unsigned nb = unsigned(int64_t(d.n_eps) * d.n_r * d.n_th);
  k_diag_partial<<<nb, DB, 0, s>>>(d, t, F, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_diag_final<<<unsigned(d.n_eps), DB, 0, s>>>(d, partial, r_in2, r_out2, out3);
  return hipGetLastError();
}

hipError_t launch_outflux(const KDims& d, const KTab& t, const double* F, double* j, hipStream_t s) {
  const int64_t nmap = int64_t(d.n_eps) * d.n_th * d.n_ph;
  k_outflux<<<unsigned((nmap + 3) / 4), 256, 0, s>>>(d, t, F, j);
  return hipGetLastError();
}
