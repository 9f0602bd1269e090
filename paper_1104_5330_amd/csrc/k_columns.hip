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

// 4 KB aligned: the 64-point line kernels read a 16 KB table with scalar loads,
// and where it started at an unaligned address in the constant segment (which
// shifts from build to build) the phi and theta passes on 64-point lines ran 60 %
// slower
__constant__ __attribute__((aligned(4096))) double c_lines[LINE_TAB_KINDS * LINE_TAB_SIZE];
__constant__ __attribute__((aligned(4096))) float c_lines_f[LINE_TAB_KINDS * LINE_TAB_SIZE];  // FP32 copy for the mixed path

template <int L, typename TC = double>
SP6_DEV const TC* line_tab(int kind) {
  if constexpr (sizeof(TC) == 8)
    return c_lines + kind * LINE_TAB_SIZE + line_tab_offset(L);
  else
    return c_lines_f + kind * LINE_TAB_SIZE + line_tab_offset(L);
}

// ---------------------------------------------------------------------------
// phi lines

// TI: stored type of the input state, TO: stored type of T and compute type
// (double, double) on the FP64 path; (double or float, float) on the mixed path.
template <int L, bool ACCUM, typename TI, typename TO>
__global__ __launch_bounds__(CB) void k_phi(KDims d, KTab t, const TI* __restrict__ Y,
                                            TO* __restrict__ T, double coef_sign, int mask_in,
                                            double in_scale) {
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

  TO s_in = TO(in_scale);
  if (mask_in && is_inflow(d, t, j, iTh)) s_in = TO(0);
  TO v[L];
#pragma unroll
  for (int k = 0; k < L; ++k) v[k] = TO(Y[base + k * stride]) * s_in;
  TO tv[ACCUM ? L : 1];
  if constexpr (ACCUM) {
#pragma unroll
    for (int k = 0; k < L; ++k) tv[k] = T[base + k * stride];
  }
  const TO s = TO(coef_sign * t.sin_Th[iTh] * t.sin_Ph[m] * t.inv_r[j] * t.inv_sin_th[l]);
  eo_split<L>(v);
  eo_pairs<L, L / 2, true>(line_tab<L, TO>(LT_DERIV), 0, v, [&](int k, TO z) {
    const TO val = s * z;
    if constexpr (ACCUM)
      T[base + k * stride] = tv[k] + val;
    else
      T[base + k * stride] = val;
  });
}

// ---------------------------------------------------------------------------
// theta DFS lines: thread = (eps, r, k < n_phi/2, column c); it owns the orbit
// {(k, c), (k + n_phi/2, c')} with c' the column at Phi_m + pi.

template <int NTH, bool ACCUM, typename TI, typename TO>
__global__ __launch_bounds__(CB) void k_theta(KDims d, KTab t, const TI* __restrict__ Y,
                                              TO* __restrict__ T, double coef_sign, int mask_in,
                                              double in_scale) {
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

  TO s_in = TO(in_scale);
  if (mask_in && is_inflow(d, t, j, iTh)) s_in = TO(0);
  TO v[L];
#pragma unroll
  for (int l = 0; l < NTH; ++l) {
    v[l] = TO(Y[ba + l * rowstride]) * s_in;
    v[L - 1 - l] = TO(Y[bb + l * rowstride]) * s_in;
  }
  TO tv[ACCUM ? L : 1];
  if constexpr (ACCUM) {
#pragma unroll
    for (int l = 0; l < NTH; ++l) {
      tv[l] = T[ba + l * rowstride];
      tv[L - 1 - l] = T[bb + l * rowstride];
    }
  }
  // partner coefficient is -s (cos(Phi + pi) = -cos Phi) and the partner
  // derivative is -z[L-1-l]; both signs cancel.
  const TO s = TO(coef_sign * t.sin_Th[iTh] * t.cos_Ph[m] * t.inv_r[j]);
  eo_split<L>(v);
  eo_pairs<L, NTH, true>(line_tab<L, TO>(LT_DERIV), 0, v, [&](int q, TO z) {
    const TO val = s * z;
    const int64_t a = (q < NTH) ? ba + q * rowstride : bb + (L - 1 - q) * rowstride;
    if constexpr (ACCUM)
      T[a] = tv[q] + val;
    else
      T[a] = val;
  });
}

// ---------------------------------------------------------------------------
// radial lines on FP64 MFMA.  Per wavefront: 16 columns x all r as one
// (NRP x KP) * (KP x 16) product, NRP = 16 NRT rows, KP = 4 KS.
// Operand layouts of v_mfma_f64_16x16x4f64 (lane l):
//   A (16 x 4): A[l % 16][l / 16];  B (4 x 16): B[l / 16][l % 16];
//   C (16 x 16): register v holds C[l / 16 + 4 v][l % 16] (rows interleaved).

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));


template <int KS, bool ACCUM>
__global__ __launch_bounds__(CB) void k_radial(KDims d, KTab t, const double* __restrict__ Y,
                                               double* __restrict__ T, int transpose, int mask_in,
                                               double in_scale) {
  constexpr int NRT = (KS + 3) / 4;
  constexpr int NWV = CB / 64;
  const int lane = threadIdx.x & 63;
  const int wave = wave_uniform(threadIdx.x >> 6);
  const int lr = lane & 15, lk = lane >> 4;
  const double* __restrict__ Dp = transpose ? t.DpadT : t.Dpad;
  double a[NRT][KS];
#pragma unroll
  for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
    for (int s = 0; s < KS; ++s) a[rt][s] = Dp[(16 * rt + lr) * t.KP + 4 * s + lk];

  // column groups of 16; the resident workgroups advance through them together
  // (round k takes groups k G .. k G + G - 1, G = gridDim NWV, the wavefronts of a
  // workgroup side by side), in the direction d.rev.  Addresses are a
  // wave-uniform row pointer plus the 32-bit per-lane byte offset of row lk,
  // column lr.  Only the last k-step and the last row tile can reach past n_r
  // (KS = ceil(n_r / 4)); every other load and store is unconditional.
  const int gpe = int(d.M / 16);
  const int ngroups = gpe * d.n_eps;
  const int gstride = int(gridDim.x) * NWV;
  const int64_t M = d.M;
  const int n_r = d.n_r;
  const uint32_t boff = (uint32_t(lk) * uint32_t(M) + uint32_t(lr)) * 8u;
  auto ld = [&](const double* row) {
    return ld_stream<NT_RAD_LD>(reinterpret_cast<const double*>(reinterpret_cast<const char*>(row) + boff));
  };
  auto ldT = [&](const double* row) {
    return ld_stream<NT_RAD_LDT>(reinterpret_cast<const double*>(reinterpret_cast<const char*>(row) + boff));
  };
  auto at = [&](double* row) { return reinterpret_cast<double*>(reinterpret_cast<char*>(row) + boff); };
  // every extent is a power of two: divisions become shifts
  const int sh_g = __builtin_ctz(gpe), sh_P = __builtin_ctz(d.n_Ph);
  for (int k = int(blockIdx.x) * NWV + wave; k < ngroups; k += gstride) {
    const int g = d.rev ? ngroups - 1 - k : k;
    const int e = g >> sh_g;
    const int c0 = (g & (gpe - 1)) * 16;
    const int64_t gb = int64_t(e) * n_r * M + c0;
    const double* __restrict__ Yg = Y + gb;
    double* __restrict__ Tg = T + gb;
    const int iTh = ((c0 + lr) >> sh_P) & (d.n_Th - 1);
    const double cT = t.cos_Th[iTh];
    double b[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const double* row = Yg + int64_t(4 * s) * M;
      if (s < KS - 1)
        b[s] = ld(row);
      else
        b[s] = 4 * s + lk < n_r ? ld(row) : 0.0;
    }
    double tv[ACCUM ? NRT * 4 : 1];
    if constexpr (ACCUM) {
#pragma unroll
      for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double* row = Tg + int64_t(16 * rt + 4 * v) * M;
          if (rt < NRT - 1)
            tv[rt * 4 + v] = ldT(row);
          else
            tv[rt * 4 + v] = 16 * rt + lk + 4 * v < n_r ? ldT(row) : 0.0;
        }
    }
    if (mask_in) {
#pragma unroll
      for (int s = 0; s < KS; ++s)
        if (is_inflow(d, t, 4 * s + lk, iTh)) b[s] = 0.0;
    }
    if (in_scale != 1.0) {
#pragma unroll
      for (int s = 0; s < KS; ++s) b[s] *= in_scale;
    }
    v4d acc[NRT];
#pragma unroll
    for (int rt = 0; rt < NRT; ++rt) {
      acc[rt] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < KS; ++s) acc[rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rt][s], b[s], acc[rt], 0, 0, 0);
    }
#pragma unroll
    for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if (rt < NRT - 1 || 16 * rt + lk + 4 * v < n_r) {
          const double val = cT * acc[rt][v];
          double* dst = at(Tg + int64_t(16 * rt + 4 * v) * M);
          if constexpr (ACCUM)
            st_stream<NT_RAD_ST>(dst, tv[rt * 4 + v] + val);
          else
            st_stream<NT_RAD_ST>(dst, val);
        }
      }
  }
}

// ---------------------------------------------------------------------------
// radial filter (in place): F := Fr F along every r line, or Fr^T F.  Same
// FP64 MFMA tiling as the radial term; a wavefront reads all rows of its 16
// columns before it writes them, so in-place is safe (no restrict).

template <int KS>
__global__ __launch_bounds__(CB) void k_radial_filter(KDims d, KTab t, double* F, int transpose) {
  constexpr int NRT = (KS + 3) / 4;
  constexpr int NWV = CB / 64;
  const int lane = threadIdx.x & 63;
  const int wave = wave_uniform(threadIdx.x >> 6);
  const int lr = lane & 15, lk = lane >> 4;
  const double* __restrict__ Fp = transpose ? t.FpadT : t.Fpad;
  double a[NRT][KS];
#pragma unroll
  for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
    for (int s = 0; s < KS; ++s) a[rt][s] = Fp[(16 * rt + lr) * t.KP + 4 * s + lk];
  const int gpe = int(d.M / 16);
  const int ngroups = gpe * d.n_eps;
  const int per_blk = ((ngroups + int(gridDim.x) - 1) / int(gridDim.x) + NWV - 1) / NWV * NWV;
  const int gend = min(ngroups, per_blk * (int(blockIdx.x) + 1));
  const int64_t M = d.M;
  const int n_r = d.n_r;
  const uint32_t boff = (uint32_t(lk) * uint32_t(M) + uint32_t(lr)) * 8u;
  auto at = [&](double* row) { return reinterpret_cast<double*>(reinterpret_cast<char*>(row) + boff); };
  const int sh_g = __builtin_ctz(gpe);
  for (int g = per_blk * int(blockIdx.x) + wave; g < gend; g += NWV) {
    const int e = g >> sh_g;
    const int c0 = (g & (gpe - 1)) * 16;
    double* Fg = F + (int64_t(e) * n_r * M + c0);
    double b[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      double* row = Fg + int64_t(4 * s) * M;
      if (s < KS - 1)
        b[s] = *at(row);
      else
        b[s] = 4 * s + lk < n_r ? *at(row) : 0.0;
    }
    v4d acc[NRT];
#pragma unroll
    for (int rt = 0; rt < NRT; ++rt) {
      acc[rt] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < KS; ++s) acc[rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rt][s], b[s], acc[rt], 0, 0, 0);
    }
#pragma unroll
    for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        if (rt < NRT - 1 || 16 * rt + lk + 4 * v < n_r) *at(Fg + int64_t(16 * rt + 4 * v) * M) = acc[rt][v];
  }
}

// ---------------------------------------------------------------------------
// backward-Euler radial solve of the split step (App. B), in place: every r line
// of direction node Theta_i is multiplied by B_i, the inverse of I + dt cos(Theta_i)
// D_r (inflow row replaced by the identity), [n_Th][NRP][KP] zero padded.  A
// group is 16 columns with the same Theta_i (one MFMA B operand): column m of the
// n_th n_ph n_Ph columns of node i lies at (m / n_Ph) plane + i n_Ph + m % n_Ph,
// so 16 lanes read runs of min(n_Ph, 16) contiguous doubles.  Groups are ordered
// with i slowest, and a wavefront reloads B_i only when i changes.  It reads all
// rows of its columns before it writes them.

template <int KS>
__global__ __launch_bounds__(CB) void k_radial_implicit(KDims d, const double* __restrict__ Bimp, int KP,
                                                        double* F) {
  constexpr int NRT = (KS + 3) / 4;
  constexpr int NWV = CB / 64;
  const int lane = threadIdx.x & 63;
  const int wave = wave_uniform(threadIdx.x >> 6);
  const int lr = lane & 15, lk = lane >> 4;
  const int Q = int(d.M / d.n_Th) >> 4;  // 16-column groups per (eps, Theta_i)
  const int per_i = Q * d.n_eps;
  const int ngroups = per_i * d.n_Th;
  const int per_blk = ((ngroups + int(gridDim.x) - 1) / int(gridDim.x) + NWV - 1) / NWV * NWV;
  const int gend = min(ngroups, per_blk * (int(blockIdx.x) + 1));
  const int64_t M = d.M;
  const int n_r = d.n_r;
  const int sh_Ph = __builtin_ctz(d.n_Ph);
  const int NRP = 16 * NRT;
  double a[NRT][KS];
  int cur = -1;
  for (int g = per_blk * int(blockIdx.x) + wave; g < gend; g += NWV) {
    const int i = g / per_i;
    const int rem = g - i * per_i;
    const int e = rem / Q;
    const int q = rem - e * Q;
    if (i != cur) {
      const double* Bi = Bimp + int64_t(i) * NRP * KP;
#pragma unroll
      for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
        for (int s = 0; s < KS; ++s) a[rt][s] = Bi[(16 * rt + lr) * KP + 4 * s + lk];
      cur = i;
    }
    const uint32_t m = uint32_t(q * 16 + lr);
    const uint32_t col = (m >> sh_Ph) * uint32_t(d.plane) + uint32_t(i << sh_Ph) + (m & uint32_t(d.n_Ph - 1));
    const uint32_t boff = (uint32_t(lk) * uint32_t(M) + col) * 8u;
    auto at = [&](double* row) { return reinterpret_cast<double*>(reinterpret_cast<char*>(row) + boff); };
    double* Fg = F + int64_t(e) * n_r * M;
    double b[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      double* row = Fg + int64_t(4 * s) * M;
      if (s < KS - 1)
        b[s] = *at(row);
      else
        b[s] = 4 * s + lk < n_r ? *at(row) : 0.0;
    }
    v4d acc[NRT];
#pragma unroll
    for (int rt = 0; rt < NRT; ++rt) {
      acc[rt] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < KS; ++s) acc[rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rt][s], b[s], acc[rt], 0, 0, 0);
    }
#pragma unroll
    for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        if (rt < NRT - 1 || 16 * rt + lk + 4 * v < n_r) *at(Fg + int64_t(16 * rt + 4 * v) * M) = acc[rt][v];
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
  eo_pairs<L, L / 2, false>(line_tab<L>(LT_FILTER), 0, v, [&](int k, double z) { F[base + k * stride] = z; });
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
  eo_pairs<L, NTH, false>(line_tab<L>(LT_FILTER), 0, v, [&](int q, double z) {
    const int64_t a = (q < NTH) ? ba + q * rowstride : bb + (L - 1 - q) * rowstride;
    F[a] = z;
  });
}

// ---------------------------------------------------------------------------
// theta and phi terms together.  One workgroup takes one (eps, r) slab restricted
// to a tile of CW in-plane columns that is closed under the DFS partner map
// c -> c' (Phi_m -> Phi_m + pi): with all n_theta x n_phi values of each of its
// columns, every phi line and every theta DFS line of the tile lies inside it.
// The tile is staged once in LDS; half of the threads take the phi lines (one
// theta row and column each), the other half the theta DFS lines (one phi index
// below n_phi / 2 and column each, partner column c' at phi + pi).  Both lines
// have length n_phi = 2 n_theta.  The theta results go back through LDS to the
// phi threads, which add their own and store T: the state is read once and T
// written once.
//
// Tile columns: with R = min(CW / 2, n_Phi / 2), tile column col is in-plane
// column cbase + (col mod R) + [col & R] n_Phi / 2 + (col div 2R) n_Phi, and its
// partner is col ^ R.  For R < n_Phi / 2 a tile is two runs of R columns of one
// Theta row, m0 .. m0 + R - 1 and their partners; otherwise whole Theta rows.

// consecutive tiles of a fused theta-phi pass taken by one XCD (blocks b, b + 8,
// ... of one XCD): 16, measured against the tiles that share one 128-byte line
// of a column run (2 FP64, 4 FP32 on the 16 x 32 sphere; FP64 236.6 -> 223.8
// us, FP32 163.4 -> 148.0 us per launch on the 8-group workloads) and on the
// 32 x 64 sphere (below)
constexpr int XCD_TILE_GROUP = 16;

template <int NTH, int CW, typename TC>
struct SPC {
  static constexpr int NPH = 2 * NTH;
  static constexpr int L = NPH;                        // phi line = theta DFS line
  static constexpr int NL = NTH * CW;                  // phi lines = theta lines
  static constexpr int NTHR = 2 * NL < 64 ? 64 : 2 * NL;
  static constexpr int NE = NTH * NPH * CW;            // values per tile
  static constexpr int EPT = (NE + NTHR - 1) / NTHR;   // staged values per thread
  static_assert(NTHR % CW == 0, "a thread keeps its tile column while staging");
  static_assert(NE * sizeof(TC) <= 65536, "tile exceeds the LDS budget");
};

// TI: stored type of the input; TC: compute type and stored type of T
template <int NTH, int CW, typename TI, typename TC>
__global__ __launch_bounds__((SPC<NTH, CW, TC>::NTHR)) void k_sphere(KDims d, KTab t, const TI* __restrict__ Y,
                                                                   TC* __restrict__ T, double coef_sign,
                                                                   int mask_in, double in_scale, int ntiles) {
  using C = SPC<NTH, CW, TC>;
  constexpr int L = C::L, NPH = C::NPH;
  __shared__ __align__(16) TC sY[C::NE];
  // blocks b, b + 8, ..., b + 8 (G - 1) run on the same XCD and take G
  // consecutive tiles (those whose column runs share 128-byte lines among them)
  constexpr int G = XCD_TILE_GROUP;
  // (descending: block b takes the place of block gridDim - 1 - b; the grid is a
  // multiple of 8 G, so the XCD pairing is kept)
  const int b = d.rev ? int(gridDim.x) - 1 - int(blockIdx.x) : int(blockIdx.x);
  const int tile = (b / (8 * G)) * (8 * G) + (b % 8) * G + (b / 8) % G;
  if (tile >= ntiles) return;
  const int tpp = d.plane / CW;
  const int ej = tile / tpp, tl = tile - ej * tpp;
  const int j = ej % d.n_r;
  const int hP = d.n_Ph >> 1;
  const int R = min(CW / 2, hP);
  int cbase;
  if (R == hP) {
    cbase = tl * CW;
  } else {
    const int tpr = hP / R;
    cbase = (tl / tpr) * d.n_Ph + (tl % tpr) * R;
  }
  auto colc = [&](int col) { return cbase + (col & (R - 1)) + ((col & R) ? hP : 0) + (col / (2 * R)) * d.n_Ph; };
  const int64_t slab = int64_t(ej) * d.M;
  const int plane = d.plane;
  const int tid = int(threadIdx.x);

  // stage the tile: element e = combo * CW + col, combo = theta * n_phi + phi
  constexpr bool PAIRS = sizeof(TI) == 8 && sizeof(TC) == 8 && CW % 2 == 0 && C::NE % (2 * C::NTHR) == 0 &&
                         C::NTHR % (CW / 2) == 0;
  if constexpr (PAIRS) {
    // 16-byte loads of two neighbouring columns of one run (runs have an even
    // length R >= 2 and start at even columns, so the pair is contiguous and
    // 16-byte aligned in an aligned state)
    constexpr int PPT = C::NE / (2 * C::NTHR);
    const int q = tid % (CW / 2);
    const int c = colc(2 * q);
    TC s_in = TC(in_scale);
    if (mask_in && is_inflow(d, t, j, c / d.n_Ph)) s_in = TC(0);
    double2 v[PPT];
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      const int p = tid + i * C::NTHR;  // pair p = combo * CW / 2 + q
      v[i] = *reinterpret_cast<const double2*>(Y + (slab + int64_t(p / (CW / 2)) * plane + c));
    }
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      const int p = tid + i * C::NTHR;
      reinterpret_cast<double2*>(sY)[p] = double2{v[i].x * s_in, v[i].y * s_in};
    }
  } else {
    const int col = tid % CW;
    const int c = colc(col);
    TC s_in = TC(in_scale);
    if (mask_in && is_inflow(d, t, j, c / d.n_Ph)) s_in = TC(0);
    TI v[C::EPT];
#pragma unroll
    for (int i = 0; i < C::EPT; ++i) {
      const int e = tid + i * C::NTHR;
      v[i] = e < C::NE ? ld_stream<NT_SPH_LD>(Y + (slab + int64_t(e / CW) * plane + c)) : TI(0);
    }
#pragma unroll
    for (int i = 0; i < C::EPT; ++i) {
      const int e = tid + i * C::NTHR;
      if (e < C::NE) sY[e] = TC(v[i]) * s_in;
    }
  }
  __syncthreads();

  const bool isPhi = tid < C::NL;
  const bool active = tid < 2 * C::NL;
  const int u = isPhi ? tid : tid - C::NL;
  const int col = u % CW, w = u / CW;  // phi thread: w = theta row; theta thread: w = phi index < n_phi / 2
  const int colp = col ^ R;
  const int c = colc(col);
  const int iTh = c / d.n_Ph, m = c % d.n_Ph;
  const TC* tab = line_tab<L, TC>(LT_DERIV_T);
  TC z[L];
  if (active) {
    if (isPhi) {
      const TC s = TC(coef_sign * t.sin_Th[iTh] * t.sin_Ph[m] * t.inv_r[j] * t.inv_sin_th[w]);
      eo_pairs_stream2<L, L / 2, true, TC>(
          tab, 0, [&](int k) { return sY[(w * NPH + k) * CW + col]; },
          [&](int k) { return sY[(w * NPH + L - 1 - k) * CW + col]; }, [&](int k, TC zz) { z[k] = s * zz; });
    } else {
      // element q < n_theta: (theta_q, phi_w, c); element L - 1 - q: (theta_q,
      // phi_w + pi, c').  The partner coefficient is -s and the partner
      // derivative -z, so both halves take s z.
      const TC s = TC(coef_sign * t.sin_Th[iTh] * t.cos_Ph[m] * t.inv_r[j]);
      eo_pairs_stream2<L, L / 2, true, TC>(
          tab, 0, [&](int q) { return sY[(q * NPH + w) * CW + col]; },
          [&](int q) { return sY[(q * NPH + w + NTH) * CW + colp]; }, [&](int q, TC zz) { z[q] = s * zz; });
    }
  }
  __syncthreads();
  if (active && !isPhi) {
#pragma unroll
    for (int q = 0; q < NTH; ++q) {
      sY[(q * NPH + w) * CW + col] = z[q];
      sY[(q * NPH + w + NTH) * CW + colp] = z[L - 1 - q];
    }
  }
  __syncthreads();
  if (isPhi) {
    const int64_t o = slab + int64_t(w) * NPH * plane + c;
#pragma unroll
    for (int k = 0; k < NPH; ++k) st_stream<NT_SPH_ST>(T + (o + int64_t(k) * plane), TC(z[k] + sY[(w * NPH + k) * CW + col]));
  }
}

// ---------------------------------------------------------------------------
// theta and phi terms together on the 32 x 64 position sphere.  A tile of CW
// in-plane columns, closed under the DFS partner map (two runs of CW / 2 columns
// of one Theta row, the second at Phi + pi), holds all 32 x 64 = 2048 values of
// each column in LDS: FP64 tiles of 8 columns (132 KB, 148 KB with the
// operator: one workgroup per CU; two 32-byte runs, or one 64-byte run when the
// state and T are in the paired in-plane order), FP32 tiles of 16 (the mixed
// path, 32-byte runs).  Both line directions run as MFMA products (v_mfma_f64_16x16x4f64, or
// v_mfma_f32_16x16x4f32) on the even/odd halves of the 64-point operator:
//   theta: P = A E, Q = B O with E, O = Y(theta_j, phi_k, c) +- Y(theta_j,
//          phi_k + pi, c') (the DFS line of column c at phi_k and, reversed, its
//          partner), one GEMM column per line (k, c);
//   phi  : the same with E, O = Y(theta_l, phi_j, c) +- Y(theta_l, phi_63-j, c),
//          one GEMM column per line (theta_l, c).
// Outputs i and 63 - i of a line are P + Q and Q - P.  The A and B blocks of the
// operator (32 x 32 each) sit in LDS in the MFMA operand order: a wavefront
// takes both 16-row blocks for U / 2 16-line blocks, and reads the operand
// columns and its lines' points at each k-step (each point serving four
// products).  The theta results go through LDS to the phi results' owners, which
// add their own and store T from registers: the state is read once and T
// written once (16 bytes per point in FP64 instead of 40 for the two separate
// passes).

template <int CW, int NW_, typename TC>
struct S64 {
  static constexpr int NTH = 32, NPH = 64, L = 64;
  static constexpr int R = CW / 2;                     // run length (columns)
  static constexpr int NW = NW_;                       // wavefronts: NW / 2 theta, NW / 2 phi
  static constexpr int NTHR = 64 * NW;
  // 16-line blocks per wavefront: each direction has 2 CW blocks of 16 lines
  // times two 16-row blocks of the operator halves, over NW / 2 wavefronts
  static constexpr int U = 8 * CW / NW;
  // theta-row stride in LDS (elements): the row groups of one LDS access fall on
  // different banks
  static constexpr int RS = NPH * CW + 16;
  static constexpr int NE = NTH * NPH * CW;            // values per tile
  static constexpr int LDSN = NTH * RS;
  static constexpr int PPT = NE / (2 * NTHR);          // column pairs per thread
  static SP6_DEV int at(int th, int ph, int col) { return th * RS + ph * CW + col; }
  static_assert(NE % (2 * NTHR) == 0, "pairs divide evenly");
  static_assert(U * NW == 8 * CW, "line blocks divide evenly");
};

template <typename T>
struct Pair2;
template <>
struct Pair2<double> {
  using type = double2;
};
template <>
struct Pair2<float> {
  using type = float2;
};

// TI: stored type of the state read; TC: LDS, product and T type (FP64 path:
// double, double on v_mfma_f64_16x16x4f64; mixed path: double or float in, float
// on v_mfma_f32_16x16x4f32).
template <int CW, int NW, typename TI, typename TC>
__global__ __launch_bounds__(64 * NW) void k_sphere64(KDims d, KTab t, const TI* __restrict__ Y,
                                                      TC* __restrict__ T, double coef_sign, int mask_in,
                                                      double in_scale, int ntiles, int paired) {
  using C = S64<CW, NW, TC>;
  using TI2 = typename Pair2<TI>::type;
  using TC2 = typename Pair2<TC>::type;
  using VC = typename std::conditional<sizeof(TC) == 8, v4d, v4f>::type;
  constexpr bool F64 = sizeof(TC) == 8;
  constexpr int NTH = C::NTH, NPH = C::NPH, R = C::R, U = C::U;
  __shared__ __align__(16) TC sY[C::LDSN];
  // operator halves in the MFMA A-operand lane order: [A, B][row block][s][lane]
  __shared__ __align__(16) TC sTab[2 * 2 * 8 * 64];
  __shared__ double sIs[NTH];  // 1 / sin(theta_l)
  // blocks b, b + 8, ..., b + 8 (G - 1) (one XCD) take G consecutive tiles (1 KB
  // of each (theta, phi) plane of the state in the paired order, FP64 or FP32):
  // measured 6.10 -> 5.57 ms (FP64) and 3.38 -> 3.16 ms (FP32) per launch on
  // the paired order against G = 4, the tiles that share one 128-byte line of the
  // plain order (where wider groups made no difference)
  constexpr int G = XCD_TILE_GROUP;
  const int b = d.rev ? int(gridDim.x) - 1 - int(blockIdx.x) : int(blockIdx.x);
  const int tile = (b / (8 * G)) * (8 * G) + (b % 8) * G + (b / 8) % G;
  if (tile >= ntiles) return;
  const int tpp = d.plane / CW;
  const int ej = tile / tpp, tl = tile - ej * tpp;
  const int j = ej % d.n_r;
  const int hP = d.n_Ph >> 1;
  const int tpr = hP / R;
  const int rowb = (tl / tpr) * d.n_Ph, gR = (tl % tpr) * R;
  const int cbase = rowb + gR;
  // in-plane column of tile column col, and where it is stored: the same, or in
  // the paired order (groups of R columns) the tile's columns side by side
  auto colc = [&](int col) { return cbase + (col & (R - 1)) + ((col & R) ? hP : 0); };
  const int mbase = rowb + 2 * gR;
  auto colm = [&](int col) { return paired ? mbase + col : colc(col); };
  const int64_t slab = int64_t(ej) * d.M;
  const int plane = d.plane;
  const int tid = int(threadIdx.x);
  const int lane = tid & 63;
  const int wave = wave_uniform(tid >> 6);

  // stage the tile with loads of two neighbouring columns of a run per lane
  {
    const int q = tid % (CW / 2);
    const int c = colc(2 * q), cm = colm(2 * q);
    double s_in = in_scale;
    if (mask_in && is_inflow(d, t, j, c / d.n_Ph)) s_in = 0.0;
    TI2 v[C::PPT];
#pragma unroll
    for (int i = 0; i < C::PPT; ++i) {
      const int p = tid + i * C::NTHR;  // pair p = combo * CW / 2 + q, combo = theta * 64 + phi
      v[i] = *reinterpret_cast<const TI2*>(Y + (slab + int64_t(p / (CW / 2)) * plane + cm));
    }
#pragma unroll
    for (int i = 0; i < C::PPT; ++i) {
      const int p = tid + i * C::NTHR;
      const int combo = p / (CW / 2);
      TC2 w;
      if constexpr (F64) {
        w.x = v[i].x * s_in;
        w.y = v[i].y * s_in;
      } else {
        w.x = TC(v[i].x);
        w.y = TC(v[i].y);
      }
      *reinterpret_cast<TC2*>(&sY[C::at(combo / NPH, combo % NPH, 2 * q)]) = w;
    }
  }
  {
    const TC* tab = line_tab<64, TC>(LT_DERIV);
#pragma unroll
    for (int r = 0; r < (2 * 2 * 8 * 64 + C::NTHR - 1) / C::NTHR; ++r) {
      const int e = tid + r * C::NTHR;
      if (e < 2 * 2 * 8 * 64) {
        const int ab = e >> 10, rb = (e >> 9) & 1, s = (e >> 6) & 7, l = e & 63;
        sTab[e] = tab[ab * 32 * 32 + (rb * 16 + (l & 15)) * 32 + 4 * s + (l >> 4)];
      }
    }
    if (tid < NTH) sIs[tid] = t.inv_sin_th[tid];
  }
  const bool isTh = wave < NW / 2;
  // a wavefront takes both 16-row blocks of the operator halves for U / 2 line
  // blocks: each staged point it reads serves four products
  const int ng = isTh ? wave : wave - NW / 2;
  constexpr int UH = U / 2;
  const int lr = lane & 15, lk = lane >> 4;
  double sc0;
  {
    const int c = colc(lr % CW);
    sc0 = coef_sign * t.sin_Th[c / d.n_Ph] * (isTh ? t.cos_Ph[c % d.n_Ph] : t.sin_Ph[c % d.n_Ph]) * t.inv_r[j];
    if constexpr (!F64) sc0 *= in_scale;  // FP32 tiles are staged unscaled
  }
  __syncthreads();

  VC accP[2][UH], accQ[2][UH];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int u = 0; u < UH; ++u) accP[h][u] = accQ[h][u] = VC{0, 0, 0, 0};
  auto mfma = [](TC a, TC x, VC c) {
    if constexpr (F64)
      return __builtin_amdgcn_mfma_f64_16x16x4f64(a, x, c, 0, 0, 0);
    else
      return __builtin_amdgcn_mfma_f32_16x16x4f32(a, x, c, 0, 0, 0);
  };
  auto products = [&](auto dir) {
    constexpr bool TH = decltype(dir)::value;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int jj = 4 * s + lk;
      TC a0[2], b0[2], x[UH], y[UH];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        a0[h] = sTab[(h * 8 + s) * 64 + lane];
        b0[h] = sTab[((2 + h) * 8 + s) * 64 + lane];
      }
#pragma unroll
      for (int u = 0; u < UH; ++u) {
        const int n = (ng * UH + u) * 16 + lr;
        const int a = n / CW, col = n % CW;
        if constexpr (TH) {
          x[u] = sY[C::at(jj, a, col)];
          y[u] = sY[C::at(jj, a + NTH, col ^ R)];
        } else {
          x[u] = sY[C::at(a, jj, col)];
          y[u] = sY[C::at(a, NPH - 1 - jj, col)];
        }
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < UH; ++u) {
        const TC e = x[u] + y[u], o = x[u] - y[u];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          accP[h][u] = mfma(a0[h], e, accP[h][u]);
          accQ[h][u] = mfma(b0[h], o, accQ[h][u]);
        }
      }
    }
  };
  if (isTh)
    products(std::true_type{});
  else
    products(std::false_type{});
  __syncthreads();  // every read of the staged tile is done
  // C layout: register v holds row lk + 4 v (FP64 product) or 4 lk + v (FP32)
  auto crow = [&](int h, int v) { return h * 16 + (F64 ? lk + 4 * v : 4 * lk + v); };
  if (isTh) {
    const TC sc = TC(sc0);
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int u = 0; u < UH; ++u) {
        const int n = (ng * UH + u) * 16 + lr;
        const int k = n / CW, col = n % CW;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = crow(h, v);
          sY[C::at(i, k, col)] = sc * (accP[h][u][v] + accQ[h][u][v]);
          sY[C::at(i, k + NTH, col ^ R)] = sc * (accQ[h][u][v] - accP[h][u][v]);
        }
      }
  }
  __syncthreads();
  if (!isTh) {
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int u = 0; u < UH; ++u) {
        const int n = (ng * UH + u) * 16 + lr;
        const int l = n / CW, col = n % CW;
        const TC sc = TC(sc0 * sIs[l]);
        const int64_t ob = slab + int64_t(l) * NPH * plane + colm(col);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = crow(h, v);
          T[ob + int64_t(i) * plane] = sY[C::at(l, i, col)] + sc * (accP[h][u][v] + accQ[h][u][v]);
          T[ob + int64_t(NPH - 1 - i) * plane] = sY[C::at(l, NPH - 1 - i, col)] + sc * (accQ[h][u][v] - accP[h][u][v]);
        }
      }
  }
}

unsigned grid_for(int64_t threads) { return unsigned((threads + CB - 1) / CB); }

template <int L, typename TI, typename TO>
void launch_phi_t(const KDims& d, const KTab& t, const void* Y, void* T, bool accum, double coef_sign,
                  bool mask_in, double in_scale, hipStream_t s) {
  const unsigned g = grid_for(int64_t(d.n_eps) * d.n_r * d.n_th * d.plane);
  const TI* y = static_cast<const TI*>(Y);
  TO* o = static_cast<TO*>(T);
  if (accum)
    k_phi<L, true, TI, TO><<<g, CB, 0, s>>>(d, t, y, o, coef_sign, mask_in, in_scale);
  else
    k_phi<L, false, TI, TO><<<g, CB, 0, s>>>(d, t, y, o, coef_sign, mask_in, in_scale);
}

template <int NTH, typename TI, typename TO>
void launch_theta_t(const KDims& d, const KTab& t, const void* Y, void* T, bool accum, double coef_sign,
                    bool mask_in, double in_scale, hipStream_t s) {
  const unsigned g = grid_for(int64_t(d.n_eps) * d.n_r * (d.n_ph / 2) * d.plane);
  const TI* y = static_cast<const TI*>(Y);
  TO* o = static_cast<TO*>(T);
  if (accum)
    k_theta<NTH, true, TI, TO><<<g, CB, 0, s>>>(d, t, y, o, coef_sign, mask_in, in_scale);
  else
    k_theta<NTH, false, TI, TO><<<g, CB, 0, s>>>(d, t, y, o, coef_sign, mask_in, in_scale);
}

template <typename TI, typename TO>
hipError_t launch_phi_p(const KDims& d, const KTab& t, const void* Y, void* T, bool accum, double coef_sign,
                        bool mask_in, double in_scale, hipStream_t s) {
  switch (d.n_ph) {
#define CASE(N) \
  case N: launch_phi_t<N, TI, TO>(d, t, Y, T, accum, coef_sign, mask_in, in_scale, s); break;
    CASE(4) CASE(8) CASE(16) CASE(32) CASE(64)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename TI, typename TO>
hipError_t launch_theta_p(const KDims& d, const KTab& t, const void* Y, void* T, bool accum, double coef_sign,
                          bool mask_in, double in_scale, hipStream_t s) {
  switch (d.n_th) {
#define CASE(N) \
  case N: launch_theta_t<N, TI, TO>(d, t, Y, T, accum, coef_sign, mask_in, in_scale, s); break;
    CASE(2) CASE(4) CASE(8) CASE(16) CASE(32)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int KS, bool ACCUM>
void launch_radial_t(const KDims& d, const KTab& t, const double* Y, double* T, bool transpose, bool mask_in,
                     double in_scale, hipStream_t s) {
  const int64_t ngroups = (d.M / 16) * d.n_eps;
  // one resident round of workgroups, advancing through the column groups together
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_radial<KS, ACCUM>, CB, 0) != hipSuccess || per_cu < 1)
    per_cu = 1;
  int64_t blocks = (ngroups + 3) / 4;
  const int64_t cap = int64_t(d.ncu) * per_cu;
  if (blocks > cap) blocks = cap;
  k_radial<KS, ACCUM><<<unsigned(blocks), CB, 0, s>>>(d, t, Y, T, transpose, mask_in, in_scale);
}

// tile width: 16 columns on both paths (FP32 tiles read 32-byte runs, four
// tiles per 128-byte line; measured faster than 32-column FP32 tiles)
int sphere_cw(const KDims& d) {
  if (d.n_ph != 2 * d.n_th || d.n_th > 16) return 0;
  return d.plane < 16 ? d.plane : 16;
}

// the 32 x 64 sphere: tiles of 8 (FP64) or 16 (FP32) columns, two runs within one
// Theta row (n_Phi >= 16)
bool sphere64_ok(const KDims& d) { return d.n_th == 32 && d.n_ph == 64 && d.n_Ph >= 16; }

template <int CW, int NW, typename TI, typename TC>
hipError_t launch_sphere64_t(const KDims& d, const KTab& t, const TI* Y, TC* T, double coef_sign, bool mask_in,
                             double in_scale, hipStream_t s, bool paired = false) {
  // the paired order of a buffer groups runs of R = CW / 2 columns: 4 for the FP64
  // state (CW = 8), 8 for the FP32 stage copy (CW = 16); an FP64 state read by
  // FP32 tiles is the caller's state, in the plain order
  if (paired && (CW / 2 != (sizeof(TI) == 8 ? 4 : 8) || sizeof(TC) != sizeof(TI))) return hipErrorInvalidValue;
  const int64_t ntiles = int64_t(d.n_eps) * d.n_r * (d.plane / CW);
  constexpr int64_t GB = 8 * XCD_TILE_GROUP;
  const int64_t nb = (ntiles + GB - 1) / GB * GB;
  if (nb > INT32_MAX) return hipErrorInvalidValue;
  k_sphere64<CW, NW, TI, TC><<<unsigned(nb), 64 * NW, 0, s>>>(d, t, Y, T, coef_sign, mask_in, in_scale, int(ntiles),
                                                              int(paired));
  return hipGetLastError();
}

hipError_t launch_sphere64(const KDims& d, const KTab& t, const double* Y, double* T, double coef_sign, bool mask_in,
                           double in_scale, hipStream_t s, bool paired) {
  return launch_sphere64_t<8, 16>(d, t, Y, T, coef_sign, mask_in, in_scale, s, paired);
}

// FP32 tiles of 16 columns (32-byte runs of an FP32 row, 133 KB of LDS): 3.89 ms
// per launch on the 4-group large grid, against 3.95 for 8-column tiles (16-byte
// runs, two workgroups per CU) and 4.44 for the separate theta and phi passes
hipError_t launch_sphere64_mixed(const KDims& d, const KTab& t, const void* Y, bool y_f32, float* T, hipStream_t s,
                                 bool paired) {
  return y_f32 ? launch_sphere64_t<16, 16>(d, t, static_cast<const float*>(Y), T, 1.0, false, 1.0, s, paired)
               : launch_sphere64_t<16, 16>(d, t, static_cast<const double*>(Y), T, 1.0, false, 1.0, s, paired);
}

template <int NTH, int CW, typename TI, typename TC>
hipError_t launch_sphere_t(const KDims& d, const KTab& t, const void* Y, void* T, double coef_sign, bool mask_in,
                           double in_scale, hipStream_t s) {
  const int64_t ntiles = int64_t(d.n_eps) * d.n_r * (d.plane / CW);
  constexpr int64_t GB = 8 * XCD_TILE_GROUP;
  const int64_t nb = (ntiles + GB - 1) / GB * GB;
  if (nb > INT32_MAX) return hipErrorInvalidValue;
  k_sphere<NTH, CW, TI, TC><<<unsigned(nb), SPC<NTH, CW, TC>::NTHR, 0, s>>>(
      d, t, static_cast<const TI*>(Y), static_cast<TC*>(T), coef_sign, mask_in, in_scale, int(ntiles));
  return hipGetLastError();
}

template <int CW, typename TI, typename TC>
hipError_t launch_sphere_n(const KDims& d, const KTab& t, const void* Y, void* T, double coef_sign, bool mask_in,
                           double in_scale, hipStream_t s) {
  switch (d.n_th) {
#define CASE(N) \
  case N: return launch_sphere_t<N, CW, TI, TC>(d, t, Y, T, coef_sign, mask_in, in_scale, s);
    CASE(2) CASE(4) CASE(8) CASE(16)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_phi(const KDims& d, const KTab& t, const double* Y, double* T, bool accum,
                      double coef_sign, bool mask_in, double in_scale, hipStream_t s) {
  return launch_phi_p<double, double>(d, t, Y, T, accum, coef_sign, mask_in, in_scale, s);
}

hipError_t launch_theta(const KDims& d, const KTab& t, const double* Y, double* T, bool accum,
                        double coef_sign, bool mask_in, double in_scale, hipStream_t s) {
  return launch_theta_p<double, double>(d, t, Y, T, accum, coef_sign, mask_in, in_scale, s);
}

hipError_t launch_phi_mixed(const KDims& d, const KTab& t, const void* Y, bool y_f32, float* T, bool accum,
                            hipStream_t s) {
  return y_f32 ? launch_phi_p<float, float>(d, t, Y, T, accum, 1.0, false, 1.0, s)
               : launch_phi_p<double, float>(d, t, Y, T, accum, 1.0, false, 1.0, s);
}

hipError_t launch_theta_mixed(const KDims& d, const KTab& t, const void* Y, bool y_f32, float* T, bool accum,
                              hipStream_t s) {
  return y_f32 ? launch_theta_p<float, float>(d, t, Y, T, accum, 1.0, false, 1.0, s)
               : launch_theta_p<double, float>(d, t, Y, T, accum, 1.0, false, 1.0, s);
}

bool sphere_fusable(const KDims& d, bool mixed) { return sphere_cw(d) > 0 || sphere64_ok(d); }

bool paired_order_ok(const KDims& d) { return sphere64_ok(d); }

hipError_t launch_sphere(const KDims& d, const KTab& t, const double* Y, double* T, double coef_sign,
                         bool mask_in, double in_scale, hipStream_t s, bool paired) {
  if (sphere64_ok(d)) return launch_sphere64(d, t, Y, T, coef_sign, mask_in, in_scale, s, paired);
  if (paired) return hipErrorInvalidValue;
  switch (sphere_cw(d)) {
    case 8: return launch_sphere_n<8, double, double>(d, t, Y, T, coef_sign, mask_in, in_scale, s);
    case 16: return launch_sphere_n<16, double, double>(d, t, Y, T, coef_sign, mask_in, in_scale, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_sphere_mixed(const KDims& d, const KTab& t, const void* Y, bool y_f32, float* T,
                               hipStream_t s, bool paired) {
  if (sphere64_ok(d)) return launch_sphere64_mixed(d, t, Y, y_f32, T, s, paired);
  if (paired) return hipErrorInvalidValue;
  switch (sphere_cw(d)) {
    case 8:
      return y_f32 ? launch_sphere_n<8, float, float>(d, t, Y, T, 1.0, false, 1.0, s)
                   : launch_sphere_n<8, double, float>(d, t, Y, T, 1.0, false, 1.0, s);
    case 16:
      return y_f32 ? launch_sphere_n<16, float, float>(d, t, Y, T, 1.0, false, 1.0, s)
                   : launch_sphere_n<16, double, float>(d, t, Y, T, 1.0, false, 1.0, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_radial(const KDims& d, const KTab& t, const double* Y, double* T, bool accum,
                         bool transpose, bool mask_in, double in_scale, hipStream_t s) {
  const int KS = t.KP / 4;
  switch (KS) {
#define CASE(N)                                                                  \
  case N:                                                                        \
    if (accum)                                                                   \
      launch_radial_t<N, true>(d, t, Y, T, transpose, mask_in, in_scale, s);     \
    else                                                                         \
      launch_radial_t<N, false>(d, t, Y, T, transpose, mask_in, in_scale, s);    \
    break;
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10)
    CASE(11) CASE(12) CASE(13) CASE(14) CASE(15) CASE(16) CASE(17) CASE(18) CASE(19) CASE(20)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_filter_radial(const KDims& d, const KTab& t, double* F, bool transpose, hipStream_t s) {
  const int64_t ngroups = (d.M / 16) * d.n_eps;
  int64_t blocks = (ngroups + 3) / 4;
  const int64_t cap = int64_t(d.ncu) * 8;
  if (blocks > cap) blocks = cap;
  switch (t.KP / 4) {
#define CASE(N) \
  case N: k_radial_filter<N><<<unsigned(blocks), CB, 0, s>>>(d, t, F, transpose ? 1 : 0); break;
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9) CASE(10)
    CASE(11) CASE(12) CASE(13) CASE(14) CASE(15) CASE(16) CASE(17) CASE(18) CASE(19) CASE(20)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_radial_implicit(const KDims& d, const KTab& t, const double* Bimp, double* F, hipStream_t s) {
  if ((d.M / d.n_Th) % 16 != 0) return hipErrorInvalidValue;
  const int64_t ngroups = (d.M / 16) * d.n_eps;
  int64_t blocks = (ngroups + 3) / 4;
  const int64_t cap = int64_t(d.ncu) * 8;
  if (blocks > cap) blocks = cap;
  switch (t.KP / 4) {
#define CASE(N) \
  case N: k_radial_implicit<N><<<unsigned(blocks), CB, 0, s>>>(d, Bimp, t.KP, F); break;
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

hipError_t init_line_tables_columns(const double* tab) {
  hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_lines), tab, sizeof(double) * LINE_TAB_KINDS * LINE_TAB_SIZE, 0, hipMemcpyHostToDevice);
  if (e != hipSuccess) return e;
  static float f[LINE_TAB_KINDS * LINE_TAB_SIZE];
  for (int i = 0; i < LINE_TAB_KINDS * LINE_TAB_SIZE; ++i) f[i] = float(tab[i]);
  return hipMemcpyToSymbol(HIP_SYMBOL(c_lines_f), f, sizeof f, 0, hipMemcpyHostToDevice);
}
