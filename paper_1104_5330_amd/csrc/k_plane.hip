// Plane passes: everything that needs a whole (Theta, Phi) plane.
//
// A workgroup stages NPW planes in LDS.  The lines have length L = 2 n_Theta =
// n_Phi: a Theta DFS line (column Phi_m followed by the reversed column
// Phi_m + pi, since the direction (-Theta, Phi) is (Theta, Phi + pi)) or a Phi
// row.  On 16 x 32 planes the even and odd halves of both line operators run as
// 16 x 16 x 16 MFMA products (one direction of one plane per wavefront); on the
// other plane shapes each lane owns one line and the wavefronts split its
// output pairs.  Forward (Eq. Liouvsph): Theta term -(sin Theta / r) dF/dTheta, Phi term
// -(sin Theta sin Phi cos theta / (r sin theta)) dF/dPhi.  The epilogue adds the
// r/theta/phi terms produced by the column passes, the collision term
// eta - (kappa + sigma) F + sigma <F> (Eq. Transp with an isotropic kernel,
// <F> with Fejer weights in cos Theta), the inflow mask (Sect. 4.2) and the RK4
// stage update, all in FP64.
#include <type_traits>

#include "k_common.h"

namespace {

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

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <int NT>
struct PC {
  static constexpr int L = 2 * NT;        // line length (Theta DFS line, Phi row)
  static constexpr int NF = 2 * NT;       // n_Phi
  static constexpr int PLANE = NT * NF;
  static constexpr int LPP = 2 * NT;      // lines per plane
  static constexpr int NPW = 64 / LPP;    // planes per workgroup
  // wavefronts, each computing PPW output pairs of every line (eight for the
  // 2048-point planes: half the registers per thread of four)
  static constexpr int NW = NT >= 32 ? 8 : (NT >= 4 ? 4 : NT);
  static constexpr int PPW = NT / NW;
  static constexpr int PTS = NPW * PLANE;  // points per workgroup (64 NT)
  static constexpr int NTHR = 64 * NW;
  static constexpr int PPT = PTS / NTHR;   // points per thread in coalesced phases
  // LDS layout: rows padded by one double so that row-wise (Phi) and column-wise
  // (Theta) line reads both spread over the banks
  static constexpr int RS = NF + 1;
  static constexpr int PS = NT * RS;
  static constexpr int PTSP = NPW * PS;
  static SP6_DEV int lds(int p) {
    const int pl = p / PLANE, r = p % PLANE;
    return pl * PS + (r / NF) * RS + (r % NF);
  }
  // plane row (Theta index) of the point tid + q NTHR a thread stages: when the
  // workgroup covers whole rows and a plane is a whole number of workgroup rounds,
  // tid / NF plus a constant per q (one base address with immediate offsets for
  // the row tables instead of one address per point)
  static SP6_DEV int row_of(int tid, int q) {
    if constexpr (NTHR % NF == 0 && PLANE % NTHR == 0)
      return tid / NF + (q * (NTHR / NF)) % NT;
    else
      return ((tid + q * NTHR) % PLANE) / NF;
  }
};

struct PlaneIdx {
  int e, j, l, k;
};

SP6_DEV PlaneIdx plane_index(const KDims& d, int64_t pid) {
  PlaneIdx p;
  p.k = int(pid % d.n_ph);
  int64_t q = pid / d.n_ph;
  p.l = int(q % d.n_th);
  q /= d.n_th;
  p.j = int(q % d.n_r);
  p.e = int(q / d.n_r);
  return p;
}

// LDS index of element q of a lane's line
template <int NT>
struct LineMap {
  int b1, s1, b2, s2;
  SP6_DEV int idx(int q) const { return q < NT ? b1 + q * s1 : b2 + (2 * NT - 1 - q) * s2; }
};

template <int NT>
SP6_DEV LineMap<NT> line_map(int pl, int li) {
  using C = PC<NT>;
  LineMap<NT> m;
  if (li < NT) {  // Theta DFS line for Phi column li and its partner li + NT
    m.b1 = pl * C::PS + li;
    m.s1 = C::RS;
    m.b2 = pl * C::PS + li + NT;
    m.s2 = C::RS;
  } else {  // Phi row i = li - NT
    const int i = li - NT;
    m.b1 = pl * C::PS + i * C::RS;
    m.s1 = 1;
    m.b2 = pl * C::PS + i * C::RS + (C::L - 1);
    m.s2 = -1;
  }
  return m;
}

// Forward coefficient of line element q (including the DFS partner sign for the
// Theta line: the partner derivative is -z).
template <int NT>
SP6_DEV double line_coef(bool isTh, int q, int li, double inv_r, double cot_th, const double* sTh,
                         const double* sPh) {
  if (isTh) {
    const int iTh = q < NT ? q : 2 * NT - 1 - q;
    const double sg = q < NT ? -1.0 : 1.0;
    return sg * sTh[iTh] * inv_r;
  }
  const int i = li - NT;
  return -sTh[i] * sPh[q] * cot_th * inv_r;
}

// ---------------------------------------------------------------------------
// anisotropic scattering, p(mu) = c0 + c1 mu + c2 mu^2.  K F needs ten angular
// moments of the plane: (sum w F, sum w omega F, sum w omega omega F) with
// omega = (cos Theta, sin Theta cos Phi, sin Theta sin Phi), tensor components
// ordered xx, yy, zz, xy, xz, yz.  A Phi row contributes through its Fourier sums
// S0, C1, S1, C2, S2 (of F, cos Phi F, sin Phi F, cos 2Phi F, sin 2Phi F) with the
// row weight wr.

constexpr int NMOM = 10;

SP6_DEV void row_moments(double wr, double cT, double sT, double S0, double C1, double S1, double C2, double S2,
                         double* m) {
  m[0] = wr * S0;
  m[1] = wr * cT * S0;
  m[2] = wr * sT * C1;
  m[3] = wr * sT * S1;
  m[4] = wr * cT * cT * S0;
  m[5] = 0.5 * wr * sT * sT * (S0 + C2);
  m[6] = 0.5 * wr * sT * sT * (S0 - C2);
  m[7] = wr * cT * sT * C1;
  m[8] = wr * cT * sT * S1;
  m[9] = 0.5 * wr * sT * sT * S2;
}

// Fourier sums of one Phi row read through ld(q), q = m
template <int NF, typename Load>
SP6_DEV void row_fourier(const double* cP, const double* sP, Load&& ld, double& S0, double& C1, double& S1, double& C2,
                         double& S2) {
  S0 = C1 = S1 = C2 = S2 = 0.0;
#pragma unroll 4
  for (int q = 0; q < NF; ++q) {
    const double v = ld(q), c = cP[q], sn = sP[q];
    S0 += v;
    C1 += c * v;
    S1 += sn * v;
    C2 += (c * c - sn * sn) * v;
    S2 += 2.0 * sn * c * v;
  }
}

// c0 m0 + c1 omega . J + c2 omega . M . omega
SP6_DEV double phase_contract(const KCoef& cf, const double* m, double ox, double oy, double oz) {
  const double dJ = ox * m[1] + oy * m[2] + oz * m[3];
  const double dM = ox * ox * m[4] + oy * oy * m[5] + oz * oz * m[6] +
                    2.0 * (ox * oy * m[7] + ox * oz * m[8] + oy * oz * m[9]);
  return cf.pc0 * m[0] + cf.pc1 * dJ + cf.pc2 * dM;
}

// sum over omega of u(omega) (K Y)(omega) from the unweighted moments U of u and
// the weighted moments M of Y: c0 M0 U0 + c1 J.U1 + c2 M:U2
SP6_DEV double phase_pair(const KCoef& cf, const double* M, const double* U) {
  const double dJ = M[1] * U[1] + M[2] * U[2] + M[3] * U[3];
  const double dM = M[4] * U[4] + M[5] * U[5] + M[6] * U[6] + 2.0 * (M[7] * U[7] + M[8] * U[8] + M[9] * U[9]);
  return cf.pc0 * M[0] * U[0] + cf.pc1 * dJ + cf.pc2 * dM;
}

// sum of v over N consecutive lanes aligned to N (the NT Phi-row lanes of a plane,
// or all 2 NT lanes of a plane)
template <int N>
SP6_DEV double plane_rows_sum(double v) {
#pragma unroll
  for (int off = 1; off < N; off <<= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// ---------------------------------------------------------------------------
// forward: L F (partial), right-hand side, or one RK4 stage.
// Persistent workgroups walk over groups of NPW planes; while the lines and the
// epilogue of one group are computed, the global loads of the next group are in
// flight (register double buffering).

struct PlaneInfo {
  double inv_r, cot_th, kappa, sigma, eta, mean;
  int j, pad;
};

// TY: stored type of the stage input, TO: stored type of T and of the next stage
// input, TC: type of the line derivatives.  The collision term, the inflow mask
// and the RK update are FP64 in every instantiation.
// AN: anisotropic scattering (plane moments instead of the angular mean).
// FP64 on 16 x 32 planes, lines on MFMA: stage 1 (no accumulator or y
// operands) at four waves per SIMD (128 VGPRs, no spills; five spill), stages
// 2, 3 and 4 at three (168 VGPRs: at four they spill and the pass went from 485
// to 526 us; at two they are no faster).  With the lines streamed from LDS the
// best caps had been five for stage 1 and four for the others.  The anisotropic FP64 pass (ten
// plane moments) at three waves per SIMD: 694 -> 625 us (four: no gain).  The
// mixed pass is as fast at one to four.  2048-point planes (eight
// wavefronts per workgroup): 128 VGPRs, so that two workgroups share a CU.
constexpr int plane_waves_per_eu(int nt, bool na, int ym, bool an, int tc_bytes) {
  if (nt == 32) return 4;
  if (nt == 16 && an && tc_bytes == 8) return 3;
  if (!(!an && tc_bytes == 8 && nt == 16)) return 1;
  if (!na) return ym == 0 ? 4 : (ym == 1 ? 1 : 3);
  return 3;
}
// YM: 0 the next stage input is based on Yin; 1 on a.ysrc; 2 on a.ysrc, and the
// accumulator's base is recovered from Yin and a.ysrc (FP64 RK4 stage 2, where
// Yin = F + dt/2 k1 and ysrc = F give F + dt/6 k1 = ysrc + (Yin - ysrc) / 3, so
// stage 1 need not write the accumulator); 4 on the accumulator source itself
// (Adams-Bashforth, whose history H is both: loaded once)
// PM: the paired in-plane order (StageArgs::pair_mode).  With PM 2 and 3 a
// thread's points are paired positions: it reads the stage state, T and the
// accumulator source and writes the paired outputs at them, stages its values in
// LDS at their columns' plain places, and reads y (PM 2) or writes the
// accumulator destination (PM 3) in the plain order at a lane offset, or at its
// points too when a.pair_all says they are paired as well; with PM 1 its points
// are plain and only ynext is written at the paired position.  On the mixed path
// (FP32 T and ynext: groups of eight columns) the FP64 accumulator stays in the
// plain order and is read and written at the same lane offset as y.
template <int NT, bool NA, int YM, typename TY, typename TO, typename TC, bool AN, int PM = 0>
__global__ __launch_bounds__(PC<NT>::NTHR) __attribute__((amdgpu_waves_per_eu(plane_waves_per_eu(NT, NA, YM, AN, sizeof(TC))))) void k_plane(KDims d, KTab t, KCoef cf, StageArgs a, int ngroups) {
  using C = PC<NT>;
  constexpr bool MIX = sizeof(TO) == 4;   // mixed path
  constexpr int PG = MIX ? 8 : 4;         // paired-order group (paired_order.h)
  static_assert(PM == 0 || (C::NF >= 2 * PG && C::NTHR % C::NF == 0 && (MIX || sizeof(TY) == 8)),
                "the paired order: n_Phi / 2 a multiple of the group, the points tid + q NTHR of a thread share a column");
  constexpr bool NY = YM == 1 || YM == 2, YR = YM == 2, YA = YM == 4;
  static_assert(!YR || !NA, "the accumulator base is either loaded or recovered");
  static_assert(!YA || NA, "y is the loaded accumulator");
  __shared__ TY sY[C::PTSP];
  __shared__ TC sR[2][C::PTSP];
  __shared__ double sTh[NT], sPh[C::NF], sCP[C::NF], sCT[NT], sWm[NT];
  __shared__ PlaneInfo sPl[C::NPW];
  // isotropic in-scattering on 16 x 32 and 32 x 64 planes: the angular mean is
  // summed from the values each thread stages (row weight times value), reduced
  // over the wavefront and then over the wavefronts in a fixed order, instead of
  // by one wavefront over the staged rows (which held a per-lane address for every
  // row element and spilled registers on the 2048-point planes)
  constexpr bool MEAN_STAGED = NT >= 16 && !AN;
  __shared__ double sMean[MEAN_STAGED ? C::NW : 1][C::NPW];
  __shared__ double sMo[AN ? C::NPW : 1][NMOM];
  __shared__ double sInvR[SP6_MAX_NR], sCot[32];

  const int tid = threadIdx.x;
  const int npl = int(d.nplanes);
  // Lines on 16 x 32 planes: the even and odd halves of the Theta and Phi line
  // operators as 16 x 16 x 16 products on v_mfma_f64_16x16x4f64 (FP64 path) or
  // v_mfma_f32_16x16x4f32 (mixed path), wavefront w taking direction w mod 2 of
  // plane w div 2, with the transposed even (first) and odd (second) blocks of
  // the table staged in LDS.  Each staged value is read from LDS twice per point
  // instead of eight times (FP64 RK4 step 2 % faster, mixed 1 %).
  constexpr bool MFL = NT == 16 && C::NW == 4 && C::NPW == 2 &&
                       ((sizeof(TY) == 8 && sizeof(TC) == 8) || sizeof(TC) == 4);
  // 32 x 64 planes (one plane per workgroup, eight wavefronts): the same products
  // with wavefront w taking direction w mod 2, output block (w / 2) mod 2 and line
  // block w / 4 of the 32 x 32 even and odd halves
  constexpr bool MFL32 = NT == 32 && C::NW == 8 && C::NPW == 1;
  __shared__ TC sTab[(MFL || MFL32) ? 2 * NT * NT : 1];
  if constexpr (MFL || MFL32) {
    const TC* tab = line_tab<C::L, TC>(LT_DERIV_T);
    for (int i = tid; i < 2 * NT * NT; i += C::NTHR) sTab[i] = tab[i];
  }
  if (tid < NT) {
    sTh[tid] = t.sin_Th[tid];
    sCT[tid] = t.cos_Th[tid];
    sWm[tid] = t.wmean[tid];
  }
  if (tid < C::NF) {
    sPh[tid] = t.sin_Ph[tid];
    sCP[tid] = t.cos_Ph[tid];
  }
  for (int i = tid; i < d.n_r; i += C::NTHR) sInvR[i] = t.inv_r[i];
  for (int i = tid; i < d.n_th; i += C::NTHR) sCot[i] = t.cot_th[i];
  __syncthreads();
  const bool useTh = a.terms & 8u, usePh = a.terms & 16u;
  const bool needT = a.T != nullptr;
  // ynext may be Yin itself (stages 2 and 3 update the stage buffer in place,
  // each workgroup only rewriting the planes it has already read): no restrict
  const TY* Yin = static_cast<const TY*>(a.Yin);
  const TO* Tin = static_cast<const TO*>(a.T);
  TO* ynext = static_cast<TO*>(a.ynext);

  // the resident workgroups advance through the plane groups together (round k
  // takes groups k gridDim .. k gridDim + gridDim - 1), in the direction d.rev;
  // every global operand of a workgroup's next group (state, T, acc, y, and the
  // per-plane coefficients) is loaded one iteration ahead (register double
  // buffering), so its loads are in flight during the lines and the epilogue.
  // Groups that lie wholly inside the array (all but possibly the last) load
  // without per-lane predicates.
  const int gstep = int(gridDim.x);
  auto gid = [&](int k) { return d.rev ? ngroups - 1 - k : k; };
  const bool apply = a.mode == PM_APPLY, scat = !apply && d.scattering;
  const int sh_ph = __builtin_ctz(d.n_ph), sh_th = __builtin_ctz(d.n_th);
  // paired order: the column m of the thread's points, the LDS (and plain-order)
  // offset of its points (PM 2, 3) and the byte offset of its plain-order or
  // paired-order operand
  int lofs = 0;
  uint32_t bo_pm = 0;
  if constexpr (PM != 0) {
    const int m = tid & (C::NF - 1);
    if constexpr (PM == 1)
      bo_pm = uint32_t(tid + paired_pos(m, C::NF / 2, PG) - m) * uint32_t(sizeof(TO));
    else {
      lofs = paired_phi(m, C::NF / 2, PG) - m;
      bo_pm = uint32_t(tid + (a.pair_all ? 0 : lofs)) * 8u;
    }
  }
  auto load_group = [&](int g, TY* yi, TO* ti, double* ai, double* yo) {
    const int plane0 = g * C::NPW;
    const int64_t base = int64_t(plane0) * C::PLANE;
    const TY* __restrict__ Yb = Yin + base;
    const TO* __restrict__ Tb = Tin + base;
    const double* __restrict__ Ab = a.accsrc + base;
    const double* __restrict__ Xb = a.ysrc + base;
    const uint32_t bx = PM == 2 ? lane_opaque(bo_pm) : 0u;
    if (plane0 + C::NPW <= npl) {
#pragma unroll
      for (int q = 0; q < C::PPT; ++q) {
        const uint32_t p = uint32_t(tid + q * C::NTHR);
        yi[q] = ld_stream<NT_PLANE_LD>(Yb + p);
        ti[q] = needT ? ld_stream<NT_PLANE_LD>(Tb + p) : TO(0);
        if constexpr (NA && (NY || YA)) {
          if constexpr (PM == 2 && MIX)
            ai[q] = ld_stream<NT_PLANE_LDA>(byte_off(Ab + q * C::NTHR, bx));
          else
            ai[q] = ld_stream<NT_PLANE_LDA>(Ab + p);
        }
        if constexpr (NY) {
          if constexpr (PM == 2)
            yo[q] = ld_stream<NT_PLANE_LDA>(byte_off(Xb + q * C::NTHR, bx));
          else
            yo[q] = ld_stream<NT_PLANE_LDA>(Xb + p);
        }
      }
    } else {
#pragma unroll
      for (int q = 0; q < C::PPT; ++q) {
        const uint32_t p = uint32_t(tid + q * C::NTHR);
        const bool ok = plane0 + int(p) / C::PLANE < npl;
        yi[q] = ok ? ld_stream<NT_PLANE_LD>(Yb + p) : TY(0);
        ti[q] = (ok && needT) ? ld_stream<NT_PLANE_LD>(Tb + p) : TO(0);
        if constexpr (NA && (NY || YA)) {
          if constexpr (PM == 2 && MIX)
            ai[q] = ok ? ld_stream<NT_PLANE_LDA>(byte_off(Ab + q * C::NTHR, bx)) : 0.0;
          else
            ai[q] = ok ? ld_stream<NT_PLANE_LDA>(Ab + p) : 0.0;
        }
        if constexpr (NY) {
          if constexpr (PM == 2)
            yo[q] = ok ? ld_stream<NT_PLANE_LDA>(byte_off(Xb + q * C::NTHR, bx)) : 0.0;
          else
            yo[q] = ok ? ld_stream<NT_PLANE_LDA>(Xb + p) : 0.0;
        }
      }
    }
  };
  // thread tid < NPW keeps the coefficients of plane g NPW + tid (the geometric
  // factors come from the LDS tables)
  struct PlaneCoef {
    double kappa, eta, sigma;
  };
  auto load_info = [&](int g, PlaneCoef& pc) {
    if (tid < C::NPW) {
      const int pid = min(g * C::NPW + tid, npl - 1);
      pc.kappa = apply ? 0.0 : cf.kappa[pid];
      pc.eta = apply ? 0.0 : cf.eta[pid];
      pc.sigma = scat ? cf.sigma[pid] : 0.0;
    }
  };
  // the last stage (acc read, no y) loads acc for the current group after the
  // group barrier instead of one group ahead: fewer registers
  constexpr bool NA_AHEAD = NA && (NY || YA);
  // inflow nodes (Sect. 4.2) among this thread's points: cos Theta > 0 (inflow at
  // r_in) and < 0 (inflow at r_out), one bit per point
  uint32_t cpos = 0, cneg = 0;
#pragma unroll
  for (int q = 0; q < C::PPT; ++q) {
    const double cT = sCT[C::row_of(tid, q)];
    cpos |= uint32_t(cT > 0.0) << q;
    cneg |= uint32_t(cT < 0.0) << q;
  }
  TY yin[C::PPT];
  TO tn[C::PPT];
  double an[NA_AHEAD ? C::PPT : 1], yn[NY ? C::PPT : 1];
  PlaneCoef pin{};
  int kk = int(blockIdx.x);
  if (kk < ngroups) {
    load_group(gid(kk), yin, tn, an, yn);
    load_info(gid(kk), pin);
  }
  for (; kk < ngroups; kk += gstep) {
    const int grp = gid(kk);
    const int plane0 = grp * C::NPW;
#pragma unroll
    for (int q = 0; q < C::PPT; ++q) sY[C::lds(tid + q * C::NTHR) + lofs] = yin[q];
    if constexpr (MEAN_STAGED) {
      if (scat) {
        static_assert(C::PLANE % C::NTHR == 0, "a thread's staged point q lies in plane q NTHR / PLANE");
        double mp[C::NPW];
#pragma unroll
        for (int pl = 0; pl < C::NPW; ++pl) mp[pl] = 0.0;
#pragma unroll
        for (int q = 0; q < C::PPT; ++q) mp[(q * C::NTHR) / C::PLANE] += sWm[C::row_of(tid, q)] * double(yin[q]);
#pragma unroll
        for (int pl = 0; pl < C::NPW; ++pl) {
          const double v = plane_rows_sum<64>(mp[pl]);
          if ((tid & 63) == 0) sMean[tid >> 6][pl] = v;
        }
      }
    }
    if (tid < C::NPW) {
      const int pid = min(plane0 + tid, npl - 1);
      const int l = (pid >> sh_ph) & (d.n_th - 1);
      const int j = (pid >> (sh_ph + sh_th)) % d.n_r;
      PlaneInfo pi;
      pi.inv_r = sInvR[j];
      pi.cot_th = sCot[l];
      pi.kappa = pin.kappa;
      pi.eta = pin.eta;
      pi.sigma = pin.sigma;
      pi.mean = 0.0;
      pi.j = j;
      pi.pad = 0;
      sPl[tid] = pi;
    }
    __syncthreads();
    TO tv[C::PPT];
    double av[NA ? C::PPT : 1], yv[NY ? C::PPT : 1];
#pragma unroll
    for (int q = 0; q < C::PPT; ++q) {
      tv[q] = tn[q];
      if constexpr (NA_AHEAD) av[q] = an[q];
      if constexpr (NY) yv[q] = yn[q];
    }
    if constexpr (NA && !NA_AHEAD) {
      const double* __restrict__ Ab = a.accsrc + int64_t(plane0) * C::PLANE;
      const uint32_t ba = PM == 3 && MIX ? lane_opaque(bo_pm) : 0u;
#pragma unroll
      for (int q = 0; q < C::PPT; ++q) {
        const uint32_t p = uint32_t(tid + q * C::NTHR);
        if constexpr (PM == 3 && MIX)
          av[q] = plane0 + int(p) / C::PLANE < npl ? ld_stream<NT_PLANE_LDA>(byte_off(Ab + q * C::NTHR, ba)) : 0.0;
        else
          av[q] = plane0 + int(p) / C::PLANE < npl ? ld_stream<NT_PLANE_LDA>(Ab + p) : 0.0;
      }
    }
    if (kk + gstep < ngroups) {
      load_group(gid(kk + gstep), yin, tn, an, yn);
      load_info(gid(kk + gstep), pin);
    }

    {  // line phase
      const int lane = tid & 63;
      const int part = wave_uniform(tid >> 6);
      const int pl = lane / C::LPP, li = lane % C::LPP;
      const bool isTh = li < NT;
      const LineMap<NT> lm = line_map<NT>(pl, li);
      const double inv_r = sPl[pl].inv_r, cot_th = sPl[pl].cot_th;
      if constexpr (AN) {
        // the ten moments (FP64).  The wavefronts share the work by Fourier
        // component of the Phi rows (S0: moments 0, 1, 4; C1: 2, 7; S1: 3, 8; C2 and
        // S2 with S0: 5, 6, 9); lane li of the plane sums half li div NT of row
        // i = li mod NT, and each moment is reduced over the 2 NT lanes of the plane
        const int i = li % NT, q0 = (li / NT) * NT, rb = pl * C::PS + i * C::RS + q0;
        const double wr = sWm[i], cT = sCT[i], sT = sTh[i];
        for (int grp = part; grp < 4; grp += C::NW) {
          if (grp == 0) {
            double S0 = 0.0;
#pragma unroll
            for (int q = 0; q < NT; ++q) S0 += double(sY[rb + q]);
            const double a0 = plane_rows_sum<2 * NT>(wr * S0), a1 = plane_rows_sum<2 * NT>(wr * cT * S0),
                         a4 = plane_rows_sum<2 * NT>(wr * cT * cT * S0);
            if (li == 0) {
              sMo[pl][0] = a0;
              sMo[pl][1] = a1;
              sMo[pl][4] = a4;
            }
          } else if (grp == 1 || grp == 2) {
            const double* tr = grp == 1 ? sCP : sPh;  // cos Phi or sin Phi
            double S = 0.0;
#pragma unroll
            for (int q = 0; q < NT; ++q) S += tr[q0 + q] * double(sY[rb + q]);
            const double b0 = plane_rows_sum<2 * NT>(wr * sT * S), b1 = plane_rows_sum<2 * NT>(wr * cT * sT * S);
            if (li == 0) {
              sMo[pl][grp == 1 ? 2 : 3] = b0;
              sMo[pl][grp == 1 ? 7 : 8] = b1;
            }
          } else {
            double S0 = 0.0, C2 = 0.0, S2 = 0.0;
#pragma unroll
            for (int q = 0; q < NT; ++q) {
              const double v = double(sY[rb + q]), c = sCP[q0 + q], sn = sPh[q0 + q];
              S0 += v;
              C2 += (c * c - sn * sn) * v;
              S2 += 2.0 * sn * c * v;
            }
            const double f = 0.5 * wr * sT * sT;
            const double c5 = plane_rows_sum<2 * NT>(f * (S0 + C2)), c6 = plane_rows_sum<2 * NT>(f * (S0 - C2)),
                         c9 = plane_rows_sum<2 * NT>(f * S2);
            if (li == 0) {
              sMo[pl][5] = c5;
              sMo[pl][6] = c6;
              sMo[pl][9] = c9;
            }
          }
        }
      } else if (MEAN_STAGED) {
        if (scat && tid < C::NPW) {
          double m = 0.0;
#pragma unroll
          for (int w = 0; w < C::NW; ++w) m += sMean[w][tid];
          sPl[tid].mean = m;
        }
      } else if (scat && part == 0) {
        // weighted row sum of each Phi row (FP64), reduced over the NT Phi lanes of the plane
        double s = 0.0;
        if (!isTh) {
#pragma unroll
          for (int q = 0; q < C::L; ++q) s += double(sY[lm.idx(q)]);
          s *= sWm[li - NT];
        }
        s = plane_rows_sum<NT>(s);
        if (li == NT) sPl[pl].mean = s;
      }
      if constexpr (MFL32) {
        // Theta (w even): P = A E, Q = B O over the 32 DFS lines (column c and,
        // reversed, c + 32), input index j = s + 8 (l / 16) so that the two row
        // groups a 16-lane LDS access spans fall on different banks; Phi (w odd):
        // P = E A^T, Q = O B^T over the 32 rows, j = 4 s + l / 16.  Outputs q and
        // 63 - q of a line are P + Q and Q - P.
        const bool th = (part & 1) == 0;
        const int ib = (part >> 1) & 1, nb = part >> 2;
        const int lr = lane & 15, lk = lane >> 4;
        using VC = typename std::conditional<sizeof(TC) == 8, v4d, v4f>::type;
        auto mfma = [](TC a, TC b, VC c) {
          if constexpr (sizeof(TC) == 8)
            return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
          else
            return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
        };
        VC cp = {0, 0, 0, 0}, cq = {0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < NT / 4; ++s) {
          const int jj = th ? s + 8 * lk : 4 * s + lk;
          const TC ta = sTab[jj * NT + ib * 16 + lr], tb = sTab[NT * NT + jj * NT + ib * 16 + lr];
          if (th) {
            const TC x = TC(sY[jj * C::RS + nb * 16 + lr]), y = TC(sY[jj * C::RS + nb * 16 + lr + NT]);
            cp = mfma(ta, x + y, cp);
            cq = mfma(tb, x - y, cq);
          } else {
            const int row = nb * 16 + lr;
            const TC x = TC(sY[row * C::RS + jj]), y = TC(sY[row * C::RS + (C::L - 1 - jj)]);
            cp = mfma(x + y, ta, cp);
            cq = mfma(x - y, tb, cq);
          }
        }
        const double ir = sPl[0].inv_r, ct = sPl[0].cot_th;
        // C row of register v: interleaved for the FP64 product, in blocks of four
        // for the FP32 one
        const int r0 = sizeof(TC) == 8 ? lk : 4 * lk, rs = sizeof(TC) == 8 ? 4 : 1;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const TC pv = cp[v] + cq[v], qv = cq[v] - cp[v];
          if (th) {  // output a of column nb 16 + lr, and a of its partner column
            const int a = ib * 16 + r0 + rs * v, col = nb * 16 + lr;
            sR[0][a * C::RS + col] = TC(line_coef<NT>(true, a, col, ir, ct, sTh, sPh) * pv);
            sR[0][a * C::RS + col + NT] = TC(line_coef<NT>(true, C::L - 1 - a, col, ir, ct, sTh, sPh) * qv);
          } else {  // row nb 16 + r0 + rs v: outputs ib 16 + lr and 63 - that
            const int row = nb * 16 + r0 + rs * v, q = ib * 16 + lr;
            sR[1][row * C::RS + q] = TC(line_coef<NT>(false, q, NT + row, ir, ct, sTh, sPh) * pv);
            sR[1][row * C::RS + (C::L - 1 - q)] = TC(line_coef<NT>(false, C::L - 1 - q, NT + row, ir, ct, sTh, sPh) * qv);
          }
        }
      } else if constexpr (MFL) {
        // Theta (w even): P = A^T E, Q = B^T O with E, O = Y[j][c] +- Y[j][c + 16]
        // (the DFS line of column c and its reversed partner half); Phi (w odd):
        // P = E A, Q = O B with E, O = Y[i][j] +- Y[i][31 - j].  Outputs q and
        // 31 - q of a line are P + Q and Q - P.
        const int mp = part >> 1;
        const bool th = (part & 1) == 0;
        const int lr = lane & 15, lk = lane >> 4;
        const int pb = mp * C::PS;
        using VC = typename std::conditional<sizeof(TC) == 8, v4d, v4f>::type;
        VC cp = {0, 0, 0, 0}, cq = {0, 0, 0, 0};
        auto mfma = [](TC a, TC b, VC c) {
          if constexpr (sizeof(TC) == 8)
            return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
          else
            return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
        };
#pragma unroll 1
        for (int k = 0; k < NT / 4; ++k) {
          const int j = 4 * k + lk;
          const TC ta = sTab[j * NT + lr], tb = sTab[NT * NT + j * NT + lr];
          if (th) {
            const TC x = TC(sY[pb + j * C::RS + lr]), y = TC(sY[pb + j * C::RS + lr + NT]);
            cp = mfma(ta, x + y, cp);
            cq = mfma(tb, x - y, cq);
          } else {
            const TC x = TC(sY[pb + lr * C::RS + j]), y = TC(sY[pb + lr * C::RS + (C::L - 1 - j)]);
            cp = mfma(x + y, ta, cp);
            cq = mfma(x - y, tb, cq);
          }
        }
        const double ir = sPl[mp].inv_r, ct = sPl[mp].cot_th;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          // C row (output index for Theta, plane row for Phi): interleaved for
          // the FP64 product, in blocks of four for the FP32 one
          const int a = sizeof(TC) == 8 ? lk + 4 * v : 4 * lk + v;
          const TC pv = cp[v] + cq[v], qv = cq[v] - cp[v];
          if (th) {  // line = column lr; outputs a and 31 - a (row a of column lr + 16)
            sR[0][pb + a * C::RS + lr] = TC(line_coef<NT>(true, a, lr, ir, ct, sTh, sPh) * pv);
            sR[0][pb + a * C::RS + lr + NT] = TC(line_coef<NT>(true, C::L - 1 - a, lr, ir, ct, sTh, sPh) * qv);
          } else {  // row a; outputs lr and 31 - lr
            sR[1][pb + a * C::RS + lr] = TC(line_coef<NT>(false, lr, NT + a, ir, ct, sTh, sPh) * pv);
            sR[1][pb + a * C::RS + (C::L - 1 - lr)] =
                TC(line_coef<NT>(false, C::L - 1 - lr, NT + a, ir, ct, sTh, sPh) * qv);
          }
        }
      } else {
        TC* out = sR[isTh ? 0 : 1];
        // the line is streamed from LDS against the transposed table instead of
        // being held in registers: fewer registers, higher occupancy
        eo_pairs_stream<C::L, C::PPW, true, TC, 2>(
            line_tab<C::L, TC>(LT_DERIV_T), part * C::PPW, [&](int q) { return TC(sY[lm.idx(q)]); },
            [&](int q, TC z) { out[lm.idx(q)] = TC(line_coef<NT>(isTh, q, li, inv_r, cot_th, sTh, sPh)) * z; });
      }
    }
    __syncthreads();

    const int64_t base = int64_t(plane0) * C::PLANE;
    const uint32_t bs = PM == 1 || PM == 3 || (PM == 2 && MIX) ? lane_opaque(bo_pm) : 0u;
#pragma unroll
    for (int q = 0; q < C::PPT; ++q) {
      const int p = tid + q * C::NTHR;
      const int pl = p / C::PLANE;
      if (plane0 + pl >= npl) continue;
      const int64_t gp = base + uint32_t(p);
      const int lp = C::lds(p) + lofs;
      double LY = double(tv[q]);
      if (useTh) LY += double(sR[0][lp]);
      if (usePh) LY += double(sR[1][lp]);
      if (a.mode == PM_APPLY) {
        st_stream<NT_PLANE_ST>(a.out + gp, LY);
        continue;
      }
      const PlaneInfo& pi = sPl[pl];
      const double Yv = double(sY[lp]);
      double inscat = pi.mean;
      if constexpr (AN) {
        const int iTh = C::row_of(tid, q), m = p % C::NF + lofs;
        inscat = phase_contract(cf, sMo[pl], sCT[iTh], sTh[iTh] * sCP[m], sTh[iTh] * sPh[m]);
      }
      double k = -LY + pi.eta - (pi.kappa + pi.sigma) * Yv + pi.sigma * inscat;
      if (d.bc && ((pi.j == 0 && ((cpos >> q) & 1u)) || (pi.j == d.n_r - 1 && ((cneg >> q) & 1u)))) k = 0.0;
      if (a.mode == PM_RHS) {
        st_stream<NT_PLANE_ST>(a.out + gp, k);
        continue;
      }
      double ab = Yv, yb = Yv;
      if constexpr (NA) ab = av[q];
      if constexpr (NY) yb = yv[q];
      if constexpr (YR) ab = yb + (Yv - yb) * (1.0 / 3.0);
      if constexpr (YA) yb = ab;
      if constexpr (PM == 3 || (PM == 2 && MIX)) {
        if (a.accdst)
          st_stream<NT_PLANE_STA>(byte_off(a.accdst + (base + q * C::NTHR), bs), ab + a.cb * k);
      } else {
        if (a.accdst) st_stream<NT_PLANE_STA>(a.accdst + gp, ab + a.cb * k);
      }
      if constexpr (PM == 1) {
        if (ynext) st_stream<NT_PLANE_ST>(byte_off(ynext + (base + q * C::NTHR), bs), TO(yb + a.cn * k));
      } else {
        if (ynext) st_stream<NT_PLANE_ST>(ynext + gp, TO(yb + a.cn * k));
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// transpose: one adjoint stage, or L^T only (lt_out).
//   u = M (xs x);  a = -(T + Theta^T + Phi^T) - (kappa + sigma) u + sigma K^T u
//   lacc = (laccsrc or lam) + a;  kbnext = ka lam + kb a
//   per plane: g_kappa -= sum u Y_s, g_eta += sum u, g_sigma += sum u (K Y_s) - sum u Y_s
//   (K = avg for isotropic scattering: sum u (K Y_s) = <Y_s> sum u)
// Transposed line: v_q = coef_q u_q; z = D v; result_q = -z_q (D^T = -D).

// four waves per SIMD: measured 10 % faster per adjoint step than three; the
// isotropic 16 x 32 instance takes 102 VGPRs (at five waves it spills, for 0.4 %)
template <int NT, bool AN>
__global__ __launch_bounds__(PC<NT>::NTHR) __attribute__((amdgpu_waves_per_eu(4))) void k_plane_adj(KDims d, KTab t, KCoef cf, AdjArgs a,
                                                            double* lt_out) {
  using C = PC<NT>;
  // isotropic scattering on 16 x 32 and 32 x 64 planes: the plane sums of u,
  // u Y_s and w Y_s (for K^T u and the gradients) are summed from the values each
  // thread loads, reduced over the wavefront and then over the wavefronts in a
  // fixed order, instead of by one wavefront over the staged rows ahead of its
  // lines (Y_s is then not staged)
  constexpr bool RED_STAGED = NT >= 16 && !AN;
  static_assert(!RED_STAGED || C::PLANE % C::NTHR == 0, "a thread's point q lies in plane q NTHR / PLANE");
  __shared__ double sU[C::PTSP];
  __shared__ double sY[RED_STAGED ? 1 : C::PTSP];
  __shared__ double sR[2][C::PTSP];
  __shared__ double sRed[RED_STAGED ? 1 : C::NPW * NT][3];
  __shared__ double sRedW[RED_STAGED ? C::NW : 1][C::NPW][3];
  __shared__ double sMoU[AN ? C::NPW : 1][NMOM], sMoY[AN ? C::NPW : 1][NMOM];
  __shared__ double sTh[NT], sPh[C::NF], sCP[C::NF], sCT[NT], sWm[NT];
  // per plane of the workgroup: geometric factors, coefficients, radial index
  struct AdjPlane {
    double inv_r, cot_th, kappa, sigma;
    int j, pad;
  };
  __shared__ AdjPlane sPA[C::NPW];

  const int tid = threadIdx.x;
  const int npl = int(d.nplanes);
  const int plane0 = int(blockIdx.x) * C::NPW;
  const int64_t gbase = int64_t(plane0) * C::PLANE;
  const bool lt = lt_out != nullptr;
  // 16 x 32 planes: the transposed lines as the MFMA products of the forward
  // pass, on the coefficient-weighted input (adjoint step 5.82 -> 5.42 ms on the
  // 4-group workload; fewer registers spilled than with streamed lines)
  constexpr bool MFA = NT == 16 && C::NW == 4 && C::NPW == 2;
  __shared__ double sTab[MFA ? 2 * NT * NT : 1];
  if constexpr (MFA) {
    const double* tab = line_tab<C::L, double>(LT_DERIV_T);
    for (int i = tid; i < 2 * NT * NT; i += C::NTHR) sTab[i] = tab[i];
  }
  const bool grads = !lt && (a.gk || a.ge || a.gs) && a.Ys;
  if (tid < NT) {
    sTh[tid] = t.sin_Th[tid];
    sCT[tid] = t.cos_Th[tid];
    sWm[tid] = t.wmean[tid];
  }
  if (tid < C::NF) {
    sPh[tid] = t.sin_Ph[tid];
    sCP[tid] = t.cos_Ph[tid];
  }
  if (tid < C::NPW) {
    // plane index (e, j, l, k) with k fastest; n_phi and n_theta are powers of two
    const int pid = min(plane0 + tid, npl - 1);
    const int sh_ph = __builtin_ctz(d.n_ph), sh_th = __builtin_ctz(d.n_th);
    const int l = (pid >> sh_ph) & (d.n_th - 1);
    const int j = (pid >> (sh_ph + sh_th)) % d.n_r;
    AdjPlane pa;
    pa.inv_r = t.inv_r[j];
    pa.cot_th = t.cot_th[l];
    pa.kappa = lt ? 0.0 : cf.kappa[pid];
    pa.sigma = (!lt && d.scattering) ? cf.sigma[pid] : 0.0;
    pa.j = j;
    pa.pad = 0;
    sPA[tid] = pa;
  }
  __syncthreads();

  double xr[C::PPT], tv[C::PPT], lv[C::PPT], cv[C::PPT];
  double ru[RED_STAGED ? C::NPW : 1], ruy[RED_STAGED ? C::NPW : 1], rwy[RED_STAGED ? C::NPW : 1];
#pragma unroll
  for (int pl = 0; pl < (RED_STAGED ? C::NPW : 1); ++pl) ru[pl] = ruy[pl] = rwy[pl] = 0.0;
#pragma unroll
  for (int q = 0; q < C::PPT; ++q) {
    const int p = tid + q * C::NTHR;
    const int pl = p / C::PLANE;
    const bool ok = plane0 + pl < npl;
    const int64_t gp = gbase + p;
    const int iTh = (p % C::PLANE) / C::NF;
    const double x = ok ? ld_stream<NT_ADJ_LD>(a.x + gp) : 0.0;
    xr[q] = x;
    double u = lt ? x : a.xs * x;
    if (!lt && d.bc) {  // inflow nodes (Sect. 4.2) are held: u = 0 there
      const int j = sPA[pl].j;
      const double c = sCT[iTh];
      if ((j == 0 && c > 0.0) || (j == d.n_r - 1 && c < 0.0)) u = 0.0;
    }
    sU[C::lds(p)] = u;
    const double ys = (grads && ok) ? ld_stream<NT_ADJ_LD>(a.Ys + gp) : 0.0;
    if constexpr (RED_STAGED) {
      const int rp = (q * C::NTHR) / C::PLANE;
      ru[rp] += u;
      ruy[rp] += u * ys;
      rwy[rp] += sWm[iTh] * ys;
    } else {
      if (grads) sY[C::lds(p)] = ys;
    }
    tv[q] = (ok && a.T) ? ld_stream<NT_ADJ_LD>(a.T + gp) : 0.0;
    lv[q] = (ok && !lt && !a.lam_is_x && a.lam) ? ld_stream<NT_ADJ_LD>(a.lam + gp) : 0.0;
    cv[q] = (ok && !lt && a.laccsrc) ? ld_stream<NT_ADJ_LD>(a.laccsrc + gp) : 0.0;
  }
  const bool need_red = !lt && (grads || d.scattering);
  if constexpr (RED_STAGED) {
    if (need_red) {
#pragma unroll
      for (int pl = 0; pl < C::NPW; ++pl) {
        const double v0 = plane_rows_sum<64>(ru[pl]), v1 = plane_rows_sum<64>(ruy[pl]),
                     v2 = plane_rows_sum<64>(rwy[pl]);
        if ((tid & 63) == 0) {
          sRedW[tid >> 6][pl][0] = v0;
          sRedW[tid >> 6][pl][1] = v1;
          sRedW[tid >> 6][pl][2] = v2;
        }
      }
    }
  }
  __syncthreads();

  {
    const int lane = tid & 63;
    const int part = wave_uniform(tid >> 6);
    const int pl = lane / C::LPP, li = lane % C::LPP;
    const bool isTh = li < NT;
    const LineMap<NT> lm = line_map<NT>(pl, li);
    const double inv_r = sPA[pl].inv_r, cot_th = sPA[pl].cot_th;
    if constexpr (!RED_STAGED) {
      if (part == 0 && !isTh && !lt) {
        // row sums of u, u Y_s and w Y_s of each Phi row (summed per plane below)
        const int i = li - NT;
        double su = 0.0, suy = 0.0, sy = 0.0;
        for (int q = 0; q < C::L; ++q) {
          const int ix = lm.idx(q);
          su += sU[ix];
          if (grads) {
            suy += sU[ix] * sY[ix];
            sy += sY[ix];
          }
        }
        sRed[pl * NT + i][0] = su;
        sRed[pl * NT + i][1] = suy;
        sRed[pl * NT + i][2] = sWm[i] * sy;
      }
    }
    if constexpr (AN) if (part == 0) {
      // unweighted moments of u (for K^T u) and weighted moments of Y_s (for the
      // sigma gradient), reduced over the NT Phi lanes of the plane
      double mu[NMOM], my[NMOM];
#pragma unroll
      for (int k = 0; k < NMOM; ++k) mu[k] = my[k] = 0.0;
      if (!isTh) {
        const int i = li - NT;
        double S0, C1, S1, C2, S2;
        row_fourier<C::NF>(sCP, sPh, [&](int q) { return sU[lm.idx(q)]; }, S0, C1, S1, C2, S2);
        row_moments(1.0, sCT[i], sTh[i], S0, C1, S1, C2, S2, mu);
        if (grads) {
          row_fourier<C::NF>(sCP, sPh, [&](int q) { return sY[lm.idx(q)]; }, S0, C1, S1, C2, S2);
          row_moments(sWm[i], sCT[i], sTh[i], S0, C1, S1, C2, S2, my);
        }
      }
#pragma unroll
      for (int k = 0; k < NMOM; ++k) {
        mu[k] = plane_rows_sum<NT>(mu[k]);
        my[k] = plane_rows_sum<NT>(my[k]);
      }
      if (li == NT) {
#pragma unroll
        for (int k = 0; k < NMOM; ++k) {
          sMoU[pl][k] = mu[k];
          sMoY[pl][k] = my[k];
        }
      }
    }
    if constexpr (MFA) {
      const int mp = part >> 1;
      const bool th = (part & 1) == 0;
      const int lr = lane & 15, lk = lane >> 4;
      const int pb = mp * C::PS;
      const double ir = sPA[mp].inv_r, ct = sPA[mp].cot_th;
      v4d cp = {0.0, 0.0, 0.0, 0.0}, cq = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
      for (int k = 0; k < NT / 4; ++k) {
        const int j = 4 * k + lk;
        const double ta = sTab[j * NT + lr], tb = sTab[NT * NT + j * NT + lr];
        if (th) {  // column lr: elements j (row j) and 31 - j (row j of column lr + 16)
          const double x = line_coef<NT>(true, j, lr, ir, ct, sTh, sPh) * sU[pb + j * C::RS + lr];
          const double y = line_coef<NT>(true, C::L - 1 - j, lr, ir, ct, sTh, sPh) * sU[pb + j * C::RS + lr + NT];
          cp = __builtin_amdgcn_mfma_f64_16x16x4f64(ta, x + y, cp, 0, 0, 0);
          cq = __builtin_amdgcn_mfma_f64_16x16x4f64(tb, x - y, cq, 0, 0, 0);
        } else {  // row lr: elements j and 31 - j
          const double x = line_coef<NT>(false, j, NT + lr, ir, ct, sTh, sPh) * sU[pb + lr * C::RS + j];
          const double y =
              line_coef<NT>(false, C::L - 1 - j, NT + lr, ir, ct, sTh, sPh) * sU[pb + lr * C::RS + (C::L - 1 - j)];
          cp = __builtin_amdgcn_mfma_f64_16x16x4f64(x + y, ta, cp, 0, 0, 0);
          cq = __builtin_amdgcn_mfma_f64_16x16x4f64(x - y, tb, cq, 0, 0, 0);
        }
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int a4 = lk + 4 * v;
        const double pv = cp[v] + cq[v], qv = cq[v] - cp[v];
        if (th) {
          sR[0][pb + a4 * C::RS + lr] = -pv;
          sR[0][pb + a4 * C::RS + lr + NT] = -qv;
        } else {
          sR[1][pb + a4 * C::RS + lr] = -pv;
          sR[1][pb + a4 * C::RS + (C::L - 1 - lr)] = -qv;
        }
      }
    } else {
      double* out = sR[isTh ? 0 : 1];
      eo_pairs_stream<C::L, C::PPW, true, double>(
          line_tab<C::L>(LT_DERIV_T), part * C::PPW,
          [&](int q) { return line_coef<NT>(isTh, q, li, inv_r, cot_th, sTh, sPh) * sU[lm.idx(q)]; },
          [&](int q, double z) { out[lm.idx(q)] = -z; });
    }
  }
  __syncthreads();

  // plane sums of u for K^T u (isotropic, staged reduction): the wavefronts'
  // partial sums in a fixed order
  double psu[RED_STAGED ? C::NPW : 1];
  if constexpr (RED_STAGED) {
#pragma unroll
    for (int pl = 0; pl < C::NPW; ++pl) {
      psu[pl] = 0.0;
      if (need_red) {
#pragma unroll
        for (int w = 0; w < C::NW; ++w) psu[pl] += sRedW[w][pl][0];
      }
    }
  }
#pragma unroll
  for (int q = 0; q < C::PPT; ++q) {
    const int p = tid + q * C::NTHR;
    const int pl = p / C::PLANE;
    if (plane0 + pl >= npl) continue;
    const int64_t gp = gbase + p;
    const int lp = C::lds(p);
    const double LTu = tv[q] + sR[0][lp] + sR[1][lp];
    if (lt) {
      lt_out[gp] = LTu;
      continue;
    }
    const double u = sU[lp];
    const int iTh = (p % C::PLANE) / C::NF;
    double av = -LTu - sPA[pl].kappa * u;
    if (d.scattering) {
      // K^T u at this direction: w(omega') times the phase-weighted sums of u
      double ktu;
      if constexpr (AN) {
        const int m = p % C::NF;
        ktu = sWm[iTh] * phase_contract(cf, sMoU[pl], sCT[iTh], sTh[iTh] * sCP[m], sTh[iTh] * sPh[m]);
      } else if constexpr (RED_STAGED) {
        ktu = sWm[iTh] * psu[(q * C::NTHR) / C::PLANE];
      } else {
        double su = 0.0;
#pragma unroll
        for (int ii = 0; ii < NT; ++ii) su += sRed[pl * NT + ii][0];
        ktu = sWm[iTh] * su;
      }
      av += sPA[pl].sigma * (ktu - u);
    }
    const double lam = a.lam_is_x ? xr[q] : lv[q];
    if (a.laccdst) st_stream<NT_ADJ_ST>(a.laccdst + gp, (a.laccsrc ? cv[q] : lam) + av);
    if (a.kbnext) st_stream<NT_ADJ_ST>(a.kbnext + gp, a.ka * lam + a.kb * av);
  }

  if (grads && tid < C::NPW) {
    const int pl = tid;
    const int pid = plane0 + pl;
    if (pid < npl) {
      double su = 0.0, suy = 0.0, my = 0.0;
      if constexpr (RED_STAGED) {
#pragma unroll
        for (int w = 0; w < C::NW; ++w) {
          su += sRedW[w][pl][0];
          suy += sRedW[w][pl][1];
          my += sRedW[w][pl][2];
        }
      } else {
        for (int ii = 0; ii < NT; ++ii) {
          su += sRed[pl * NT + ii][0];
          suy += sRed[pl * NT + ii][1];
          my += sRed[pl * NT + ii][2];
        }
      }
      if (a.gk) a.gk[pid] -= suy;
      if (a.ge) a.ge[pid] += su;
      if (a.gs && d.scattering) {
        double uky = my * su;  // sum over the plane of u (K Y_s)
        if constexpr (AN) uky = phase_pair(cf, sMoY[pl], sMoU[pl]);
        a.gs[pid] += uky - suy;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// filter of the Theta DFS lines, then of the Phi rows (in place)

template <int NT>
__global__ __launch_bounds__(PC<NT>::NTHR) void k_filter_plane(KDims d, KTab t, double* __restrict__ F) {
  using C = PC<NT>;
  __shared__ double sY[C::PTSP];
  __shared__ double sR[C::PTSP];
  const int tid = threadIdx.x;
  const int64_t plane0 = int64_t(blockIdx.x) * C::NPW;
  const int64_t gbase = plane0 * C::PLANE;
  const int64_t npl = d.nplanes;
#pragma unroll
  for (int q = 0; q < C::PPT; ++q) {
    const int p = tid + q * C::NTHR;
    sY[C::lds(p)] = (plane0 + p / C::PLANE < npl) ? F[gbase + p] : 0.0;
  }
  __syncthreads();
  const int lane = tid & 63;
  const int part = wave_uniform(tid >> 6);
  const int pl = lane / C::LPP, li = lane % C::LPP;
  const bool isTh = li < NT;
  const LineMap<NT> lm = line_map<NT>(pl, li);
  if (isTh)
    eo_pairs_stream<C::L, C::PPW, false, double>(
        line_tab<C::L>(LT_FILTER_T), part * C::PPW, [&](int q) { return sY[lm.idx(q)]; },
        [&](int q, double z) { sR[lm.idx(q)] = z; });
  __syncthreads();
  if (!isTh)
    eo_pairs_stream<C::L, C::PPW, false, double>(
        line_tab<C::L>(LT_FILTER_T), part * C::PPW, [&](int q) { return sR[lm.idx(q)]; },
        [&](int q, double z) { sY[lm.idx(q)] = z; });
  __syncthreads();
#pragma unroll
  for (int q = 0; q < C::PPT; ++q) {
    const int p = tid + q * C::NTHR;
    if (plane0 + p / C::PLANE < npl) F[gbase + p] = sY[C::lds(p)];
  }
}

template <int NT>
unsigned plane_blocks(const KDims& d) {
  return unsigned((d.nplanes + PC<NT>::NPW - 1) / PC<NT>::NPW);
}

}  // namespace

// persistent grid: as many workgroups as can be resident at once
template <typename K>
unsigned persistent_blocks(const KDims& d, K kernel, int threads, int64_t work) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || per_cu < 1) per_cu = 1;
  const int64_t cap = int64_t(d.ncu) * per_cu;
  return unsigned(work < cap ? work : cap);
}

template <int NT, bool NA, int YM, typename TY, typename TO, typename TC, bool AN, int PM = 0>
void launch_plane_t(const KDims& d, const KTab& t, const KCoef& c, const StageArgs& a, hipStream_t s) {
  const int ng = int((d.nplanes + PC<NT>::NPW - 1) / PC<NT>::NPW);
  const unsigned nb = persistent_blocks(d, k_plane<NT, NA, YM, TY, TO, TC, AN, PM>, PC<NT>::NTHR, ng);
  k_plane<NT, NA, YM, TY, TO, TC, AN, PM><<<nb, PC<NT>::NTHR, 0, s>>>(d, t, c, a, ng);
}

// the FP64 RK4 stages in the paired order (launch_plane has checked the shape,
// the stage form of each mode and that the stage matches the mode)
template <int NT, bool AN, typename TY, typename TO, typename TC>
void launch_plane_paired(const KDims& d, const KTab& t, const KCoef& c, const StageArgs& a, hipStream_t s) {
  if constexpr (sizeof(TY) == 8 && sizeof(TO) == 4) {
    // the mixed path's first stage (FP64 state in, checked by launch_plane)
    if constexpr (2 * NT >= 16) launch_plane_t<NT, false, 0, TY, TO, TC, AN, 1>(d, t, c, a, s);
  } else if constexpr (2 * NT >= 16) {
    switch (a.pair_mode) {
      case 1: launch_plane_t<NT, false, 0, TY, TO, TC, AN, 1>(d, t, c, a, s); break;
      case 2:
        if constexpr (sizeof(TO) == 8) {
          if (a.accrec) {
            launch_plane_t<NT, false, 2, TY, TO, TC, AN, 2>(d, t, c, a, s);
            break;
          }
          if (!a.accsrc) {
            launch_plane_t<NT, false, 0, TY, TO, TC, AN, 2>(d, t, c, a, s);
            break;
          }
        }
        launch_plane_t<NT, true, 1, TY, TO, TC, AN, 2>(d, t, c, a, s);
        break;
      default: launch_plane_t<NT, true, 0, TY, TO, TC, AN, 3>(d, t, c, a, s); break;
    }
  }
}

template <int NT, typename TY, typename TO, typename TC>
void launch_plane_nt(const KDims& d, const KTab& t, const KCoef& c, const StageArgs& a, hipStream_t s) {
  const bool na = a.accsrc != nullptr, ny = a.ysrc != nullptr;
  const bool an = d.scattering && c.aniso && a.mode != PM_APPLY;
  if (a.pair_mode) {
    if (an) launch_plane_paired<NT, true, TY, TO, TC>(d, t, c, a, s);
    else launch_plane_paired<NT, false, TY, TO, TC>(d, t, c, a, s);
    return;
  }
  if constexpr (sizeof(TY) == 8 && sizeof(TO) == 8) {
    if (na && ny && a.accsrc == a.ysrc) {  // y is the accumulator source: load it once (AB2 step 3 % faster)
      if (an) launch_plane_t<NT, true, 4, TY, TO, TC, true>(d, t, c, a, s);
      else launch_plane_t<NT, true, 4, TY, TO, TC, false>(d, t, c, a, s);
      return;
    }
    if (a.accrec) {  // checked by launch_plane: ysrc given, no accumulator source
      if (an) launch_plane_t<NT, false, 2, TY, TO, TC, true>(d, t, c, a, s);
      else launch_plane_t<NT, false, 2, TY, TO, TC, false>(d, t, c, a, s);
      return;
    }
  }
  if (an) {
    if (na && ny) launch_plane_t<NT, true, 1, TY, TO, TC, true>(d, t, c, a, s);
    else if (na) launch_plane_t<NT, true, 0, TY, TO, TC, true>(d, t, c, a, s);
    else if (ny) launch_plane_t<NT, false, 1, TY, TO, TC, true>(d, t, c, a, s);
    else launch_plane_t<NT, false, 0, TY, TO, TC, true>(d, t, c, a, s);
  } else {
    if (na && ny) launch_plane_t<NT, true, 1, TY, TO, TC, false>(d, t, c, a, s);
    else if (na) launch_plane_t<NT, true, 0, TY, TO, TC, false>(d, t, c, a, s);
    else if (ny) launch_plane_t<NT, false, 1, TY, TO, TC, false>(d, t, c, a, s);
    else launch_plane_t<NT, false, 0, TY, TO, TC, false>(d, t, c, a, s);
  }
}

template <int NT>
void launch_plane_n(const KDims& d, const KTab& t, const KCoef& c, const StageArgs& a, hipStream_t s) {
  if (!a.mixed)
    launch_plane_nt<NT, double, double, double>(d, t, c, a, s);
  else if (a.yin_f32)
    launch_plane_nt<NT, float, float, float>(d, t, c, a, s);
  else
    launch_plane_nt<NT, double, float, float>(d, t, c, a, s);
}

hipError_t launch_plane(const KDims& d, const KTab& t, const KCoef& c, const StageArgs& a, hipStream_t s) {
  if (a.accrec && (a.mixed || a.mode != PM_STAGE || a.accsrc || !a.ysrc)) return hipErrorInvalidValue;
  if (a.pair_mode) {
    // the FP64 RK4 stage forms: 1 (no accumulator, no y), 2 (stage 1 on a
    // paired state: no accumulator, no y; stage 2: accumulator recovered from y;
    // stage 3: accumulator and y), 3 (accumulator, no y, no ynext)
    // (mixed path: stage 1 also writes the accumulator; no recovered
    // accumulator, the state F always in the plain order)
    const bool na = a.accsrc != nullptr, ny = a.ysrc != nullptr;
    const bool s1 = !na && !ny && (a.mixed || !a.accdst) && a.ynext;
    bool form = false;
    switch (a.pair_mode) {
      case 1: form = s1; break;
      case 2:
        form = (s1 && a.pair_all && !a.mixed) ||
               (ny && a.accdst && a.ynext && (a.accrec ? !na && !a.mixed : (na && a.accsrc != a.ysrc)));
        break;
      case 3: form = na && !ny && a.accdst && !a.ynext; break;
      default: break;
    }
    // (mixed path: the first stage reads the FP64 state, the others the FP32 copy)
    const bool mixed_ok = !a.mixed || (!a.pair_all && (a.pair_mode == 1) == !a.yin_f32);
    if (!form || !mixed_ok || a.mode != PM_STAGE || !paired_order_ok(d) || d.n_Ph != 2 * d.n_Th)
      return hipErrorInvalidValue;
  }
  switch (d.n_Th) {
#define CASE(N)                          \
  case N:                                \
    launch_plane_n<N>(d, t, c, a, s);    \
    break;
    CASE(2) CASE(4) CASE(8) CASE(16) CASE(32)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_plane_adj(const KDims& d, const KTab& t, const KCoef& c, const AdjArgs& a, hipStream_t s) {
  switch (d.n_Th) {
#define CASE(N) \
  case N:                                                                                  \
    if (d.scattering && c.aniso)                                                           \
      k_plane_adj<N, true><<<plane_blocks<N>(d), PC<N>::NTHR, 0, s>>>(d, t, c, a, nullptr);  \
    else                                                                                   \
      k_plane_adj<N, false><<<plane_blocks<N>(d), PC<N>::NTHR, 0, s>>>(d, t, c, a, nullptr); \
    break;
    CASE(2) CASE(4) CASE(8) CASE(16) CASE(32)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_plane_LT(const KDims& d, const KTab& t, const double* G, const double* T, double* out,
                           hipStream_t s) {
  AdjArgs a{};
  a.x = G;
  a.xs = 1.0;
  a.T = T;
  KCoef c{};
  switch (d.n_Th) {
#define CASE(N) \
  case N: k_plane_adj<N, false><<<plane_blocks<N>(d), PC<N>::NTHR, 0, s>>>(d, t, c, a, out); break;
    CASE(2) CASE(4) CASE(8) CASE(16) CASE(32)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_filter_plane(const KDims& d, const KTab& t, double* F, hipStream_t s) {
  switch (d.n_Th) {
#define CASE(N) \
  case N: k_filter_plane<N><<<plane_blocks<N>(d), PC<N>::NTHR, 0, s>>>(d, t, F); break;
    CASE(2) CASE(4) CASE(8) CASE(16) CASE(32)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t init_line_tables_plane(const double* tab) {
  hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_lines), tab, sizeof(double) * LINE_TAB_KINDS * LINE_TAB_SIZE, 0, hipMemcpyHostToDevice);
  if (e != hipSuccess) return e;
  static float f[LINE_TAB_KINDS * LINE_TAB_SIZE];
  for (int i = 0; i < LINE_TAB_KINDS * LINE_TAB_SIZE; ++i) f[i] = float(tab[i]);
  return hipMemcpyToSymbol(HIP_SYMBOL(c_lines_f), f, sizeof f, 0, hipMemcpyHostToDevice);
}
