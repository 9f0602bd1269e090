// Internal declarations shared by the host API and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/sp6d.h"
#include "paired_order.h"

// largest supported n_r (descriptor validation; per-workgroup LDS tables)
constexpr int SP6_MAX_NR = 80;

// device address of the fixed scratch of sp6_step_noalloc (SP6_NOALLOC_SCRATCH_BYTES
// bytes, 256-byte aligned) on `device`, the current device; cached per device
hipError_t noalloc_scratch_ptr(int device, void** out);

// ---------------------------------------------------------------------------
// sizes and device tables, passed to kernels by value

struct KDims {
  int n_eps, n_r, n_th, n_ph, n_Th, n_Ph;
  int plane;        // n_Th * n_Ph: one (Theta, Phi) plane
  int64_t M;        // n_th * n_ph * plane: points per (eps, r)
  int64_t P;        // all points
  int64_t nplanes;  // n_eps * n_r * n_th * n_ph
  int bc, scattering;
  int ncu;          // compute units of the device (persistent grids)
  // traversal direction of the pass passes (fused theta-phi, radial, plane):
  // 0 ascending addresses, 1 descending.  The host alternates it from one pass
  // to the next, so that a pass first reads what the previous one touched last
  // (still in the last-level cache).  Results do not depend on it.
  int rev;
};

struct KTab {
  const double* inv_r;       // [n_r]
  const double* inv_sin_th;  // [n_th]
  const double* cot_th;      // [n_th] cos/sin
  const double* sin_Th;      // [n_Th]
  const double* cos_Th;      // [n_Th]
  const double* sin_Ph;      // [n_Ph]
  const double* cos_Ph;      // [n_Ph]
  const double* wmean;       // [n_Th]  w_i (2 pi / n_Ph) / (4 pi)
  const double* wflux;       // [n_Th]  w_i (2 pi / n_Ph) cos(Theta_i) where cos > 0, else 0
  const double* Dpad;        // radial matrix, zero padded [NRP][KP]
  const double* DpadT;       // its transpose, same padding
  const double* Fpad;        // radial filter matrix, same padding
  const double* FpadT;       // its transpose
  const double* qN;          // [n_r * n_th * n_Th] weights of the particle number
  const double* qJ;          // [n_th * n_Th] weights of the boundary flux (without r^2)
  // mixed precision copies
  const uint16_t* Dsplit;    // bf16x3 split of the radial matrix, [3][NRP][KP3] (bf16 bits)
  int KP, NRP, KP3;
};

struct KCoef {
  const double* kappa;  // [nplanes]
  const double* sigma;
  const double* eta;
  const double* g_in;   // [n_eps][n_th][n_ph][plane]
  const double* g_out;
  // scattering phase function p(mu) = pc0 + pc1 mu + pc2 mu^2; aniso = 0 when
  // isotropic (pc1 = pc2 = 0, pc0 = 1)
  double pc0, pc1, pc2;
  int aniso;
};

// ---------------------------------------------------------------------------
// host tables

struct HostTables {
  std::vector<double> r, theta, phi, Theta, Phi;
  std::vector<double> w_r, w_th, w_ph, w_Th, w_Ph;
  std::vector<double> Dr;  // n_r x n_r, row major
  std::vector<double> inv_r, inv_sin_th, cot_th, sin_Th, cos_Th, sin_Ph, cos_Ph, wmean, wflux;
  std::vector<double> Dpad, DpadT, Fpad, FpadT;
  std::vector<double> qN, qJ;
  int KP = 0, NRP = 0;
};

void build_host_tables(const sp6_desc& d, HostTables& t);
// Chebyshev-Gauss-Lobatto nodes of [a, b] (ascending) and their collocation
// derivative matrix (n x n, row major)
std::vector<double> cgl_nodes(int n, double a, double b);
std::vector<double> cgl_derivative(int n, double a, double b);
// [4][2728]: derivative, filter, and the transposes of both, for every supported
// line length (even/odd form)
std::vector<double> build_line_tables();
// copy the line tables into the constant memory of each kernel file (current device)
hipError_t init_line_tables_columns(const double* tab);
hipError_t init_line_tables_plane(const double* tab);
std::string validate_desc(const sp6_desc& d, sp6_status* code);

// ---------------------------------------------------------------------------
// launchers (defined in the .hip files); all return hipSuccess or an error

enum PlaneMode { PM_APPLY = 0, PM_RHS = 1, PM_STAGE = 2 };

// Stage arguments of the plane pass.  Yin, T and ynext are FP64 on the FP64 path;
// on the mixed path T and ynext are FP32 and Yin is FP64 (first stage, apply,
// rhs) or FP32 (later stages).  Everything else is FP64.
struct StageArgs {
  int mode;              // PlaneMode
  const void* Yin;       // stage input
  const void* T;         // sum of the r, theta, phi terms of L Yin (may be null = 0)
  double* out;           // PM_APPLY / PM_RHS output
  // PM_STAGE: accdst = (accsrc ? accsrc : Yin) + cb * k ; ynext = (ysrc ? ysrc : Yin) + cn * k,
  // or with accrec (FP64, ysrc given, no accsrc) accdst = (ysrc + (Yin - ysrc) / 3) + cb * k
  const double* accsrc;
  double* accdst;
  double cb;
  const double* ysrc;
  void* ynext;
  double cn;
  int accrec;
  uint32_t terms;        // bit 3 Theta, bit 4 Phi
  int mixed;             // 0: FP64 path; 1: mixed path
  int yin_f32;           // mixed path: Yin is FP32
  // FP64 RK4 stages on the 32 x 64 sphere (paired_order_ok), operands in the
  // paired in-plane order (paired_order.h): 0 none; 1 ynext (stage 1 on the
  // caller's plain state); 2 Yin, T, accsrc, accdst and ynext, ysrc plain
  // (stages 2, 3, and stage 1 on a paired state); 3 Yin, T and accsrc, accdst
  // plain (stage 4).  pair_all (modes 2, 3): ysrc or accdst paired as well.
  int pair_mode;
  int pair_all;
};

// the 32 x 64 position sphere with n_Phi >= 16: where the fused theta-phi tiles of
// eight FP64 columns apply, and with them the paired order
bool paired_order_ok(const KDims& d);

hipError_t launch_phi(const KDims& d, const KTab& t, const double* Y, double* T, bool accum,
                      double coef_sign, bool mask_in, double in_scale, hipStream_t s);
hipError_t launch_theta(const KDims& d, const KTab& t, const double* Y, double* T, bool accum,
                        double coef_sign, bool mask_in, double in_scale, hipStream_t s);
// theta and phi terms together into T (not accumulated), for n_phi = 2 n_theta,
// n_theta <= 16, and for the 32 x 64 sphere with n_Phi >= 16; the separate passes
// take every other shape
bool sphere_fusable(const KDims& d, bool mixed);
// paired: Y and T in the paired in-plane order (paired_order_ok only)
hipError_t launch_sphere(const KDims& d, const KTab& t, const double* Y, double* T, double coef_sign,
                         bool mask_in, double in_scale, hipStream_t s, bool paired = false);
hipError_t launch_sphere_mixed(const KDims& d, const KTab& t, const void* Y, bool y_f32, float* T,
                               hipStream_t s, bool paired = false);
hipError_t launch_radial(const KDims& d, const KTab& t, const double* Y, double* T, bool accum,
                         bool transpose, bool mask_in, double in_scale, hipStream_t s);
hipError_t launch_plane(const KDims& d, const KTab& t, const KCoef& c, const StageArgs& a,
                        hipStream_t s);

struct AdjArgs {
  const double* x;       // input (lam or kb), scaled by xs, masked
  double xs;
  const double* T;       // transposed r/theta/phi terms of M xs x
  const double* Ys;      // stage input (for the coefficient gradients), may be null
  const double* lam;     // dLoss/dF_{n+1} (for kb_next)
  const double* laccsrc; // null: lacc = lam + a
  double* laccdst;
  double* kbnext;        // may be null
  double ka, kb;         // kbnext = ka * lam + kb * a
  double* gk;
  double* ge;
  double* gs;
  int lam_is_x;          // x == lam (stage 4): reuse the loaded value
};
hipError_t launch_plane_adj(const KDims& d, const KTab& t, const KCoef& c, const AdjArgs& a,
                            hipStream_t s);
hipError_t launch_plane_LT(const KDims& d, const KTab& t, const double* G, const double* T,
                           double* out, hipStream_t s);

// Fokker-Planck energy coupling: (M0, Q) of every plane of Y (FP64, or FP32 with
// y_f32) into mq, then eta_eff = eta + sigma S per plane (D: energy-node
// derivative, gam: nodes)
hipError_t launch_fp_source(const KDims& d, const KTab& t, const void* Y, bool y_f32, const double* D,
                            const double* gam, double alpha, double* mq, const double* eta, const double* sigma,
                            double* eta_eff, hipStream_t s);

// its adjoint: per plane the moments of the stage input Y and the masked sum
// of X = xs x (mom), then the direction-polynomial coefficients C per plane and
// sigma's gradient (gs, may be null); then lacc += p, kbnext += kb p with
// p(w) = wq(w) sum_k C_k phi_k(w) (kbnext may be null)
hipError_t launch_fp_adj(const KDims& d, const KTab& t, const double* Y, const double* X, double xs, const double* D,
                         const double* gam, double alpha, double* mom, const double* sigma, double* C, double* gs,
                         hipStream_t s);
hipError_t launch_fp_adj_apply(const KDims& d, const KTab& t, const double* C, double* lacc, double* kbnext, double kb,
                               hipStream_t s);

// filter, projection, diagnostics
// the angular line filters, then (radial = 1) the radial filter or (radial = 2)
// its transpose, in place
hipError_t launch_filter(const KDims& d, const KTab& t, double* F, int radial, hipStream_t s);
hipError_t launch_filter_radial(const KDims& d, const KTab& t, double* F, bool transpose, hipStream_t s);
// backward-Euler radial solve of the split step: F := B_i F on every r line of
// direction node Theta_i (Bimp: [n_Th][NRP][KP], zero padded), in place
hipError_t launch_radial_implicit(const KDims& d, const KTab& t, const double* Bimp, double* F, hipStream_t s);
hipError_t launch_project(const KDims& d, const KTab& t, const KCoef& c, double* F, hipStream_t s);
hipError_t launch_diag(const KDims& d, const KTab& t, const double* F, double* partial, double r_in2,
                       double r_out2, double* out3, hipStream_t s);
size_t diag_partial_count(const KDims& d);
hipError_t launch_outflux(const KDims& d, const KTab& t, const double* F, double* j, hipStream_t s);
hipError_t launch_outflux_T(const KDims& d, const KTab& t, const double* jbar, double* out, hipStream_t s);

// mixed precision: FP32 column passes (input FP64 or FP32, T in FP32) and the
// split-bf16 radial MFMA pass
hipError_t launch_phi_mixed(const KDims& d, const KTab& t, const void* Y, bool y_f32, float* T, bool accum,
                            hipStream_t s);
hipError_t launch_theta_mixed(const KDims& d, const KTab& t, const void* Y, bool y_f32, float* T, bool accum,
                              hipStream_t s);
hipError_t launch_radial_bf16x3(const KDims& d, const KTab& t, const void* Y, bool y_f32, float* T, bool accum,
                                hipStream_t s);
// host: split of the padded radial matrix into three bf16 planes [3][NRP][KP3]
void build_radial_split(const HostTables& h, int n_r, std::vector<uint16_t>& out, int* KP3);
