/*
 * sp6d.h - C ABI of the MI355X (gfx950) 6D spectral transport hot path.
 *
 * The library advances the radiative transport equation
 *     dF/dt + L_sph F = eta - (kappa + sigma) F + sigma <F>
 * on the doubly spherical grid (r, theta, phi) x (Theta, Phi) x eps of
 * Bonazzola, Vasset & Peres (2011):
 *   - L_sph is the Liouville operator in doubly spherical coordinates
 *     (Sect. 4.1, Eq. Liouvsph), with sin(Phi) in the two singular terms;
 *   - the right-hand side is the linear, coherent, isotropic collision term
 *     (Sect. 2.2 Eq. Transp with Sect. 3.1 Eqs. sigmadif and sigman at B = 0,
 *     the plasma density absorbed into kappa, sigma and eta, induced-process
 *     factors dropped), <F> being the angular mean over (Theta, Phi);
 *   - the discretisation is collocation: Chebyshev-Gauss-Lobatto in r on
 *     [r_in, r_out] (the shell of Sect. 4.1), Fourier in phi and Phi, and
 *     double-Fourier-sphere (DFS) lines in theta and Theta on half-shifted
 *     nodes theta_l = (l + 1/2) pi / n_theta, Theta_i = (i + 1/2) pi / n_Theta;
 *   - inflow conditions follow the characteristic analysis of Sect. 4.2
 *     (Eq. Sphedif): F is prescribed at r_in where cos(Theta) > 0 and at r_out
 *     where cos(Theta) < 0, and the right-hand side is zero at those nodes;
 *   - time stepping is classical RK4 (the paper uses Adams-Bashforth 2,
 *     Sect. 5.1); the discrete adjoint of the RK4 step is provided.
 *
 * Conventions shared by every entry point:
 *   - States are FP64 device arrays in C order [eps][r][theta][phi][Theta][Phi]
 *     (Phi fastest), owned by the caller, 16-byte aligned, never aliased with
 *     another array argument of the same call, and (device memory) on the
 *     handle's GPU.
 *   - Coefficient fields (kappa, sigma, eta, gradients) are FP64 device arrays
 *     [eps][r][theta][phi] (isotropic, one value per (Theta, Phi) plane).
 *   - All device work is enqueued on the handle's HIP stream; only
 *     sp6_diagnostics (host outputs) and sp6_destroy synchronise.
 *   - Arguments are validated on the host before anything is enqueued; a
 *     failing call returns a non-zero status, enqueues nothing and leaves every
 *     buffer untouched.  sp6_last_error() then describes the failure.
 *   - A handle is not thread safe; distinct handles are independent.
 *   - No C++ exception crosses this interface.
 */
#ifndef SP6D_H
#define SP6D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sp6_grid_s* sp6_grid; /* opaque; created and freed by the library */

typedef enum {
  SP6_OK = 0,
  SP6_ERR_ARG = 1,   /* null/misaligned/aliased pointer, bad scalar argument */
  SP6_ERR_SHAPE = 2, /* grid sizes outside the supported set */
  SP6_ERR_ALLOC = 3, /* device allocation failed */
  SP6_ERR_HIP = 4,   /* a HIP runtime call failed; message in sp6_last_error */
  SP6_ERR_STATE = 5  /* call not allowed in the handle's current state/mode */
} sp6_status;

enum { SP6_FP64 = 0, SP6_MIXED = 1 };

/* Grid and physics switches.
 * Supported sizes: 1 <= n_eps; 3 <= n_r <= 80; n_theta, n_Theta in
 * {2, 4, 8, 16, 32}; n_phi in {4, 8, 16, 32, 64}; n_Phi == 2 * n_Theta;
 * 0 < r_in < r_out.  Any other combination returns SP6_ERR_SHAPE. */
typedef struct {
  int32_t n_eps, n_r, n_theta, n_phi, n_Theta, n_Phi;
  double r_in, r_out;
  int32_t precision;  /* SP6_FP64, or SP6_MIXED: derivative passes in FP32 (radial
                         matrix as split-bf16 MFMA with FP32 accumulation), RK
                         accumulation, inflow handling and filter in FP64 */
  int32_t bc;         /* 0: no inflow mask (exactness tests); 1: inflow injection */
  int32_t scattering; /* 0/1: include sigma (<F> - F) */
  int32_t filter;     /* 0: off; 1: exponential filter exp(-36 (|k|/k_max)^36) on every
                         theta, phi, Theta and Phi line after each RK4 step (the
                         paper only mentions coefficient-space viscosity, App. B);
                         2: the same, then on the Chebyshev expansion of every r
                         line (the paper treats the radial discontinuity of its
                         shell problem, Sect. 5.3, by finite differences) */
} sp6_desc;

/* Host-only check of a descriptor (no GPU needed).  SP6_OK if sp6_create would
 * accept it. */
sp6_status sp6_validate_desc(const sp6_desc* desc);

/* Create a handle: builds the node/matrix/weight tables on the host in FP64,
 * allocates tables and scratch on the current HIP device (about 3 state-sized
 * FP64 arrays for sp6_step, 6 for sp6_adjoint_step, allocated on first use) and
 * copies the tables on `hip_stream` (NULL = default stream).  Coefficients start
 * unset; inflow planes start at zero. */
sp6_status sp6_create(const sp6_desc* desc, void* hip_stream, sp6_grid* out);

/* Free everything the handle owns; NULL-safe; synchronises its stream first. */
void sp6_destroy(sp6_grid grid);

sp6_status sp6_set_stream(sp6_grid grid, void* hip_stream);

/* Message of the last failure on the calling thread ("" if none). */
const char* sp6_last_error(void);

/* Host arrays of sizes n_r, n_theta, n_phi, n_Theta, n_Phi; any may be NULL. */
sp6_status sp6_get_nodes(sp6_grid grid, double* r, double* theta, double* phi, double* Theta,
                         double* Phi);
/* Quadrature weights used by the diagnostics and the angular mean: Clenshaw-Curtis
 * in r (for dr), Fejer's first rule in cos(theta) and cos(Theta), trapezoid in phi
 * and Phi.  Host arrays as in sp6_get_nodes. */
sp6_status sp6_get_weights(sp6_grid grid, double* w_r, double* w_theta, double* w_phi,
                           double* w_Theta, double* w_Phi);

/* Copy kappa (absorption), sigma (total scattering opacity) and eta (emission),
 * each [n_eps][n_r][n_theta][n_phi] on the device, into library storage (stream
 * ordered; the caller may reuse its buffers afterwards). */
sp6_status sp6_set_coefficients(sp6_grid grid, const double* kappa, const double* sigma,
                                const double* eta);

/* Phase function of coherent scattering (Eq. sigmadif): the in-scattered term is
 * sigma (K F)(omega) with (K F)(omega) = sum over the (Theta, Phi) nodes omega' of
 * w(omega') p(omega . omega') F(omega'), w = w_i (2 pi / n_Phi) / (4 pi) (Fejer
 * weights in cos Theta), and p(mu) = c0 + c1 mu + c2 mu^2 with c0 = 1 - c2 / 3, so
 * that p averages to one over the sphere and sigma is the total scattering
 * opacity.  c1 = c2 = 0 (the default) is isotropic scattering (Eq. sigman with
 * B = 0); Eq. sigman gives c1 = B / A (Eqs. crossnun, crossnup: -1/3 neutrons,
 * -1/10 protons); Thomson scattering (Eq. sigmaTh, normalised as the kernel of
 * App. B, Eq. speccons) is c1 = 0, c2 = 3/4.  Takes effect on handles created with
 * scattering = 1, for sp6_rhs, sp6_step and sp6_adjoint_step.  SP6_ERR_ARG if c1 or
 * c2 is not finite or p is negative somewhere on [-1, 1]; the handle keeps its
 * previous kernel then. */
sp6_status sp6_set_scattering_kernel(sp6_grid grid, double c1, double c2);

/* Fokker-Planck energy coupling (Sect. 3.2, Eq. Transpfp).  enable = 1: the n_eps
 * energy groups are taken as the Chebyshev-Gauss-Lobatto nodes gamma_k of
 * [gamma_min, gamma_max] (ascending, k = 0 first), and every right-hand side of
 * sp6_rhs and the RK4 steps (sp6_step, _stages, _noalloc, _timed,
 * _radial_implicit; FP64 and mixed) gains, per (eps, r, theta, phi) plane, the
 * isotropic source
 *   sigma S,  S = (1/4pi) d/dgamma [alpha gamma^2 dM0/dgamma + (gamma^2 - 2 alpha gamma) M0]
 *               + 3/(128 pi^2) dQ/dgamma,
 *   M0 = int F dw,  Q = int int (1 - mu + mu^2 - mu^3) F(w') F(w'') dw' dw'',
 * gamma derivatives by Chebyshev collocation across the groups, angular integrals
 * by the plane quadrature (Fejer in cos Theta, uniform in Phi).  sigma is the
 * handle's scattering coefficient (n sigma_Th); with the Thomson kernel
 * (sp6_set_scattering_kernel(grid, 0, 0.75)) the right-hand side is Eq.
 * (Transpfp).  The sign is the one for which the energy diffusion runs forward
 * and the Bose distribution of Eq. (Bose) is steady; the printed Eq. (Kompa) has
 * the opposite overall sign.  The source is added to eta, so it is zero at the
 * inflow nodes with the rest of the right-hand side; sp6_step_ab2 takes it too.
 * On the mixed path the moment pass reads the FP32 stage copy; the source is
 * formed in FP64.  sp6_adjoint_step(_stages) then transpose the step's
 * linearisation at its stage inputs (the source is nonlinear in F), and the
 * sigma gradient includes the source.  enable = 0 turns it off (the other
 * arguments are ignored).  Needs a handle created with scattering = 1
 * (SP6_ERR_STATE), 2 <= n_eps <= 64 (SP6_ERR_SHAPE), 0 <= gamma_min < gamma_max
 * and alpha >= 0, finite (SP6_ERR_ARG).  Allocates three per-plane device arrays
 * on first use, and two more on the first adjoint step with the coupling on;
 * the stepping calls themselves allocate nothing for it. */
sp6_status sp6_set_energy_coupling(sp6_grid grid, int32_t enable, double gamma_min, double gamma_max,
                                   double alpha);

/* Inflow planes [n_eps][n_theta][n_phi][n_Theta][n_Phi] at r_in and r_out (device);
 * only the incoming half (cos Theta > 0 at r_in, < 0 at r_out) is used.
 * NULL sets that plane to zero. */
sp6_status sp6_set_inflow(sp6_grid grid, const double* g_in, const double* g_out);

/* F := inflow values at the inflow nodes (the t = 0 projection). */
sp6_status sp6_project_inflow(sp6_grid grid, double* F);

/* LF = L_sph F (Eq. Liouvsph) at every node; no collision term, no mask. */
sp6_status sp6_apply_L(sp6_grid grid, const double* F, double* LF);

/* Sum of a subset of the five terms of Eq. (Liouvsph): bit 0 r, bit 1 theta,
 * bit 2 phi, bit 3 Theta, bit 4 Phi (for per-term checks). */
sp6_status sp6_apply_L_terms(sp6_grid grid, uint32_t term_mask, const double* F, double* out);

/* out = L^T G, the exact transpose of sp6_apply_L as a matrix on nodal values.
 * FP64 handles only (SP6_ERR_STATE on a mixed handle). */
sp6_status sp6_apply_LT(sp6_grid grid, const double* G, double* out);

/* out = -L F + eta - (kappa + sigma) F + sigma <F>, zero at inflow nodes when
 * bc = 1 (sigma terms only when scattering = 1).  Needs coefficients. */
sp6_status sp6_rhs(sp6_grid grid, const double* F, double* out);

/* nsteps >= 0 classical RK4 steps of size dt > 0, in place on F (then the
 * filter if enabled).  Needs coefficients.  F is in the C-order state layout when the
 * call returns; between the steps of one call on the 32 x 64 position sphere
 * (FP64, no filter, no energy coupling) it is held with every Theta row of a
 * plane reordered, so after an error mid-call its contents are unspecified. */
sp6_status sp6_step(sp6_grid grid, double* F, double dt, int32_t nsteps);

/* nsteps >= 0 steps of the split scheme of App. B, in place on F: one RK4 step of
 * size dt for the angular terms and the collision term (the radial term left
 * out), then the radial term by a backward-Euler step, F := B_i F along every r
 * line of direction node Theta_i, B_i = (I + dt cos(Theta_i) D_r)^-1 with the
 * inflow row (r_in if cos > 0, r_out if cos < 0) replaced by the identity when
 * bc = 1; then the filter if enabled.  The radial term sets no step limit.  The
 * B_i are built on the host (Gauss-Jordan, partial pivoting) and kept on the
 * device for the last dt used (n_Theta n_r^2 doubles, padded).  SP6_ERR_ARG if a
 * matrix is singular.  Needs coefficients. */
sp6_status sp6_step_radial_implicit(sp6_grid grid, double* F, double dt, int32_t nsteps);

/* nsteps >= 0 steps of the second-order Adams-Bashforth scheme the paper uses
 * (Sect. 5.1), in place on F: F_{n+1} = F_n + dt (3/2 k_n - 1/2 k_{n-1}),
 * k_n = right-hand side at F_n.  H (device, state layout, caller-owned, distinct
 * from F) carries the history H_n = F_n - (dt/2) k_{n-1} between calls:
 * start = 1 takes the first step with k_{-1} = k_0 (forward Euler) and
 * initialises H; start = 0 continues from H (same dt as the call that wrote it).
 * With the filter enabled it acts on F and H after every step.  One right-hand
 * side evaluation per step.  FP64 handles only (SP6_ERR_STATE on a mixed
 * handle); needs coefficients. */
sp6_status sp6_step_ab2(sp6_grid grid, double* F, double* H, double dt, int32_t nsteps, int32_t start);

/* Same as sp6_step, with a HIP event recorded on the handle's stream before the
 * first launch and after every kernel launch.  On return (the stream is
 * synchronised) kernel_ms[c] holds the summed duration and launches[c] the number
 * of launches of kernel class c: 0 phi pass, 1 theta pass, 2 radial pass, 3 plane
 * pass (Theta, Phi, collision, inflow, RK stage), 4 filter, 5 theta and phi
 * passes fused into one (used when n_phi = 2 n_theta <= 32, and for n_theta = 32,
 * n_phi = 64, n_Phi >= 16), 6 energy-coupling source (sp6_set_energy_coupling).
 * Both arrays are host arrays of 7 entries.  For measurement only. */
sp6_status sp6_step_timed(sp6_grid grid, double* F, double dt, int32_t nsteps, double* kernel_ms,
                          int64_t* launches);

/* Discrete adjoint of one sp6_step(F_n, dt, 1).  lam: in dLoss/dF_{n+1}, out
 * dLoss/dF_n (in place).  grad_kappa/eta/sigma ([n_eps][n_r][n_theta][n_phi],
 * device) are ACCUMULATED (+=) with d(F_{n+1}) / d(coefficient) applied to lam;
 * any may be NULL.  F_n is the state at the start of the step (read only).
 * FP64 handles only. */
sp6_status sp6_adjoint_step(sp6_grid grid, const double* F_n, double dt, double* lam,
                            double* grad_kappa, double* grad_eta, double* grad_sigma);

/* One sp6_step(F, dt, 1) that also keeps its stage inputs: Ystages (device,
 * 3 state arrays back to back, caller-owned, distinct from F) receives Y2, Y3,
 * Y4 = F_n + (dt/2) k1, F_n + (dt/2) k2, F_n + dt k3.  F is advanced exactly as by
 * sp6_step.  FP64 handles only.  For sp6_adjoint_step_stages. */
sp6_status sp6_step_stages(sp6_grid grid, double* F, double dt, double* Ystages);

/* sp6_adjoint_step with the stage inputs of the step read from Ystages (as
 * written by sp6_step_stages from the same F_n, dt and coefficients) instead of
 * recomputed: three fewer stage evaluations.  Same results as
 * sp6_adjoint_step. */
sp6_status sp6_adjoint_step_stages(sp6_grid grid, const double* F_n, const double* Ystages, double dt, double* lam,
                                   double* grad_kappa, double* grad_eta, double* grad_sigma);

/* Apply the spectral filter once, in place: the angular line filters, and the
 * radial one when desc.filter = 2 (desc.filter = 0 still applies the angular
 * filters). */
sp6_status sp6_apply_filter(sp6_grid grid, double* F);

/* Particle number N (App. A Eq. Npho) and fluxes through r_in and r_out
 * (Eq. Flux), host arrays [n_eps].  Synchronises the stream. */
sp6_status sp6_diagnostics(sp6_grid grid, const double* F, double* N, double* J_in,
                           double* J_out);

/* Outgoing-flux map j[eps][theta][phi] (device) at r_out: the sum over
 * cos(Theta_i) > 0 and Phi_m of w_i (2 pi / n_Phi) cos(Theta_i) F. */
sp6_status sp6_outgoing_flux(sp6_grid grid, const double* F, double* j);

/* Transpose of sp6_outgoing_flux (for the gradient of a flux loss): out is a
 * device state array, zero everywhere except at r_out, where
 * out[eps][theta][phi][i][m] = jbar[eps][theta][phi] w_i (2 pi / n_Phi) cos(Theta_i)
 * for cos(Theta_i) > 0 (and 0 otherwise).  jbar: device [n_eps][n_theta][n_phi]. */
sp6_status sp6_outgoing_flux_T(sp6_grid grid, const double* jbar, double* out);

/* Size of the fixed device scratch of sp6_step_noalloc, per GPU. */
#define SP6_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)

/* sp6_step without any device allocation, for callers that cannot allocate
 * (code under HIP graph capture before a handle's first step, serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, kernels and results as
 * sp6_step; the step's scratch (FP64: T, stage buffer and accumulator, 24 bytes
 * per point; mixed: FP32 stage copy and T plus the FP64 accumulator, 16 bytes
 * per point) lives in one fixed array of SP6_NOALLOC_SCRATCH_BYTES per GPU inside
 * the library (looked up by sp6_create), so FP64 handles of up to 11,184,810
 * points and mixed handles of up to 16,777,216 points are accepted; larger ones
 * return SP6_ERR_SHAPE.  Every call on a GPU shares that GPU's array, which keeps
 * the last call's contents (nothing in it needs to start at zero): calls that
 * overlap on one GPU (other streams, other threads, other handles) race and
 * must be serialised by the caller.  Needs coefficients. */
sp6_status sp6_step_noalloc(sp6_grid grid, double* F, double dt, int32_t nsteps);

/* Bytes of device memory the handle currently holds. */
sp6_status sp6_device_bytes(sp6_grid grid, size_t* bytes);

#ifdef __cplusplus
}
#endif

#endif /* SP6D_H */
