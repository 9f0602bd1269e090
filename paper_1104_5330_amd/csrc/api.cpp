// C ABI of the 6D spectral transport hot path: handle management, host-side
// argument validation and the kernel sequences of apply_L, rhs, step and
// adjoint_step.  No exception crosses the interface.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "range_check.h"
#include "sp6_internal.h"

hipError_t launch_filter_columns(const KDims& d, const KTab& t, double* F, hipStream_t s);

namespace {

thread_local std::string g_err;

sp6_status fail(sp6_status code, const std::string& msg) {
  g_err = msg;
  return code;
}

sp6_status hip_fail(hipError_t e, const char* where) {
  std::string m = std::string(where) + ": " + hipGetErrorString(e);
  (void)hipGetLastError();
  return fail(SP6_ERR_HIP, m);
}

#define HIP_TRY(expr, where)                   \
  do {                                         \
    hipError_t _e = (expr);                    \
    if (_e != hipSuccess) return hip_fail(_e, where); \
  } while (0)

}  // namespace

struct sp6_grid_s {
  sp6_desc desc{};
  KDims d{};
  KTab t{};
  KCoef c{};
  HostTables h;
  hipStream_t stream = nullptr;
  int device = 0;
  std::vector<void*> allocs;
  size_t bytes = 0;
  bool coeffs_set = false;
  double* kappa = nullptr;
  double* sigma = nullptr;
  double* eta = nullptr;
  double* g_in = nullptr;
  double* g_out = nullptr;
  // scratch (allocated on first use)
  double* T = nullptr;
  double* Ybuf = nullptr;
  double* acc = nullptr;
  double* Y2 = nullptr;
  double* Y3 = nullptr;
  double* Y4 = nullptr;
  double* KB = nullptr;
  double* LACC = nullptr;
  double* diag_partial = nullptr;
  double* diag_out = nullptr;
  float* Yf = nullptr;
  float* Tf = nullptr;
  // backward-Euler radial matrices for the split step, [n_Theta][NRP][KP], and
  // the dt they were built for
  double* Bimp = nullptr;
  double imp_dt = 0.0;
  // device address of the fixed scratch of sp6_step_noalloc on this device
  void* noalloc = nullptr;
  // Fokker-Planck energy coupling: energy-node derivative [n_eps][n_eps] and
  // nodes, (M0, Q) per plane, and the emissivity with the source added
  bool fp_on = false;
  double fp_alpha = 0.0;
  double* fp_D = nullptr;
  double* fp_gam = nullptr;
  double* fp_mq = nullptr;
  double* fp_eta = nullptr;
  double* fp_mom = nullptr;  // adjoint: 20 moments and the masked sum per plane
  double* fp_C = nullptr;    // adjoint: 20 direction-polynomial coefficients per plane
  std::vector<double> fp_host;  // host copy of D and the nodes (source of the uploads)

  hipError_t alloc(void** p, size_t n) {
    hipError_t e = hipMalloc(p, n);
    if (e == hipSuccess) {
      allocs.push_back(*p);
      bytes += n;
    }
    return e;
  }
};

namespace {

template <typename T>
hipError_t upload(sp6_grid g, const std::vector<T>& v, const T** out) {
  void* p = nullptr;
  const size_t n = (v.empty() ? 1 : v.size()) * sizeof(T);
  hipError_t e = g->alloc(&p, n);
  if (e != hipSuccess) return e;
  if (!v.empty()) {
    e = hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, g->stream);
    if (e != hipSuccess) return e;
  }
  *out = static_cast<const T*>(p);
  return hipSuccess;
}

size_t state_bytes(const sp6_grid g) { return size_t(g->d.P) * sizeof(double); }

// the filter after a step (Sect. 4.2: F is prescribed at the inflow nodes, so
// with the inflow conditions on the filter is followed by the inflow values)
hipError_t filter_step(sp6_grid g, double* F) {
  hipError_t e = launch_filter(g->d, g->t, F, g->desc.filter == 2 ? 1 : 0, g->stream);
  if (e == hipSuccess && g->d.bc) e = launch_project(g->d, g->t, g->c, F, g->stream);
  return e;
}

// the transpose of the linear part of filter_step, in place: zero at the inflow
// nodes, then the transposed filter
hipError_t filter_step_T(sp6_grid g, double* x) {
  hipError_t e = hipSuccess;
  if (g->d.bc) {
    KCoef c0 = g->c;
    c0.g_in = nullptr;
    c0.g_out = nullptr;
    e = launch_project(g->d, g->t, c0, x, g->stream);
  }
  if (e == hipSuccess) e = launch_filter(g->d, g->t, x, g->desc.filter == 2 ? 2 : 0, g->stream);
  return e;
}

// sizes for the next theta-phi, radial or plane pass, with the traversal
// direction flipped from the previous such pass
const KDims& next_pass(sp6_grid g) {
  g->d.rev ^= 1;
  return g->d;
}

sp6_status check_grid(sp6_grid g) {
  if (!g) return fail(SP6_ERR_ARG, "grid handle is NULL");
  return SP6_OK;
}

// A device array of `bytes` bytes: non-null, 16-byte aligned, device memory, and
// [p, p + bytes) inside the one device allocation that contains p.  (A caching
// allocator hands out parts of larger allocations, so a buffer that is too
// short but followed by more of its allocation is not detected; one that runs
// past the allocation's end is.)
sp6_status check_dev(sp6_grid g, const void* p, size_t bytes, const char* name) {
  if (!p) return fail(SP6_ERR_ARG, std::string(name) + " is NULL");
  if (reinterpret_cast<uintptr_t>(p) % 16 != 0) return fail(SP6_ERR_ARG, std::string(name) + " is not 16-byte aligned");
  hipPointerAttribute_t attr;
  std::memset(&attr, 0, sizeof attr);
  hipError_t e = hipPointerGetAttributes(&attr, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(SP6_ERR_ARG, std::string(name) + " is not a device pointer");
  }
  if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged && attr.type != hipMemoryTypeUnified)
    return fail(SP6_ERR_ARG, std::string(name) + " is not device memory");
  if (attr.type == hipMemoryTypeDevice && attr.device != g->device)
    return fail(SP6_ERR_ARG, std::string(name) + " is on device " + std::to_string(attr.device) +
                                 ", the handle on device " + std::to_string(g->device));
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  e = hipMemGetAddressRange(&base, &size, const_cast<void*>(p));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(SP6_ERR_ARG, std::string(name) + ": the device allocation holding it could not be found");
  }
  if (!sp6_range_inside(reinterpret_cast<uintptr_t>(base), size, reinterpret_cast<uintptr_t>(p), bytes))
    return fail(SP6_ERR_ARG, std::string(name) + " is too small: " + std::to_string(bytes) +
                                 " bytes from it run past the end of its device allocation");
  return SP6_OK;
}

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  const char* x = static_cast<const char*>(a);
  const char* y = static_cast<const char*>(b);
  return x < y + nb && y < x + na;
}

sp6_status check_distinct(const void* a, const char* na, const void* b, const char* nb, size_t bytes_a,
                          size_t bytes_b) {
  if (a && b && overlap(a, bytes_a, b, bytes_b))
    return fail(SP6_ERR_ARG, std::string(na) + " and " + nb + " overlap");
  return SP6_OK;
}

// Optional per-launch timing: an event before the first launch and after every
// launch, all on the handle's stream; launch i of kernel class cls[i] spans
// events i and i + 1.
struct Timer {
  std::vector<hipEvent_t> ev;
  std::vector<int> cls;
  hipError_t mark(hipStream_t s, int c) {
    hipEvent_t e;
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return r;
    ev.push_back(e);
    if (c >= 0) cls.push_back(c);
    return hipEventRecord(e, s);
  }
  ~Timer() {
    for (auto e : ev) (void)hipEventDestroy(e);
  }
};

enum { KC_PHI = 0, KC_THETA = 1, KC_RADIAL = 2, KC_PLANE = 3, KC_FILTER = 4, KC_SPHERE = 5, KC_ENERGY = 6, KC_COUNT = 7 };

hipError_t ensure(sp6_grid g, double** p, size_t n) {
  if (*p) return hipSuccess;
  return g->alloc(reinterpret_cast<void**>(p), n);
}

hipError_t ensure_step_scratch(sp6_grid g) {
  hipError_t e = ensure(g, &g->T, state_bytes(g));
  if (e == hipSuccess) e = ensure(g, &g->Ybuf, state_bytes(g));
  if (e == hipSuccess) e = ensure(g, &g->acc, state_bytes(g));
  return e;
}

// the r, theta and phi terms of L Y (or of L^T for the transposed passes) into T
// (paired: Y and T in the paired in-plane order, for the fused theta-phi pass of
// the 32 x 64 sphere; the radial pass works column by column in either order)
hipError_t column_terms(sp6_grid g, const double* Y, uint32_t terms, bool transpose, bool mask_in,
                        double in_scale, bool* wrote, Timer* tm = nullptr, double* Tdst = nullptr,
                        bool paired = false) {
  hipError_t e = hipSuccess;
  bool acc = false;
  const double sg = transpose ? -1.0 : 1.0;
  double* T = Tdst ? Tdst : g->T;
  if (paired && !((terms & 6u) == 6u && paired_order_ok(g->d))) return hipErrorInvalidValue;
  if ((terms & 6u) == 6u && sphere_fusable(g->d, false)) {
    e = launch_sphere(next_pass(g), g->t, Y, T, sg, mask_in, in_scale, g->stream, paired);
    if (e == hipSuccess && tm) e = tm->mark(g->stream, KC_SPHERE);
    if (e != hipSuccess) return e;
    acc = true;
    terms &= ~6u;
  }
  if (terms & 4u) {
    e = launch_phi(g->d, g->t, Y, T, acc, sg, mask_in, in_scale, g->stream);
    if (e == hipSuccess && tm) e = tm->mark(g->stream, KC_PHI);
    if (e != hipSuccess) return e;
    acc = true;
  }
  if (terms & 2u) {
    e = launch_theta(g->d, g->t, Y, T, acc, sg, mask_in, in_scale, g->stream);
    if (e == hipSuccess && tm) e = tm->mark(g->stream, KC_THETA);
    if (e != hipSuccess) return e;
    acc = true;
  }
  if (terms & 1u) {
    e = launch_radial(next_pass(g), g->t, Y, T, acc, transpose, mask_in, in_scale, g->stream);
    if (e == hipSuccess && tm) e = tm->mark(g->stream, KC_RADIAL);
    if (e != hipSuccess) return e;
    acc = true;
  }
  *wrote = acc;
  return e;
}

// mixed path: the r, theta and phi terms of L Y in FP32 (Y stored in FP64 or FP32)
// (paired: the FP32 stage copy and T in the paired in-plane order)
hipError_t column_terms_mixed(sp6_grid g, const void* Y, bool y_f32, uint32_t terms, bool* wrote,
                              Timer* tm = nullptr, float* Tdst = nullptr, bool paired = false) {
  hipError_t e = hipSuccess;
  bool acc = false;
  float* Tf = Tdst ? Tdst : g->Tf;
  if (paired && !((terms & 6u) == 6u && y_f32 && paired_order_ok(g->d))) return hipErrorInvalidValue;
  if ((terms & 6u) == 6u && sphere_fusable(g->d, true)) {
    e = launch_sphere_mixed(next_pass(g), g->t, Y, y_f32, Tf, g->stream, paired);
    if (e == hipSuccess && tm) e = tm->mark(g->stream, KC_SPHERE);
    if (e != hipSuccess) return e;
    acc = true;
    terms &= ~6u;
  }
  if (terms & 4u) {
    e = launch_phi_mixed(g->d, g->t, Y, y_f32, Tf, acc, g->stream);
    if (e == hipSuccess && tm) e = tm->mark(g->stream, KC_PHI);
    if (e != hipSuccess) return e;
    acc = true;
  }
  if (terms & 2u) {
    e = launch_theta_mixed(g->d, g->t, Y, y_f32, Tf, acc, g->stream);
    if (e == hipSuccess && tm) e = tm->mark(g->stream, KC_THETA);
    if (e != hipSuccess) return e;
    acc = true;
  }
  if (terms & 1u) {
    e = launch_radial_bf16x3(next_pass(g), g->t, Y, y_f32, Tf, acc, g->stream);
    if (e == hipSuccess && tm) e = tm->mark(g->stream, KC_RADIAL);
    if (e != hipSuccess) return e;
    acc = true;
  }
  *wrote = acc;
  return e;
}

hipError_t ensure_f32(sp6_grid g, float** p) {
  if (*p) return hipSuccess;
  return g->alloc(reinterpret_cast<void**>(p), size_t(g->d.P) * sizeof(float));
}

// The coefficients of a right-hand side of the stage input Y: the handle's, or
// with the energy coupling on, with eta + sigma S(Y) as the emissivity
hipError_t rhs_coefs(sp6_grid g, const void* Y, bool y_f32, KCoef* c, Timer* tm = nullptr) {
  *c = g->c;
  if (!g->fp_on) return hipSuccess;
  hipError_t e = launch_fp_source(g->d, g->t, Y, y_f32, g->fp_D, g->fp_gam, g->fp_alpha, g->fp_mq, g->eta, g->sigma,
                                  g->fp_eta, g->stream);
  if (e == hipSuccess && tm) e = tm->mark(g->stream, KC_ENERGY);
  c->eta = g->fp_eta;
  return e;
}

sp6_status fp64_rhs_like(sp6_grid g, const double* F, double* out, int mode, uint32_t terms) {
  HIP_TRY(hipSetDevice(g->device), "hipSetDevice");
  const bool mixed = g->desc.precision == SP6_MIXED;
  bool wrote = false;
  if (mixed) {
    HIP_TRY(ensure_f32(g, &g->Tf), "allocate scratch");
    HIP_TRY(column_terms_mixed(g, F, false, terms, &wrote), "column passes");
  } else {
    HIP_TRY(ensure(g, &g->T, state_bytes(g)), "allocate scratch");
    HIP_TRY(column_terms(g, F, terms, false, false, 1.0, &wrote), "column passes");
  }
  StageArgs a{};
  a.mode = mode;
  a.Yin = F;
  a.mixed = mixed;
  a.yin_f32 = 0;
  a.T = wrote ? (mixed ? static_cast<const void*>(g->Tf) : static_cast<const void*>(g->T)) : nullptr;
  a.out = out;
  a.terms = terms;
  KCoef c = g->c;
  if (mode == PM_RHS) HIP_TRY(rhs_coefs(g, F, false, &c), "energy coupling");
  HIP_TRY(launch_plane(next_pass(g), g->t, c, a, g->stream), "plane pass");
  return SP6_OK;
}

sp6_status check_state_io(sp6_grid g, const void* in, const char* nin, const void* out, const char* nout) {
  const size_t B = state_bytes(g);
  sp6_status s = check_dev(g, in, B, nin);
  if (s) return s;
  s = check_dev(g, out, B, nout);
  if (s) return s;
  return check_distinct(in, nin, out, nout, B, B);
}

// Scratch of the RK4 step: T and (FP64 path) the stage buffer and accumulator,
// or (mixed path) the FP32 stage copy and T plus the FP64 accumulator
struct StepBufs {
  double* T = nullptr;
  double* Y = nullptr;
  double* acc = nullptr;
  float* Yf = nullptr;
  float* Tf = nullptr;
};

sp6_status run_steps(sp6_grid g, double* F, double dt, int32_t nsteps, Timer* tm, bool radial_implicit = false,
                     double* Ystages = nullptr, const StepBufs* given = nullptr);

}  // namespace

extern "C" {

const char* sp6_last_error(void) { return g_err.c_str(); }

sp6_status sp6_validate_desc(const sp6_desc* desc) {
  if (!desc) return fail(SP6_ERR_ARG, "desc is NULL");
  sp6_status code;
  std::string m = validate_desc(*desc, &code);
  if (code != SP6_OK) return fail(code, m);
  return SP6_OK;
}

// The line-operator tables live in constant memory, one copy per device and
// kernel file; they are written once per device per process.
static hipError_t init_device_tables(int device) {
  static std::mutex mu;
  static std::set<int> done;
  std::lock_guard<std::mutex> lock(mu);
  if (done.count(device)) return hipSuccess;
  const std::vector<double> tab = build_line_tables();
  hipError_t e = init_line_tables_columns(tab.data());
  if (e == hipSuccess) e = init_line_tables_plane(tab.data());
  if (e == hipSuccess) done.insert(device);
  return e;
}

sp6_status sp6_create(const sp6_desc* desc, void* hip_stream, sp6_grid* out) {
  if (!out) return fail(SP6_ERR_ARG, "out is NULL");
  *out = nullptr;
  sp6_status st = sp6_validate_desc(desc);
  if (st) return st;
  sp6_grid g = nullptr;
  try {
    g = new sp6_grid_s();
    g->desc = *desc;
    build_host_tables(*desc, g->h);
  } catch (...) {
    delete g;
    return fail(SP6_ERR_ALLOC, "host allocation failed");
  }
  g->stream = static_cast<hipStream_t>(hip_stream);
  hipError_t e = hipGetDevice(&g->device);
  if (e != hipSuccess) {
    delete g;
    return hip_fail(e, "hipGetDevice");
  }
  e = init_device_tables(g->device);
  if (e != hipSuccess) {
    delete g;
    return hip_fail(e, "copy line tables");
  }
  KDims& d = g->d;
  d.n_eps = desc->n_eps;
  d.n_r = desc->n_r;
  d.n_th = desc->n_theta;
  d.n_ph = desc->n_phi;
  d.n_Th = desc->n_Theta;
  d.n_Ph = desc->n_Phi;
  d.plane = d.n_Th * d.n_Ph;
  d.M = int64_t(d.n_th) * d.n_ph * d.plane;
  d.P = d.M * d.n_r * d.n_eps;
  d.nplanes = int64_t(d.n_eps) * d.n_r * d.n_th * d.n_ph;
  d.bc = desc->bc;
  d.scattering = desc->scattering;
  if ((e = hipDeviceGetAttribute(&d.ncu, hipDeviceAttributeMultiprocessorCount, g->device)) != hipSuccess) {
    delete g;
    return hip_fail(e, "hipDeviceGetAttribute");
  }
  if (d.ncu < 1) d.ncu = 1;
  if ((e = noalloc_scratch_ptr(g->device, &g->noalloc)) != hipSuccess) {
    delete g;
    return hip_fail(e, "scratch address of sp6_step_noalloc");
  }

  const HostTables& h = g->h;
  KTab& t = g->t;
#define UP(field) \
  if ((e = upload(g, h.field, &t.field)) != hipSuccess) goto fail_hip;
  UP(inv_r) UP(inv_sin_th) UP(cot_th) UP(sin_Th) UP(cos_Th) UP(sin_Ph) UP(cos_Ph) UP(wmean) UP(wflux)
  UP(Dpad) UP(DpadT) UP(Fpad) UP(FpadT) UP(qN) UP(qJ)
#undef UP
  t.KP = h.KP;
  t.NRP = h.NRP;
  if (desc->precision == SP6_MIXED) {
    std::vector<uint16_t> split;
    build_radial_split(h, desc->n_r, split, &t.KP3);
    if ((e = upload(g, split, &t.Dsplit)) != hipSuccess) goto fail_hip;
  }
  {
    const size_t cb = size_t(d.nplanes) * sizeof(double);
    const size_t gb = size_t(d.n_eps) * d.M * sizeof(double);
    if ((e = g->alloc(reinterpret_cast<void**>(&g->kappa), cb)) != hipSuccess) goto fail_hip;
    if ((e = g->alloc(reinterpret_cast<void**>(&g->sigma), cb)) != hipSuccess) goto fail_hip;
    if ((e = g->alloc(reinterpret_cast<void**>(&g->eta), cb)) != hipSuccess) goto fail_hip;
    if ((e = g->alloc(reinterpret_cast<void**>(&g->g_in), gb)) != hipSuccess) goto fail_hip;
    if ((e = g->alloc(reinterpret_cast<void**>(&g->g_out), gb)) != hipSuccess) goto fail_hip;
    if ((e = hipMemsetAsync(g->g_in, 0, gb, g->stream)) != hipSuccess) goto fail_hip;
    if ((e = hipMemsetAsync(g->g_out, 0, gb, g->stream)) != hipSuccess) goto fail_hip;
    if ((e = g->alloc(reinterpret_cast<void**>(&g->diag_partial), diag_partial_count(d) * sizeof(double))) != hipSuccess)
      goto fail_hip;
    if ((e = g->alloc(reinterpret_cast<void**>(&g->diag_out), size_t(3) * d.n_eps * sizeof(double))) != hipSuccess)
      goto fail_hip;
  }
  g->c.kappa = g->kappa;
  g->c.sigma = g->sigma;
  g->c.eta = g->eta;
  g->c.g_in = g->g_in;
  g->c.g_out = g->g_out;
  g->c.pc0 = 1.0;
  g->c.pc1 = 0.0;
  g->c.pc2 = 0.0;
  g->c.aniso = 0;
  // host tables must stay alive until the copies are done
  if ((e = hipStreamSynchronize(g->stream)) != hipSuccess) goto fail_hip;
  *out = g;
  return SP6_OK;
fail_hip : {
  sp6_status s = (e == hipErrorOutOfMemory) ? fail(SP6_ERR_ALLOC, "device allocation failed") : hip_fail(e, "sp6_create");
  (void)hipStreamSynchronize(g->stream);
  for (void* p : g->allocs) (void)hipFree(p);
  delete g;
  return s;
}
}

void sp6_destroy(sp6_grid g) {
  if (!g) return;
  (void)hipSetDevice(g->device);
  (void)hipStreamSynchronize(g->stream);
  for (void* p : g->allocs) (void)hipFree(p);
  delete g;
}

sp6_status sp6_set_stream(sp6_grid g, void* hip_stream) {
  if (sp6_status s = check_grid(g)) return s;
  g->stream = static_cast<hipStream_t>(hip_stream);
  return SP6_OK;
}

sp6_status sp6_get_nodes(sp6_grid g, double* r, double* theta, double* phi, double* Theta, double* Phi) {
  if (sp6_status s = check_grid(g)) return s;
  const HostTables& h = g->h;
  if (r) std::memcpy(r, h.r.data(), h.r.size() * sizeof(double));
  if (theta) std::memcpy(theta, h.theta.data(), h.theta.size() * sizeof(double));
  if (phi) std::memcpy(phi, h.phi.data(), h.phi.size() * sizeof(double));
  if (Theta) std::memcpy(Theta, h.Theta.data(), h.Theta.size() * sizeof(double));
  if (Phi) std::memcpy(Phi, h.Phi.data(), h.Phi.size() * sizeof(double));
  return SP6_OK;
}

sp6_status sp6_get_weights(sp6_grid g, double* w_r, double* w_theta, double* w_phi, double* w_Theta,
                           double* w_Phi) {
  if (sp6_status s = check_grid(g)) return s;
  const HostTables& h = g->h;
  if (w_r) std::memcpy(w_r, h.w_r.data(), h.w_r.size() * sizeof(double));
  if (w_theta) std::memcpy(w_theta, h.w_th.data(), h.w_th.size() * sizeof(double));
  if (w_phi) std::memcpy(w_phi, h.w_ph.data(), h.w_ph.size() * sizeof(double));
  if (w_Theta) std::memcpy(w_Theta, h.w_Th.data(), h.w_Th.size() * sizeof(double));
  if (w_Phi) std::memcpy(w_Phi, h.w_Ph.data(), h.w_Ph.size() * sizeof(double));
  return SP6_OK;
}

sp6_status sp6_set_coefficients(sp6_grid g, const double* kappa, const double* sigma, const double* eta) {
  if (sp6_status s = check_grid(g)) return s;
  const size_t cb = size_t(g->d.nplanes) * sizeof(double);
  if (sp6_status s = check_dev(g, kappa, cb, "kappa")) return s;
  if (sp6_status s = check_dev(g, sigma, cb, "sigma")) return s;
  if (sp6_status s = check_dev(g, eta, cb, "eta")) return s;
  HIP_TRY(hipSetDevice(g->device), "hipSetDevice");
  HIP_TRY(hipMemcpyAsync(g->kappa, kappa, cb, hipMemcpyDeviceToDevice, g->stream), "copy kappa");
  HIP_TRY(hipMemcpyAsync(g->sigma, sigma, cb, hipMemcpyDeviceToDevice, g->stream), "copy sigma");
  HIP_TRY(hipMemcpyAsync(g->eta, eta, cb, hipMemcpyDeviceToDevice, g->stream), "copy eta");
  g->coeffs_set = true;
  return SP6_OK;
}

sp6_status sp6_set_scattering_kernel(sp6_grid g, double c1, double c2) {
  if (sp6_status s = check_grid(g)) return s;
  if (!std::isfinite(c1) || !std::isfinite(c2)) return fail(SP6_ERR_ARG, "c1 and c2 must be finite");
  const double c0 = 1.0 - c2 / 3.0;
  auto p = [&](double mu) { return c0 + c1 * mu + c2 * mu * mu; };
  double pmin = std::min(p(-1.0), p(1.0));
  if (c2 > 0.0) {
    const double mu = -c1 / (2.0 * c2);
    if (mu > -1.0 && mu < 1.0) pmin = std::min(pmin, p(mu));
  }
  if (pmin < 0.0) return fail(SP6_ERR_ARG, "phase function p(mu) = c0 + c1 mu + c2 mu^2 is negative on [-1, 1]");
  g->c.pc0 = c0;
  g->c.pc1 = c1;
  g->c.pc2 = c2;
  g->c.aniso = (c1 != 0.0 || c2 != 0.0) ? 1 : 0;
  return SP6_OK;
}

sp6_status sp6_set_energy_coupling(sp6_grid g, int32_t enable, double gamma_min, double gamma_max, double alpha) {
  if (sp6_status s = check_grid(g)) return s;
  if (!enable) {
    g->fp_on = false;
    return SP6_OK;
  }
  if (!g->desc.scattering) return fail(SP6_ERR_STATE, "the energy coupling needs scattering = 1 (its source scales with sigma)");
  const int n = g->desc.n_eps;
  if (n < 2 || n > 64) return fail(SP6_ERR_SHAPE, "the energy coupling needs 2 <= n_eps <= 64 (Chebyshev nodes of gamma)");
  if (!(gamma_min >= 0.0) || !(gamma_max > gamma_min) || !std::isfinite(gamma_max))
    return fail(SP6_ERR_ARG, "need 0 <= gamma_min < gamma_max, finite");
  if (!(alpha >= 0.0) || !std::isfinite(alpha)) return fail(SP6_ERR_ARG, "alpha must be finite and >= 0");
  HIP_TRY(hipSetDevice(g->device), "hipSetDevice");
  const size_t pb = size_t(g->d.nplanes) * sizeof(double);
  HIP_TRY(ensure(g, &g->fp_D, size_t(n) * n * sizeof(double)), "allocate energy tables");
  HIP_TRY(ensure(g, &g->fp_gam, size_t(n) * sizeof(double)), "allocate energy tables");
  HIP_TRY(ensure(g, &g->fp_mq, 2 * pb), "allocate energy scratch");
  HIP_TRY(ensure(g, &g->fp_eta, pb), "allocate energy scratch");
  // the previous upload may still be in flight from the host copy
  HIP_TRY(hipStreamSynchronize(g->stream), "synchronise");
  g->fp_host = cgl_derivative(n, gamma_min, gamma_max);
  const std::vector<double> gam = cgl_nodes(n, gamma_min, gamma_max);
  g->fp_host.insert(g->fp_host.end(), gam.begin(), gam.end());
  HIP_TRY(hipMemcpyAsync(g->fp_D, g->fp_host.data(), size_t(n) * n * sizeof(double), hipMemcpyHostToDevice, g->stream),
          "upload energy tables");
  HIP_TRY(hipMemcpyAsync(g->fp_gam, g->fp_host.data() + size_t(n) * n, size_t(n) * sizeof(double),
                         hipMemcpyHostToDevice, g->stream),
          "upload energy tables");
  g->fp_alpha = alpha;
  g->fp_on = true;
  return SP6_OK;
}

sp6_status sp6_set_inflow(sp6_grid g, const double* g_in, const double* g_out) {
  if (sp6_status s = check_grid(g)) return s;
  const size_t gb = size_t(g->d.n_eps) * g->d.M * sizeof(double);
  if (g_in)
    if (sp6_status s = check_dev(g, g_in, gb, "g_in")) return s;
  if (g_out)
    if (sp6_status s = check_dev(g, g_out, gb, "g_out")) return s;
  HIP_TRY(hipSetDevice(g->device), "hipSetDevice");
  if (g_in)
    HIP_TRY(hipMemcpyAsync(g->g_in, g_in, gb, hipMemcpyDeviceToDevice, g->stream), "copy g_in");
  else
    HIP_TRY(hipMemsetAsync(g->g_in, 0, gb, g->stream), "clear g_in");
  if (g_out)
    HIP_TRY(hipMemcpyAsync(g->g_out, g_out, gb, hipMemcpyDeviceToDevice, g->stream), "copy g_out");
  else
    HIP_TRY(hipMemsetAsync(g->g_out, 0, gb, g->stream), "clear g_out");
  return SP6_OK;
}

sp6_status sp6_project_inflow(sp6_grid g, double* F) {
  if (sp6_status s = check_grid(g)) return s;
  if (sp6_status s = check_dev(g, F, state_bytes(g), "F")) return s;
  HIP_TRY(hipSetDevice(g->device), "hipSetDevice");
  HIP_TRY(launch_project(g->d, g->t, g->c, F, g->stream), "project inflow");
  return SP6_OK;
}

sp6_status sp6_apply_L_terms(sp6_grid g, uint32_t term_mask, const double* F, double* out) {
  if (sp6_status s = check_grid(g)) return s;
  if (term_mask == 0 || term_mask > 31u) return fail(SP6_ERR_ARG, "term_mask must be in [1, 31]");
  if (sp6_status s = check_state_io(g, F, "F", out, "out")) return s;
  return fp64_rhs_like(g, F, out, PM_APPLY, term_mask);
}

sp6_status sp6_apply_L(sp6_grid g, const double* F, double* LF) { return sp6_apply_L_terms(g, 31u, F, LF); }

sp6_status sp6_apply_LT(sp6_grid g, const double* G, double* out) {
  if (sp6_status s = check_grid(g)) return s;
  if (g->desc.precision != SP6_FP64) return fail(SP6_ERR_STATE, "apply_LT is FP64-only");
  if (sp6_status s = check_state_io(g, G, "G", out, "out")) return s;
  HIP_TRY(hipSetDevice(g->device), "hipSetDevice");
  HIP_TRY(ensure(g, &g->T, state_bytes(g)), "allocate scratch");
  bool wrote = false;
  HIP_TRY(column_terms(g, G, 7u, true, false, 1.0, &wrote), "transposed column passes");
  HIP_TRY(launch_plane_LT(g->d, g->t, G, g->T, out, g->stream), "transposed plane pass");
  return SP6_OK;
}

sp6_status sp6_rhs(sp6_grid g, const double* F, double* out) {
  if (sp6_status s = check_grid(g)) return s;
  if (!g->coeffs_set) return fail(SP6_ERR_STATE, "coefficients not set (call sp6_set_coefficients)");
  if (sp6_status s = check_state_io(g, F, "F", out, "out")) return s;
  return fp64_rhs_like(g, F, out, PM_RHS, 31u);
}

sp6_status sp6_apply_filter(sp6_grid g, double* F) {
  if (sp6_status s = check_grid(g)) return s;
  if (sp6_status s = check_dev(g, F, state_bytes(g), "F")) return s;
  HIP_TRY(hipSetDevice(g->device), "hipSetDevice");
  HIP_TRY(launch_filter(g->d, g->t, F, g->desc.filter == 2 ? 1 : 0, g->stream), "filter");
  return SP6_OK;
}

}  // extern "C"

namespace {

// the backward-Euler radial matrices (I + dt cos Theta_i D_r, inflow row replaced
// by the identity) inverted on the host by Gauss-Jordan elimination with partial
// pivoting, padded like the radial matrix, uploaded once per dt
sp6_status ensure_radial_implicit(sp6_grid g, double dt) {
  if (g->Bimp && g->imp_dt == dt) return SP6_OK;
  const HostTables& h = g->h;
  const int n = g->desc.n_r, nTh = g->desc.n_Theta;
  const size_t per = size_t(h.NRP) * h.KP;
  std::vector<double> pad(per * nTh, 0.0), A(size_t(n) * 2 * n);
  for (int i = 0; i < nTh; ++i) {
    const double c = h.cos_Th[i];
    const int brow = c > 0.0 ? 0 : n - 1;
    for (int r = 0; r < n; ++r)
      for (int k = 0; k < 2 * n; ++k) {
        double v = 0.0;
        if (k < n) {
          v = (r == k ? 1.0 : 0.0) + dt * c * h.Dr[size_t(r) * n + k];
          if (g->desc.bc && r == brow) v = (r == k) ? 1.0 : 0.0;
        } else {
          v = (k - n == r) ? 1.0 : 0.0;
        }
        A[size_t(r) * 2 * n + k] = v;
      }
    for (int col = 0; col < n; ++col) {
      int piv = col;
      for (int r = col + 1; r < n; ++r)
        if (std::fabs(A[size_t(r) * 2 * n + col]) > std::fabs(A[size_t(piv) * 2 * n + col])) piv = r;
      if (A[size_t(piv) * 2 * n + col] == 0.0) return fail(SP6_ERR_ARG, "backward-Euler radial matrix is singular for this dt");
      if (piv != col)
        for (int k = 0; k < 2 * n; ++k) std::swap(A[size_t(piv) * 2 * n + k], A[size_t(col) * 2 * n + k]);
      const double inv = 1.0 / A[size_t(col) * 2 * n + col];
      for (int k = 0; k < 2 * n; ++k) A[size_t(col) * 2 * n + k] *= inv;
      for (int r = 0; r < n; ++r) {
        if (r == col) continue;
        const double f = A[size_t(r) * 2 * n + col];
        if (f != 0.0)
          for (int k = 0; k < 2 * n; ++k) A[size_t(r) * 2 * n + k] -= f * A[size_t(col) * 2 * n + k];
      }
    }
    for (int r = 0; r < n; ++r)
      for (int k = 0; k < n; ++k) pad[per * i + size_t(r) * h.KP + k] = A[size_t(r) * 2 * n + n + k];
  }
  hipError_t e = hipSuccess;
  if (!g->Bimp) e = g->alloc(reinterpret_cast<void**>(&g->Bimp), pad.size() * sizeof(double));
  if (e == hipSuccess)
    e = hipMemcpyAsync(g->Bimp, pad.data(), pad.size() * sizeof(double), hipMemcpyHostToDevice, g->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(g->stream);  // pad is a local buffer
  HIP_TRY(e, "radial matrices");
  g->imp_dt = dt;
  return SP6_OK;
}

// Ystages (one step, FP64): the stage inputs Y2, Y3, Y4 are written there, back
// to back, instead of into the handle's stage buffer
sp6_status run_steps(sp6_grid g, double* F, double dt, int32_t nsteps, Timer* tm, bool radial_implicit,
                     double* Ystages, const StepBufs* given) {
  if (sp6_status s = check_grid(g)) return s;
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(SP6_ERR_ARG, "dt must be finite and > 0");
  if (nsteps < 0) return fail(SP6_ERR_ARG, "nsteps must be >= 0");
  if (!g->coeffs_set) return fail(SP6_ERR_STATE, "coefficients not set (call sp6_set_coefficients)");
  if (sp6_status s = check_dev(g, F, state_bytes(g), "F")) return s;
  if (nsteps == 0) return SP6_OK;
  HIP_TRY(hipSetDevice(g->device), "hipSetDevice");
  const bool mixed = g->desc.precision == SP6_MIXED;
  StepBufs b;
  if (given) {
    b = *given;
  } else {
    if (mixed) {
      HIP_TRY(ensure_f32(g, &g->Yf), "allocate scratch");
      HIP_TRY(ensure_f32(g, &g->Tf), "allocate scratch");
      HIP_TRY(ensure(g, &g->acc, state_bytes(g)), "allocate scratch");
    } else {
      HIP_TRY(ensure_step_scratch(g), "allocate scratch");
    }
    b.T = g->T, b.Y = g->Ybuf, b.acc = g->acc, b.Yf = g->Yf, b.Tf = g->Tf;
  }
  if (radial_implicit)
    if (sp6_status st = ensure_radial_implicit(g, dt)) return st;
  const KDims& d = g->d;
  const uint32_t cols = radial_implicit ? 6u : 7u;  // without the radial term in the split step
  // Stage buffers in the paired in-plane order on the 32 x 64 sphere: the stage
  // state, T and (FP64) the accumulator of stages 2 to 4 (the fused theta-phi pass
  // then moves one 64-byte run per tile row instead of two 32-byte runs; on the
  // mixed path the FP32 stage copy and T).  Not with stored stage states (the
  // adjoint reads them in the plain order) or the energy coupling (its moment
  // pass reads the stage states in the plain order).
  const bool paired = !Ystages && !g->fp_on && paired_order_ok(d) && d.n_Ph == 2 * d.n_Th;
  // and (FP64) F itself between the steps of one call (the last step writes it in
  // the plain order again), unless the filter runs between steps (its plane and
  // theta passes read the plain order)
  const bool keepF = paired && !mixed && !g->desc.filter;
  if (tm) HIP_TRY(tm->mark(g->stream, -1), "event");
  for (int32_t n = 0; n < nsteps; ++n) {
    const bool Fp = keepF && n > 0;  // F holds the paired order
    for (int s = 1; s <= 4; ++s) {
      bool wrote = false;
      StageArgs a{};
      a.mode = PM_STAGE;
      a.terms = cols | 24u;
      a.mixed = mixed;
      if (mixed) {
        // stage 1 reads the FP64 state; later stages the FP32 stage copy
        const void* Yin = (s == 1) ? static_cast<const void*>(F) : static_cast<const void*>(b.Yf);
        HIP_TRY(column_terms_mixed(g, Yin, s != 1, cols, &wrote, tm, b.Tf, paired && s > 1), "column passes");
        a.Yin = Yin;
        a.yin_f32 = s != 1;
        a.T = b.Tf;
        if (paired) a.pair_mode = s == 1 ? 1 : (s == 4 ? 3 : 2);
      } else {
        const double* Yin = (s == 1) ? F : (Ystages ? Ystages + size_t(s - 2) * size_t(d.P) : b.Y);
        HIP_TRY(column_terms(g, Yin, cols, false, false, 1.0, &wrote, tm, b.T, paired && (s > 1 || Fp)),
                "column passes");
        a.Yin = Yin;
        a.T = b.T;
        if (paired) {
          a.pair_mode = s == 1 ? (Fp ? 2 : 1) : (s == 4 ? 3 : 2);
          a.pair_all = s == 1 ? 1 : (s == 4 ? (keepF && n + 1 < nsteps) : Fp);
        }
      }
      void* ybuf = mixed ? static_cast<void*>(b.Yf) : static_cast<void*>(b.Y);
      if (Ystages && s <= 3) ybuf = Ystages + size_t(s - 1) * size_t(d.P);
      switch (s) {
        case 1:
          a.accsrc = nullptr, a.accdst = b.acc, a.cb = dt / 6.0;
          a.ysrc = nullptr, a.ynext = ybuf, a.cn = 0.5 * dt;
          // FP64: the accumulator is first written in stage 2, from F and
          // Y2 = F + dt/2 k1 (8 of 32 bytes per point)
          if (!mixed) a.accdst = nullptr;
          break;
        case 2:
          a.accsrc = b.acc, a.accdst = b.acc, a.cb = dt / 3.0;
          a.ysrc = F, a.ynext = ybuf, a.cn = 0.5 * dt;
          if (!mixed) a.accsrc = nullptr, a.accrec = 1;
          break;
        case 3:
          a.accsrc = b.acc, a.accdst = b.acc, a.cb = dt / 3.0;
          a.ysrc = F, a.ynext = ybuf, a.cn = dt;
          break;
        default:
          a.accsrc = b.acc, a.accdst = F, a.cb = dt / 6.0;
          a.ysrc = nullptr, a.ynext = nullptr, a.cn = 0.0;
          break;
      }
      KCoef c = g->c;
      HIP_TRY(rhs_coefs(g, a.Yin, mixed && a.yin_f32, &c, tm), "energy coupling");
      HIP_TRY(launch_plane(next_pass(g), g->t, c, a, g->stream), "plane pass");
      if (tm) HIP_TRY(tm->mark(g->stream, KC_PLANE), "event");
    }
    if (radial_implicit) {
      HIP_TRY(launch_radial_implicit(d, g->t, g->Bimp, F, g->stream), "radial solve");
      if (tm) HIP_TRY(tm->mark(g->stream, KC_RADIAL), "event");
    }
    if (g->desc.filter) {
      HIP_TRY(filter_step(g, F), "filter");
      if (tm) HIP_TRY(tm->mark(g->stream, KC_FILTER), "event");
    }
  }
  return SP6_OK;
}

}  // namespace

extern "C" {

sp6_status sp6_step(sp6_grid g, double* F, double dt, int32_t nsteps) { return run_steps(g, F, dt, nsteps, nullptr); }

sp6_status sp6_step_noalloc(sp6_grid g, double* F, double dt, int32_t nsteps) {
  if (sp6_status s = check_grid(g)) return s;
  const bool mixed = g->desc.precision == SP6_MIXED;
  const size_t P = size_t(g->d.P);
  auto up = [](size_t n) { return (n + 255) / 256 * 256; };
  const size_t need = mixed ? 2 * up(4 * P) + up(8 * P) : 3 * up(8 * P);
  if (need > SP6_NOALLOC_SCRATCH_BYTES)
    return fail(SP6_ERR_SHAPE, "sp6_step_noalloc: the step needs " + std::to_string(need) +
                                   " bytes of scratch, more than its fixed " +
                                   std::to_string(size_t(SP6_NOALLOC_SCRATCH_BYTES)) + " bytes");
  if (!g->noalloc) return fail(SP6_ERR_STATE, "sp6_step_noalloc: no scratch address on this device");
  char* base = static_cast<char*>(g->noalloc);
  StepBufs b;
  if (mixed) {
    b.Yf = reinterpret_cast<float*>(base);
    b.Tf = reinterpret_cast<float*>(base + up(4 * P));
    b.acc = reinterpret_cast<double*>(base + 2 * up(4 * P));
  } else {
    b.T = reinterpret_cast<double*>(base);
    b.Y = reinterpret_cast<double*>(base + up(8 * P));
    b.acc = reinterpret_cast<double*>(base + 2 * up(8 * P));
  }
  return run_steps(g, F, dt, nsteps, nullptr, false, nullptr, &b);
}

sp6_status sp6_step_stages(sp6_grid g, double* F, double dt, double* Ystages) {
  if (sp6_status s = check_grid(g)) return s;
  if (g->desc.precision != SP6_FP64) return fail(SP6_ERR_STATE, "sp6_step_stages needs an FP64 handle");
  const size_t B = state_bytes(g);
  if (sp6_status s = check_dev(g, F, B, "F")) return s;
  if (sp6_status s = check_dev(g, Ystages, 3 * B, "Ystages")) return s;
  if (sp6_status s = check_distinct(F, "F", Ystages, "Ystages", B, 3 * B)) return s;
  return run_steps(g, F, dt, 1, nullptr, false, Ystages);
}

sp6_status sp6_step_radial_implicit(sp6_grid g, double* F, double dt, int32_t nsteps) {
  return run_steps(g, F, dt, nsteps, nullptr, true);
}

sp6_status sp6_step_ab2(sp6_grid g, double* F, double* H, double dt, int32_t nsteps, int32_t start) {
  if (sp6_status s = check_grid(g)) return s;
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(SP6_ERR_ARG, "dt must be finite and > 0");
  if (nsteps < 0) return fail(SP6_ERR_ARG, "nsteps must be >= 0");
  if (start != 0 && start != 1) return fail(SP6_ERR_ARG, "start must be 0 or 1");
  if (g->desc.precision != SP6_FP64) return fail(SP6_ERR_STATE, "sp6_step_ab2 needs an FP64 handle");
  if (!g->coeffs_set) return fail(SP6_ERR_STATE, "coefficients not set (call sp6_set_coefficients)");
  if (sp6_status s = check_state_io(g, F, "F", H, "H")) return s;
  if (nsteps == 0) return SP6_OK;
  HIP_TRY(hipSetDevice(g->device), "hipSetDevice");
  HIP_TRY(ensure(g, &g->T, state_bytes(g)), "allocate scratch");
  const KDims& d = g->d;
  for (int32_t n = 0; n < nsteps; ++n) {
    bool wrote = false;
    HIP_TRY(column_terms(g, F, 7u, false, false, 1.0, &wrote), "column passes");
    // one plane pass: with k = rhs(F_n),
    //   first step: H = F + (dt/2) k, F = F + dt k
    //   later:      F = H + (3 dt/2) k, H = H + dt k
    StageArgs a{};
    a.mode = PM_STAGE;
    a.terms = 31u;
    a.Yin = F;
    a.T = wrote ? g->T : nullptr;
    a.accdst = H;
    a.ynext = F;
    if (start && n == 0) {
      a.accsrc = nullptr, a.cb = 0.5 * dt;
      a.ysrc = nullptr, a.cn = dt;
    } else {
      a.accsrc = H, a.cb = dt;
      a.ysrc = H, a.cn = 1.5 * dt;
    }
    KCoef c = g->c;
    HIP_TRY(rhs_coefs(g, F, false, &c), "energy coupling");
    HIP_TRY(launch_plane(next_pass(g), g->t, c, a, g->stream), "plane pass");
    if (g->desc.filter) {
      // H = F - (dt/2) k with k zero at the inflow nodes: H holds the inflow values too
      HIP_TRY(filter_step(g, F), "filter");
      HIP_TRY(filter_step(g, H), "filter of H");
    }
  }
  return SP6_OK;
}

sp6_status sp6_step_timed(sp6_grid g, double* F, double dt, int32_t nsteps, double* kernel_ms, int64_t* launches) {
  if (!kernel_ms || !launches) return fail(SP6_ERR_ARG, "kernel_ms and launches must not be NULL");
  Timer tm;
  sp6_status st = run_steps(g, F, dt, nsteps, &tm);
  if (st) return st;
  for (int c = 0; c < KC_COUNT; ++c) {
    kernel_ms[c] = 0.0;
    launches[c] = 0;
  }
  if (tm.ev.empty()) return SP6_OK;
  HIP_TRY(hipEventSynchronize(tm.ev.back()), "event synchronize");
  for (size_t i = 0; i < tm.cls.size(); ++i) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, tm.ev[i], tm.ev[i + 1]), "event elapsed");
    kernel_ms[tm.cls[i]] += ms;
    launches[tm.cls[i]] += 1;
  }
  return SP6_OK;
}

namespace {

// the discrete adjoint of one RK4 step; Ystages = null: recompute the stage
// inputs Y2, Y3, Y4 from F_n into scratch, else read them from Ystages
sp6_status adjoint_core(sp6_grid g, const double* Fn, const double* Ystages, double dt, double* lam, double* gk,
                        double* ge, double* gs) {
  if (sp6_status s = check_grid(g)) return s;
  if (g->desc.precision != SP6_FP64) return fail(SP6_ERR_STATE, "adjoint_step is FP64-only");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(SP6_ERR_ARG, "dt must be finite and > 0");
  if (!g->coeffs_set) return fail(SP6_ERR_STATE, "coefficients not set (call sp6_set_coefficients)");
  if (sp6_status s = check_state_io(g, Fn, "F_n", lam, "lam")) return s;
  if (Ystages) {
    const size_t B3 = 3 * state_bytes(g);
    if (sp6_status s = check_dev(g, Ystages, B3, "Ystages")) return s;
    if (sp6_status s = check_distinct(Ystages, "Ystages", Fn, "F_n", B3, state_bytes(g))) return s;
    if (sp6_status s = check_distinct(Ystages, "Ystages", lam, "lam", B3, state_bytes(g))) return s;
  }
  const size_t cb = size_t(g->d.nplanes) * sizeof(double);
  double* gr[3] = {gk, ge, gs};
  const char* gn[3] = {"grad_kappa", "grad_eta", "grad_sigma"};
  for (int i = 0; i < 3; ++i) {
    if (!gr[i]) continue;
    if (sp6_status s = check_dev(g, gr[i], cb, gn[i])) return s;
    if (sp6_status s = check_distinct(gr[i], gn[i], Fn, "F_n", cb, state_bytes(g))) return s;
    if (sp6_status s = check_distinct(gr[i], gn[i], lam, "lam", cb, state_bytes(g))) return s;
    for (int j = 0; j < i; ++j)
      if (sp6_status s = check_distinct(gr[i], gn[i], gr[j], gn[j], cb, cb)) return s;
    if (Ystages)
      if (sp6_status s = check_distinct(gr[i], gn[i], Ystages, "Ystages", cb, 3 * state_bytes(g))) return s;
  }
  HIP_TRY(hipSetDevice(g->device), "hipSetDevice");
  const size_t B = state_bytes(g);
  const size_t P = size_t(g->d.P);
  HIP_TRY(ensure(g, &g->T, B), "allocate scratch");
  if (!Ystages) {
    HIP_TRY(ensure(g, &g->Y2, B), "allocate scratch");
    HIP_TRY(ensure(g, &g->Y3, B), "allocate scratch");
    HIP_TRY(ensure(g, &g->Y4, B), "allocate scratch");
  }
  HIP_TRY(ensure(g, &g->KB, B), "allocate scratch");
  HIP_TRY(ensure(g, &g->LACC, B), "allocate scratch");
  if (g->fp_on) {
    HIP_TRY(ensure(g, &g->fp_mom, 21 * size_t(g->d.nplanes) * sizeof(double)), "allocate scratch");
    HIP_TRY(ensure(g, &g->fp_C, 20 * size_t(g->d.nplanes) * sizeof(double)), "allocate scratch");
  }
  const KDims& d = g->d;
  if (g->desc.filter) HIP_TRY(filter_step_T(g, lam), "transposed filter of lam");
  double* Ys[5] = {nullptr, const_cast<double*>(Fn), g->Y2, g->Y3, g->Y4};
  if (Ystages)
    for (int k = 0; k < 3; ++k) Ys[k + 2] = const_cast<double*>(Ystages) + k * P;
  // recompute the stage inputs Y2, Y3, Y4 from F_n (unless given)
  const double cn[4] = {0.0, 0.5 * dt, 0.5 * dt, dt};
  for (int s = 1; s <= 3 && !Ystages; ++s) {
    bool wrote = false;
    HIP_TRY(column_terms(g, Ys[s], 7u, false, false, 1.0, &wrote), "column passes");
    StageArgs a{};
    a.mode = PM_STAGE;
    a.Yin = Ys[s];
    a.T = g->T;
    a.terms = 31u;
    a.ysrc = (s == 1) ? nullptr : Fn;
    a.ynext = Ys[s + 1];
    a.cn = cn[s];
    KCoef c = g->c;
    HIP_TRY(rhs_coefs(g, Ys[s], false, &c), "energy coupling");
    HIP_TRY(launch_plane(next_pass(g), g->t, c, a, g->stream), "plane pass");
  }
  // transposed stages 4, 3, 2, 1
  for (int s = 4; s >= 1; --s) {
    const double* x = (s == 4) ? lam : g->KB;
    const double xs = (s == 4) ? dt / 6.0 : 1.0;
    bool wrote = false;
    HIP_TRY(column_terms(g, x, 7u, true, d.bc != 0, xs, &wrote), "transposed column passes");
    AdjArgs a{};
    a.x = x;
    a.xs = xs;
    a.T = g->T;
    a.Ys = Ys[s];
    a.gk = gk;
    a.ge = ge;
    a.gs = gs;
    a.lam_is_x = (s == 4);
    switch (s) {
      case 4:
        a.lam = lam, a.laccsrc = nullptr, a.laccdst = g->LACC, a.kbnext = g->KB, a.ka = dt / 3.0, a.kb = dt;
        break;
      case 3:
        a.lam = lam, a.laccsrc = g->LACC, a.laccdst = g->LACC, a.kbnext = g->KB, a.ka = dt / 3.0, a.kb = 0.5 * dt;
        break;
      case 2:
        a.lam = lam, a.laccsrc = g->LACC, a.laccdst = g->LACC, a.kbnext = g->KB, a.ka = dt / 6.0, a.kb = 0.5 * dt;
        break;
      default:
        a.lam = nullptr, a.laccsrc = g->LACC, a.laccdst = lam, a.kbnext = nullptr;
        break;
    }
    // energy coupling: the transpose of its linearisation at Y_s, formed from x
    // before the plane pass overwrites it (x and kbnext share KB), added after
    // it to the two outputs, which are linear in the stage's transposed result
    if (g->fp_on)
      HIP_TRY(launch_fp_adj(d, g->t, Ys[s], x, xs, g->fp_D, g->fp_gam, g->fp_alpha, g->fp_mom, g->sigma, g->fp_C, gs,
                            g->stream),
              "energy coupling (adjoint)");
    HIP_TRY(launch_plane_adj(d, g->t, g->c, a, g->stream), "transposed plane pass");
    if (g->fp_on)
      HIP_TRY(launch_fp_adj_apply(d, g->t, g->fp_C, a.laccdst, a.kbnext, a.kb, g->stream), "energy coupling (adjoint)");
  }
  return SP6_OK;
}

}  // namespace

sp6_status sp6_adjoint_step(sp6_grid g, const double* Fn, double dt, double* lam, double* gk, double* ge,
                            double* gs) {
  return adjoint_core(g, Fn, nullptr, dt, lam, gk, ge, gs);
}

sp6_status sp6_adjoint_step_stages(sp6_grid g, const double* Fn, const double* Ystages, double dt, double* lam,
                                   double* gk, double* ge, double* gs) {
  if (!Ystages) return fail(SP6_ERR_ARG, "Ystages is NULL");
  return adjoint_core(g, Fn, Ystages, dt, lam, gk, ge, gs);
}

sp6_status sp6_diagnostics(sp6_grid g, const double* F, double* N, double* J_in, double* J_out) {
  if (sp6_status s = check_grid(g)) return s;
  if (sp6_status s = check_dev(g, F, state_bytes(g), "F")) return s;
  HIP_TRY(hipSetDevice(g->device), "hipSetDevice");
  const double rin = g->h.r.front(), rout = g->h.r.back();
  HIP_TRY(launch_diag(g->d, g->t, F, g->diag_partial, rin * rin, rout * rout, g->diag_out, g->stream), "diagnostics");
  std::vector<double> host(size_t(3) * g->d.n_eps);
  HIP_TRY(hipMemcpyAsync(host.data(), g->diag_out, host.size() * sizeof(double), hipMemcpyDeviceToHost, g->stream),
          "copy diagnostics");
  HIP_TRY(hipStreamSynchronize(g->stream), "synchronize");
  for (int e = 0; e < g->d.n_eps; ++e) {
    if (N) N[e] = host[3 * e];
    if (J_in) J_in[e] = host[3 * e + 1];
    if (J_out) J_out[e] = host[3 * e + 2];
  }
  return SP6_OK;
}

sp6_status sp6_outgoing_flux(sp6_grid g, const double* F, double* j) {
  if (sp6_status s = check_grid(g)) return s;
  if (sp6_status s = check_dev(g, F, state_bytes(g), "F")) return s;
  const size_t jb = size_t(g->d.n_eps) * g->d.n_th * g->d.n_ph * sizeof(double);
  if (sp6_status s = check_dev(g, j, jb, "j")) return s;
  if (sp6_status s = check_distinct(F, "F", j, "j", state_bytes(g), jb)) return s;
  HIP_TRY(hipSetDevice(g->device), "hipSetDevice");
  HIP_TRY(launch_outflux(g->d, g->t, F, j, g->stream), "outgoing flux");
  return SP6_OK;
}

sp6_status sp6_outgoing_flux_T(sp6_grid g, const double* jbar, double* out) {
  if (sp6_status s = check_grid(g)) return s;
  const size_t jb = size_t(g->d.n_eps) * g->d.n_th * g->d.n_ph * sizeof(double);
  if (sp6_status s = check_dev(g, jbar, jb, "jbar")) return s;
  if (sp6_status s = check_dev(g, out, state_bytes(g), "out")) return s;
  if (sp6_status s = check_distinct(jbar, "jbar", out, "out", jb, state_bytes(g))) return s;
  HIP_TRY(hipSetDevice(g->device), "hipSetDevice");
  HIP_TRY(launch_outflux_T(g->d, g->t, jbar, out, g->stream), "outgoing flux transpose");
  return SP6_OK;
}

sp6_status sp6_device_bytes(sp6_grid g, size_t* bytes) {
  if (sp6_status s = check_grid(g)) return s;
  if (!bytes) return fail(SP6_ERR_ARG, "bytes is NULL");
  *bytes = g->bytes;
  return SP6_OK;
}

}  // extern "C"
