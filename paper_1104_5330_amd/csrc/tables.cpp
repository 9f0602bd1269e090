// Host-side construction of nodes, differentiation matrices, quadrature weights
// and the per-direction coefficient tables, all in FP64.
//
// Nodes: Chebyshev-Gauss-Lobatto in r on the shell [r_in, r_out] (Sect. 4.1),
// half-shifted theta_l = (l + 1/2) pi / n_theta and Theta_i = (i + 1/2) pi / n_Theta
// (no node on a pole or on Theta = pi/2), equispaced phi and Phi.
#include <cmath>
#include <cstdio>

#include "sp6_internal.h"

namespace {

bool pow2_in(int v, int lo, int hi) {
  if (v < lo || v > hi) return false;
  return (v & (v - 1)) == 0;
}

// Periodic Fourier collocation derivative on L equispaced points:
// D_jk = (1/2) (-1)^(j-k) cot(pi (j - k) / L), D_jj = 0 (Nyquist mode mapped to 0).
std::vector<double> fourier_matrix(int L) {
  std::vector<double> D(size_t(L) * L, 0.0);
  for (int j = 0; j < L; ++j)
    for (int k = 0; k < L; ++k)
      if (j != k) {
        double sgn = ((j - k) & 1) ? -1.0 : 1.0;
        D[size_t(j) * L + k] = 0.5 * sgn / std::tan(M_PI * double(j - k) / double(L));
      }
  return D;
}

// Grid form of the exponential filter exp(-36 (|k| / (L/2))^36) on L points.
std::vector<double> filter_matrix(int L) {
  std::vector<double> F(size_t(L) * L, 0.0);
  for (int k = -(L / 2); k < L / 2; ++k) {
    double s = std::exp(-36.0 * std::pow(std::fabs(double(k)) / (0.5 * L), 36.0));
    for (int j = 0; j < L; ++j)
      for (int l = 0; l < L; ++l) F[size_t(j) * L + l] += s * std::cos(2.0 * M_PI * k * (j - l) / L) / L;
  }
  return F;
}

// Even/odd split of a centro-antisymmetric (derivative) or centro-symmetric
// (filter) L x L matrix D.  With e_j = v_j + v_{L-1-j}, o_j = v_j - v_{L-1-j}
// (j < h = L/2), p = A e and q = B o, where
//   A_ij = (D_ij + D_{i,L-1-j}) / 2,  B_ij = (D_ij - D_{i,L-1-j}) / 2,
// one gets (Dv)_i = p_i + q_i and (Dv)_{L-1-i} = q_i - p_i (centro-antisymmetric)
// or p_i - q_i (centro-symmetric): L^2 / 2 multiply-adds per line instead of L^2.
// Stored as A then B, row major.
std::vector<double> even_odd(const std::vector<double>& D, int L) {
  int h = L / 2;
  std::vector<double> ab(size_t(2) * h * h);
  for (int i = 0; i < h; ++i)
    for (int j = 0; j < h; ++j) {
      double dij = D[size_t(i) * L + j], dik = D[size_t(i) * L + (L - 1 - j)];
      ab[size_t(i) * h + j] = 0.5 * (dij + dik);
      ab[size_t(h) * h + size_t(i) * h + j] = 0.5 * (dij - dik);
    }
  return ab;
}

std::vector<double> fejer(int n) {
  std::vector<double> w(n);
  for (int i = 0; i < n; ++i) {
    double t = (i + 0.5) * M_PI / n, s = 1.0;
    for (int k = 1; k <= n / 2; ++k) s -= 2.0 * std::cos(2.0 * k * t) / (4.0 * k * k - 1.0);
    w[i] = s * 2.0 / n;
  }
  return w;
}

std::vector<double> clenshaw_curtis(int n_r) {
  int N = n_r - 1;
  std::vector<double> w(n_r);
  for (int j = 0; j < n_r; ++j) {
    double t = M_PI * j / N, s = 1.0;
    for (int k = 1; k <= N / 2; ++k) s -= ((2 * k == N) ? 1.0 : 2.0) * std::cos(2.0 * k * t) / (4.0 * k * k - 1.0);
    w[j] = s * ((j == 0 || j == N) ? 1.0 : 2.0) / N;
  }
  return w;
}

}  // namespace

// Kinds 0/1: derivative and filter tables, A then B row major (A[i][j] at i h + j);
// kinds 2/3: the same tables transposed (A[i][j] at j h + i), so that the
// entries of consecutive output pairs at one j are contiguous.
std::vector<double> build_line_tables() {
  std::vector<double> out;
  for (int kind = 0; kind < 4; ++kind)
    for (int L = 4; L <= 64; L *= 2) {
      std::vector<double> ab = even_odd((kind % 2) == 0 ? fourier_matrix(L) : filter_matrix(L), L);
      if (kind >= 2) {
        const int h = L / 2;
        std::vector<double> tr(ab.size());
        for (int half = 0; half < 2; ++half)
          for (int i = 0; i < h; ++i)
            for (int j = 0; j < h; ++j) tr[size_t(half) * h * h + size_t(j) * h + i] = ab[size_t(half) * h * h + size_t(i) * h + j];
        ab.swap(tr);
      }
      out.insert(out.end(), ab.begin(), ab.end());
    }
  return out;
}

std::string validate_desc(const sp6_desc& d, sp6_status* code) {
  char buf[256];
  *code = SP6_ERR_SHAPE;
  if (d.n_eps < 1) return "n_eps must be >= 1";
  if (d.n_r < 3 || d.n_r > SP6_MAX_NR) return "n_r must be in [3, 80]";
  if (!pow2_in(d.n_theta, 2, 32)) return "n_theta must be a power of two in [2, 32]";
  if (!pow2_in(d.n_Theta, 2, 32)) return "n_Theta must be a power of two in [2, 32]";
  if (!pow2_in(d.n_phi, 4, 64)) return "n_phi must be a power of two in [4, 64]";
  if (d.n_Phi != 2 * d.n_Theta) return "n_Phi must equal 2 * n_Theta";
  double P = double(d.n_eps) * d.n_r * d.n_theta * d.n_phi * d.n_Theta * d.n_Phi;
  if (P > 4.0e10) {
    std::snprintf(buf, sizeof buf, "grid of %.3g points is above the supported maximum 4e10", P);
    return buf;
  }
  // plane, column-group and tile counts are 32-bit in the kernels
  const double planes = double(d.n_eps) * d.n_r * d.n_theta * d.n_phi;
  if (planes > 2147483647.0) {
    std::snprintf(buf, sizeof buf, "%.3g (Theta, Phi) planes is above the supported maximum 2^31 - 1", planes);
    return buf;
  }
  *code = SP6_ERR_ARG;
  if (!(d.r_in > 0.0) || !(d.r_out > d.r_in) || !std::isfinite(d.r_out)) return "need 0 < r_in < r_out";
  if (d.precision != SP6_FP64 && d.precision != SP6_MIXED) return "precision must be SP6_FP64 or SP6_MIXED";
  if (d.bc != 0 && d.bc != 1) return "bc must be 0 or 1";
  if (d.scattering != 0 && d.scattering != 1) return "scattering must be 0 or 1";
  if (d.filter < 0 || d.filter > 2) return "filter must be 0, 1 or 2";
  *code = SP6_OK;
  return "";
}

std::vector<double> cgl_nodes(int n, double a, double b) {
  std::vector<double> x(n);
  for (int j = 0; j < n; ++j) x[j] = 0.5 * (a + b) - 0.5 * (b - a) * std::cos(M_PI * j / (n - 1));
  return x;
}

// Chebyshev-Gauss-Lobatto derivative, ascending nodes.  Off-diagonal entries
// (c_i / c_j) (-1)^(i+j) / (x_i - x_j) with the node difference in product form
// 2 sin(pi (i+j) / 2N) sin(pi (i-j) / 2N); the matrix is made exactly
// centro-antisymmetric and its diagonal is minus the off-diagonal row sum.
std::vector<double> cgl_derivative(int n, double a, double b) {
  const int N = n - 1;
  std::vector<double> D(size_t(n) * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      if (i == j) continue;
      double ci = (i == 0 || i == N) ? 2.0 : 1.0, cj = (j == 0 || j == N) ? 2.0 : 1.0;
      double dx = 2.0 * std::sin(M_PI * (i + j) / (2.0 * N)) * std::sin(M_PI * (i - j) / (2.0 * N));
      double sgn = ((i + j) & 1) ? -1.0 : 1.0;
      D[size_t(i) * n + j] = (ci / cj) * sgn / dx;
    }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      if (i == j || i * n + j > (N - i) * n + (N - j)) continue;  // each mirror pair once
      double p = D[size_t(i) * n + j], q = D[size_t(N - i) * n + (N - j)];
      double v = 0.5 * (p - q);
      D[size_t(i) * n + j] = v;
      D[size_t(N - i) * n + (N - j)] = -v;
    }
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int j = 0; j < n; ++j)
      if (j != i) s += D[size_t(i) * n + j];
    D[size_t(i) * n + i] = -s;
  }
  const double scale = 2.0 / (b - a);
  for (auto& v : D) v *= scale;
  return D;
}

void build_host_tables(const sp6_desc& d, HostTables& t) {
  const int nr = d.n_r, nth = d.n_theta, nph = d.n_phi, nTh = d.n_Theta, nPh = d.n_Phi;
  const int N = nr - 1;
  t.r = cgl_nodes(nr, d.r_in, d.r_out);
  t.theta.resize(nth);
  for (int l = 0; l < nth; ++l) t.theta[l] = (l + 0.5) * M_PI / nth;
  t.phi.resize(nph);
  for (int k = 0; k < nph; ++k) t.phi[k] = 2.0 * M_PI * k / nph;
  t.Theta.resize(nTh);
  for (int i = 0; i < nTh; ++i) t.Theta[i] = (i + 0.5) * M_PI / nTh;
  t.Phi.resize(nPh);
  for (int m = 0; m < nPh; ++m) t.Phi[m] = 2.0 * M_PI * m / nPh;

  // weights
  t.w_r = clenshaw_curtis(nr);
  for (auto& w : t.w_r) w *= 0.5 * (d.r_out - d.r_in);
  t.w_th = fejer(nth);
  t.w_Th = fejer(nTh);
  t.w_ph.assign(nph, 2.0 * M_PI / nph);
  t.w_Ph.assign(nPh, 2.0 * M_PI / nPh);

  t.Dr = cgl_derivative(nr, d.r_in, d.r_out);

  t.NRP = ((nr + 15) / 16) * 16;
  t.KP = ((nr + 3) / 4) * 4;
  t.Dpad.assign(size_t(t.NRP) * t.KP, 0.0);
  t.DpadT.assign(size_t(t.NRP) * t.KP, 0.0);
  for (int i = 0; i < nr; ++i)
    for (int j = 0; j < nr; ++j) {
      t.Dpad[size_t(i) * t.KP + j] = t.Dr[size_t(i) * nr + j];
      t.DpadT[size_t(i) * t.KP + j] = t.Dr[size_t(j) * nr + i];
    }

  // radial filter: exp(-36 (k/N)^36) on the Chebyshev interpolant of an r line,
  // Fr = V diag(s) V^-1 with V_jk = T_k(x_j) = (-1)^k cos(pi k j / N) on the
  // ascending nodes x_j = -cos(pi j / N), and the discrete orthogonality of the
  // CGL nodes for V^-1: (V^-1)_kj = 2 T_k(x_j) / (N c_k c_j), c_0 = c_N = 2, else 1
  {
    auto Tkj = [&](int k, int j) { return ((k & 1) ? -1.0 : 1.0) * std::cos(M_PI * double(k) * j / N); };
    auto c = [&](int i) { return (i == 0 || i == N) ? 2.0 : 1.0; };
    std::vector<double> Fr(size_t(nr) * nr, 0.0);
    for (int k = 0; k < nr; ++k) {
      const double sk = std::exp(-36.0 * std::pow(double(k) / N, 36.0)) * 2.0 / (N * c(k));
      for (int i = 0; i < nr; ++i) {
        const double a = Tkj(k, i) * sk;
        for (int j = 0; j < nr; ++j) Fr[size_t(i) * nr + j] += a * Tkj(k, j) / c(j);
      }
    }
    t.Fpad.assign(size_t(t.NRP) * t.KP, 0.0);
    t.FpadT.assign(size_t(t.NRP) * t.KP, 0.0);
    for (int i = 0; i < nr; ++i)
      for (int j = 0; j < nr; ++j) {
        t.Fpad[size_t(i) * t.KP + j] = Fr[size_t(i) * nr + j];
        t.FpadT[size_t(i) * t.KP + j] = Fr[size_t(j) * nr + i];
      }
  }

  // pointwise coefficient factors
  t.inv_r.resize(nr);
  for (int j = 0; j < nr; ++j) t.inv_r[j] = 1.0 / t.r[j];
  t.inv_sin_th.resize(nth);
  t.cot_th.resize(nth);
  for (int l = 0; l < nth; ++l) {
    t.inv_sin_th[l] = 1.0 / std::sin(t.theta[l]);
    t.cot_th[l] = std::cos(t.theta[l]) / std::sin(t.theta[l]);
  }
  t.sin_Th.resize(nTh);
  t.cos_Th.resize(nTh);
  t.wmean.resize(nTh);
  t.wflux.resize(nTh);
  for (int i = 0; i < nTh; ++i) {
    t.sin_Th[i] = std::sin(t.Theta[i]);
    t.cos_Th[i] = std::cos(t.Theta[i]);
    t.wmean[i] = t.w_Th[i] * (2.0 * M_PI / nPh) / (4.0 * M_PI);
    t.wflux[i] = t.cos_Th[i] > 0 ? t.w_Th[i] * (2.0 * M_PI / nPh) * t.cos_Th[i] : 0.0;
  }
  t.sin_Ph.resize(nPh);
  t.cos_Ph.resize(nPh);
  for (int m = 0; m < nPh; ++m) {
    t.sin_Ph[m] = std::sin(t.Phi[m]);
    t.cos_Ph[m] = std::cos(t.Phi[m]);
  }
  // particle number weights w_r r^2 w_theta (2 pi / n_phi) w_Theta (2 pi / n_Phi),
  // flux weights w_theta (2 pi / n_phi) w_Theta cos(Theta) (2 pi / n_Phi)
  t.qN.resize(size_t(nr) * nth * nTh);
  for (int j = 0; j < nr; ++j)
    for (int l = 0; l < nth; ++l)
      for (int i = 0; i < nTh; ++i)
        t.qN[(size_t(j) * nth + l) * nTh + i] = t.w_r[j] * t.r[j] * t.r[j] * t.w_th[l] * (2.0 * M_PI / nph) *
                                                 t.w_Th[i] * (2.0 * M_PI / nPh);
  t.qJ.resize(size_t(nth) * nTh);
  for (int l = 0; l < nth; ++l)
    for (int i = 0; i < nTh; ++i)
      t.qJ[size_t(l) * nTh + i] = t.w_th[l] * (2.0 * M_PI / nph) * t.w_Th[i] * t.cos_Th[i] * (2.0 * M_PI / nPh);
}
