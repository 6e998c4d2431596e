// Host float64 tables of the B-spline / collocation discretisation.
//
// B-spline values use the Cox-de Boor recursion on the nonzero span (the
// paper expands S, p and the test functions in order-r, C^(r-1) B-splines on
// a uniform mesh); integrals use (r+1)-point Gauss-Legendre rules per
// element, exact for the degree-2r integrands of the mass matrix (eq. 14) and
// of the projection of a piecewise-linear nodal field.
#include "tables.h"

#include <cmath>
#include <cstdio>

namespace crv {

static double knot(int ne, int r, int k) {
  // open uniform knot vector: r+1 zeros, e/Ne, r+1 ones
  if (k <= r) return 0.0;
  if (k >= ne + r) return 1.0;
  return double(k - r) / double(ne);
}

void gauss_rule01(int npts, std::vector<double>& x, std::vector<double>& w) {
  // roots of the Legendre polynomial P_n by Newton's method on the three-term
  // recurrence, mapped from [-1,1] to [0,1]
  x.assign(npts, 0.0);
  w.assign(npts, 0.0);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < npts; ++i) {
    double z = std::cos(pi * (i + 0.75) / (npts + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= npts; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (npts == 1) { p1 = z; p0 = 1.0; }
      dp = npts * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= npts; ++k) {
      double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    if (npts == 1) { p1 = z; p0 = 1.0; }
    dp = npts * (z * p1 - p0) / (z * z - 1.0);
    double wt = 2.0 / ((1.0 - z * z) * dp * dp);
    // ascending order on [0,1]
    x[npts - 1 - i] = 0.5 * (1.0 + z);
    w[npts - 1 - i] = 0.5 * wt;
  }
}

void local_basis(int ne, int r, double x, double* val, double* der, int* first) {
  int e = int(std::floor(x * ne));
  if (e >= ne) e = ne - 1;
  if (e < 0) e = 0;
  const int s = e + r;  // knot span index: knot(s) <= x < knot(s+1)
  // degree-0: only N_{s,0} = 1; build up the r+1 nonzero functions
  // N_{s-k..s, k} for k = 1..r, keeping the degree r-1 values for derivatives
  double n[8] = {1.0, 0, 0, 0, 0, 0, 0, 0};
  double nprev[8] = {0};
  for (int k = 1; k <= r; ++k) {
    if (k == r)
      for (int j = 0; j < r; ++j) nprev[j] = n[j];
    double nn[8] = {0};
    // entry j corresponds to global index s-k+j
    for (int j = 0; j <= k; ++j) {
      const int i = s - k + j;
      double v = 0.0;
      // (x - t_i)/(t_{i+k} - t_i) N_{i,k-1}: N_{i,k-1} is entry j-1 of level k-1
      if (j >= 1) {
        double den = knot(ne, r, i + k) - knot(ne, r, i);
        if (den > 0) v += (x - knot(ne, r, i)) / den * n[j - 1];
      }
      // (t_{i+k+1} - x)/(t_{i+k+1} - t_{i+1}) N_{i+1,k-1}: entry j of level k-1
      if (j <= k - 1) {
        double den = knot(ne, r, i + k + 1) - knot(ne, r, i + 1);
        if (den > 0) v += (knot(ne, r, i + k + 1) - x) / den * n[j];
      }
      nn[j] = v;
    }
    for (int j = 0; j <= k; ++j) n[j] = nn[j];
  }
  for (int j = 0; j <= r; ++j) val[j] = n[j];
  if (der) {
    for (int j = 0; j <= r; ++j) {
      const int i = s - r + j;
      double d = 0.0;
      if (r == 0) { der[j] = 0.0; continue; }
      if (j >= 1) {
        double den = knot(ne, r, i + r) - knot(ne, r, i);
        if (den > 0) d += r / den * nprev[j - 1];
      }
      if (j <= r - 1) {
        double den = knot(ne, r, i + r + 1) - knot(ne, r, i + 1);
        if (den > 0) d -= r / den * nprev[j];
      }
      der[j] = d;
    }
  }
  *first = e;
}

std::vector<double> mass_band(int ne, int r) {
  const int nb = ne + r;
  std::vector<double> band(size_t(nb) * (r + 1), 0.0);
  std::vector<double> gx, gw;
  gauss_rule01(r + 1, gx, gw);
  const double he = 1.0 / ne;
  double v[8], d[8];
  for (int e = 0; e < ne; ++e) {
    for (int g = 0; g <= r; ++g) {
      const double x = (e + gx[g]) * he;
      int f;
      local_basis(ne, r, x, v, d, &f);
      for (int a = 0; a <= r; ++a)
        for (int b = a; b <= r; ++b)
          band[size_t(f + a) * (r + 1) + (b - a)] += gw[g] * he * v[a] * v[b];
    }
  }
  return band;
}

void projection_table(int ne, int r, std::vector<int>& first, std::vector<double>& qv) {
  const int nb = ne + r;
  first.assign(nb, 0);
  qv.assign(size_t(nb) * (r + 2), 0.0);
  // B_k is supported on elements k-r..k; its hat partners are nodes k-r..k+1
  // (indices outside 0..Ne carry zero weight and are skipped by the consumer)
  for (int k = 0; k < nb; ++k) first[k] = k - r;
  std::vector<double> gx, gw;
  gauss_rule01(r + 1, gx, gw);
  const double he = 1.0 / ne;
  double v[8], d[8];
  for (int e = 0; e < ne; ++e) {
    for (int g = 0; g <= r; ++g) {
      const double xi = gx[g];
      const double x = (e + xi) * he;
      int f;
      local_basis(ne, r, x, v, d, &f);
      const double hat[2] = {1.0 - xi, xi};  // nodes e, e+1
      for (int a = 0; a <= r; ++a) {
        const int k = f + a;
        for (int c = 0; c < 2; ++c) {
          const int node = e + c;
          const int t = node - first[k];
          qv[size_t(k) * (r + 2) + t] += gw[g] * he * v[a] * hat[c];
        }
      }
    }
  }
}

void knot_table(int ne, int r, std::vector<int>& first, std::vector<double>& kv) {
  const int n = ne + 1;
  first.assign(n, 0);
  kv.assign(size_t(n) * (r + 1), 0.0);
  double v[8], d[8];
  for (int i = 0; i < n; ++i) {
    int f;
    local_basis(ne, r, double(i) / double(ne), v, d, &f);
    first[i] = f;
    for (int t = 0; t <= r; ++t) kv[size_t(i) * (r + 1) + t] = v[t];
  }
}

void gauss_tables(int ne, int r, std::vector<double>& gb, std::vector<double>& gdb,
                  std::vector<double>& xi, std::vector<double>& w) {
  const int ng = r + 1;
  gauss_rule01(ng, xi, w);
  const double he = 1.0 / ne;
  for (auto& x : w) x *= he;
  gb.assign(size_t(ne) * ng * (r + 1), 0.0);
  gdb.assign(size_t(ne) * ng * (r + 1), 0.0);
  double v[8], d[8];
  for (int e = 0; e < ne; ++e)
    for (int g = 0; g < ng; ++g) {
      int f;
      local_basis(ne, r, (e + xi[g]) * he, v, d, &f);
      for (int a = 0; a <= r; ++a) {
        gb[(size_t(e) * ng + g) * (r + 1) + a] = v[a];
        gdb[(size_t(e) * ng + g) * (r + 1) + a] = d[a];
      }
    }
}

void dst_table(int m, int mp, std::vector<double>& s, std::vector<double>& lam) {
  const double pi = 3.14159265358979323846;
  s.assign(size_t(mp) * mp, 0.0);
  lam.assign(mp, 0.0);
  const double c = std::sqrt(2.0 / (m + 1));
  for (int k = 0; k < m; ++k) {
    for (int j = 0; j < m; ++j)
      s[size_t(k) * mp + j] = c * std::sin(double(k + 1) * double(j + 1) * pi / double(m + 1));
    const double sn = std::sin(double(k + 1) * pi / (2.0 * (m + 1)));
    lam[k] = 4.0 * sn * sn;
  }
}

// d-th derivative of the cardinal B-spline of degree p at x (truncated-power
// form: sum_k (-1)^k C(p+1, k) (x-k)_+^(p-d) / (p-d)!)
static double cardinal_bspline(int p, double x, int d) {
  double s = 0.0, binom = 1.0;
  for (int k = 0; k <= p + 1; ++k) {
    if (x > k) s += ((k & 1) ? -binom : binom) * std::pow(x - k, p - d);
    binom = binom * (p + 1 - k) / (k + 1);
  }
  double fact = 1.0;
  for (int i = 2; i <= p - d; ++i) fact *= i;
  return s / fact;
}

void bspline_symbols(int r, int m, int mp, std::vector<double>& sym) {
  const double pi = 3.14159265358979323846;
  std::vector<double> mt(r + 1), kt(r + 1);
  for (int t = 0; t <= r; ++t) {
    mt[t] = cardinal_bspline(2 * r + 1, r + 1 + t, 0);
    kt[t] = -cardinal_bspline(2 * r + 1, r + 1 + t, 2);
  }
  sym.assign(size_t(2) * mp, 1.0);
  for (int k = 0; k < m; ++k) {
    const double th = double(k + 1) * pi / double(m + 1);
    double ms = mt[0], ks = kt[0];
    for (int t = 1; t <= r; ++t) {
      ms += 2.0 * mt[t] * std::cos(t * th);
      ks += 2.0 * kt[t] * std::cos(t * th);
    }
    sym[k] = ms;
    sym[mp + k] = ks;
  }
}

bool well_sources(const double* wells, int n_wells, int ne, int dim, double radius,
                  std::vector<double>& q_inj, std::vector<double>& q_prod, std::string& err) {
  const int n = ne + 1;
  size_t total = 1;
  for (int d = 0; d < dim; ++d) total *= n;
  q_inj.assign(total, 0.0);
  q_prod.assign(total, 0.0);
  const double h = 1.0 / ne;
  double hd = 1.0;
  for (int d = 0; d < dim; ++d) hd *= h;
  const double r2 = radius * radius;
  std::vector<unsigned char> disc(size_t(n) * n);
  for (int w = 0; w < n_wells; ++w) {
    const double xw = wells[3 * w], yw = wells[3 * w + 1], rate = wells[3 * w + 2];
    long cnt = 0;
    bool touches = false;
    for (int j = 0; j < n; ++j) {
      const double dy = double(j) / double(ne) - yw;
      const double dy2 = dy * dy;
      for (int i = 0; i < n; ++i) {
        const double dx = double(i) / double(ne) - xw;
        const double dx2 = dx * dx;
        const double s = dy2 + dx2;
        const bool in = s <= r2;
        disc[size_t(j) * n + i] = in;
        if (in) {
          if (i == 0 || j == 0 || i == ne || j == ne) touches = true;
          cnt += (dim == 2) ? 1 : (n - 2);
        }
      }
    }
    if (cnt == 0) {
      err = "well " + std::to_string(w) + " covers no node";
      return false;
    }
    if (touches) {
      err = "well " + std::to_string(w) + " reaches the boundary";
      return false;
    }
    const double val = rate / (hd * double(cnt));
    std::vector<double>& q = rate >= 0 ? q_inj : q_prod;
    const int kz0 = dim == 2 ? 0 : 1, kz1 = dim == 2 ? 1 : n - 1;
    for (int k = kz0; k < kz1; ++k)
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i)
          if (disc[size_t(j) * n + i]) q[(size_t(k) * n + j) * n + i] += val;
  }
  return true;
}

std::vector<double> pack_gemm_a(const std::vector<double>& a, int M, int K) {
  std::vector<double> out(size_t(M) * K);
  for (int mb = 0; mb < M / 32; ++mb)
    for (int kc = 0; kc < K / 16; ++kc)
      for (int lane = 0; lane < 64; ++lane)
        for (int u = 0; u < 8; ++u) {
          const int row = 32 * mb + (lane & 31), col = 16 * kc + 2 * u + (lane >> 5);
          out[((size_t(mb) * (K / 16) + kc) * 64 + lane) * 8 + u] = a[size_t(row) * K + col];
        }
  return out;
}

}  // namespace crv
