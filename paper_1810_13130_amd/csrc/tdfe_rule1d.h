// The one-dimensional reference rule of the spectral elements (Sec. spectral
// FE): Gauss-Lobatto-Legendre nodes and weights (the nodal points and the
// quadrature of the overlap), the Gauss-Legendre rule with nq = p + 1 points
// (the quadrature of the Hamiltonian), and the interpolation and derivative
// tables between them, all as constexpr functions.  The host set-up evaluates
// them at run time; the operator kernels evaluate them at compile time for
// their order, so every coefficient of a 1D contraction is a constant of the
// instruction stream (literal or scalar move) rather than a memory operand.
// Both evaluations run the same IEEE double arithmetic and give the same bits.
#pragma once

namespace tdfe1d {

constexpr int MAXN = 9;  // p <= 8
constexpr double kPi = 3.14159265358979323846;

constexpr double cabs(double x) { return x < 0.0 ? -x : x; }

// cos on [0, pi] by its Taylor series after reflection to [0, pi/2]; used for
// the starting points of the Newton iterations only
constexpr double ccos(double x) {
  bool neg = false;
  if (x > 0.5 * kPi) {
    x = kPi - x;
    neg = true;
  }
  const double x2 = x * x;
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 24; ++k) {
    term *= -x2 / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return neg ? -sum : sum;
}

constexpr double cpow(double x, int n) {
  double r = 1.0;
  for (int k = 0; k < n; ++k) r *= x;
  return r;
}

// P_m(x) and P_m'(x) by the three-term recurrence
constexpr void legendre(int m, double x, double& P, double& dP) {
  if (m == 0) {
    P = 1.0;
    dP = 0.0;
    return;
  }
  double p0 = 1.0, p1 = x;
  for (int k = 2; k <= m; ++k) {
    const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  P = p1;
  dP = (cabs(x) < 1.0) ? m * (x * p1 - p0) / (x * x - 1.0) : 0.5 * m * (m + 1) * cpow(x, m + 1);
}

struct Rule {
  int p = 0, n = 0, nq = 0;
  double xi[MAXN] = {}, w[MAXN] = {};    // GLL nodes and weights
  double eta[MAXN] = {}, wq[MAXN] = {};  // Gauss points and weights
  double B[MAXN * MAXN] = {};            // B[a*MAXN+i] = l_i(eta_a)   (GLL Lagrange basis)
  double D[MAXN * MAXN] = {};            // D[a*MAXN+i] = l_i'(eta_a)
  double Dg[MAXN * MAXN] = {};           // Dg[a*MAXN+b] = g_b'(eta_a) (Gauss-point Lagrange basis)
};

// barycentric Lagrange basis on nodes[0..n) evaluated (value, derivative) at x
constexpr void lagrange_eval(int n, const double* nodes, double x, double* val, double* der) {
  double lam[MAXN] = {};
  for (int i = 0; i < n; ++i) {
    lam[i] = 1.0;
    for (int m = 0; m < n; ++m)
      if (m != i) lam[i] /= (nodes[i] - nodes[m]);
  }
  int hit = -1;
  for (int i = 0; i < n; ++i)
    if (cabs(x - nodes[i]) < 1e-14) hit = i;
  if (hit >= 0) {
    for (int i = 0; i < n; ++i) {
      val[i] = (i == hit) ? 1.0 : 0.0;
      if (i != hit) {
        der[i] = (lam[i] / lam[hit]) / (nodes[hit] - nodes[i]);
      } else {
        double s = 0.0;
        for (int m = 0; m < n; ++m)
          if (m != hit) s += 1.0 / (nodes[hit] - nodes[m]);
        der[i] = s;
      }
    }
    return;
  }
  double den = 0.0;
  for (int i = 0; i < n; ++i) den += lam[i] / (x - nodes[i]);
  for (int i = 0; i < n; ++i) {
    val[i] = (lam[i] / (x - nodes[i])) / den;
    double s = 0.0;
    for (int m = 0; m < n; ++m)
      if (m != i) s += 1.0 / (x - nodes[m]);
    der[i] = val[i] * s;
  }
}

constexpr Rule make_rule(int p) {
  Rule R{};
  R.p = p;
  R.n = p + 1;
  R.nq = p + 1;
  // GLL: the end points and the roots of P_p' (Newton with P_p'' from
  // Legendre's equation), weights 2 / (p (p + 1) P_p(x)^2)
  R.xi[0] = -1.0;
  R.xi[p] = 1.0;
  for (int i = 1; i < p; ++i) {
    double r = -ccos(kPi * i / p);
    for (int it = 0; it < 100; ++it) {
      double P = 0.0, dP = 0.0;
      legendre(p, r, P, dP);
      const double d2P = (2.0 * r * dP - p * (p + 1.0) * P) / (1.0 - r * r);
      const double dr = dP / d2P;
      r -= dr;
      if (cabs(dr) < 1e-16) break;
    }
    R.xi[i] = r;
  }
  for (int i = 0; i <= p; ++i) {
    double P = 0.0, dP = 0.0;
    legendre(p, R.xi[i], P, dP);
    R.w[i] = 2.0 / (p * (p + 1.0) * P * P);
  }
  // Gauss: roots of P_nq, weights 2 / ((1 - x^2) P_nq'(x)^2)
  const int nq = R.nq;
  for (int i = 0; i < nq; ++i) {
    double r = -ccos(kPi * (i + 0.75) / (nq + 0.5));
    for (int it = 0; it < 100; ++it) {
      double P = 0.0, dP = 0.0;
      legendre(nq, r, P, dP);
      const double dr = P / dP;
      r -= dr;
      if (cabs(dr) < 1e-16) break;
    }
    double P = 0.0, dP = 0.0;
    legendre(nq, r, P, dP);
    R.eta[i] = r;
    R.wq[i] = 2.0 / ((1.0 - r * r) * dP * dP);
  }
  for (int a = 0; a < nq; ++a) {
    double v[MAXN] = {}, dv[MAXN] = {};
    lagrange_eval(R.n, R.xi, R.eta[a], v, dv);
    for (int i = 0; i < R.n; ++i) {
      R.B[a * MAXN + i] = v[i];
      R.D[a * MAXN + i] = dv[i];
    }
    lagrange_eval(nq, R.eta, R.eta[a], v, dv);
    for (int b = 0; b < nq; ++b) R.Dg[a * MAXN + b] = dv[b];
  }
  return R;
}

}  // namespace tdfe1d
