// rt_arrow.h -- SVD of the incremental-SVD core (App. B, eq. svd_core) by its
// secular equation.
//
// The core is K = [[diag(s), a], [0, nu]] ((r+1) x (r+1), s descending and
// positive) or, for a rank-deficient snapshot, K = [diag(s), a] (r x (r+1)).
// K K^T = D + z z^T with D = diag(s_j^2) (plus a zero pole for the nu row)
// and z = (a, nu), so the squared singular values are the roots of the
// secular function f(lambda) = 1 + sum_j z_j^2 / (d_j - lambda), one in each
// interval between consecutive poles and one above the largest.  Each root is
// found in coordinates shifted to its nearer pole, with pole differences
// formed as (s_a - s_b)(s_a + s_b) so that they keep full relative accuracy;
// the vector z is then recomputed from the roots (Gu and Eisenstat), which
// makes the singular vectors numerically orthogonal:
//   left  u_k ~ (z_j / (d_j - lambda_k))_j,
//   right v_k ~ (s_j z_j / (d_j - lambda_k))_{j < r}, -1 in the last column
// (v = K^T u / sigma, using z^T (D - lambda)^{-1} z = -1 at a root).
// Rows whose coupling z_j is below rounding deflate to (s_j, e_j, e_j).
// Equal poles make the secular equation degenerate: the routine then declines
// and the caller uses one-sided Jacobi instead.
//
// Everything is written per root / per component so that the same functions
// run on one wave (lane = root) and on the host (loops) for testing.
#pragma once
#include <math.h>

#ifndef RT_HD
#define RT_HD __host__ __device__
#endif

namespace arrow {

constexpr int N = 24;  // capacity (rows of the core)

struct Problem {
  int m;           // number of non-deflated poles
  int rows, cols;  // core shape
  double scale;    // max(s_0, |z|)
  // non-deflated poles in ascending order
  double s[N];     // sqrt of the pole (0 for the nu row)
  double z[N];     // coupling
  int row[N];      // core row of the pole
};

// d_a - d_b for poles with square roots sa, sb, to full relative accuracy
RT_HD inline double pole_diff(double sa, double sb) { return (sa - sb) * (sa + sb); }

// 1/x: a true division on the host; on the device the hardware reciprocal
// refined by two Newton steps (within about an ulp).
RT_HD inline double rcp(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
#else
  return 1.0 / x;
#endif
}

// Identity combine: one lane evaluates all terms.
struct Whole {
  RT_HD double operator()(double v) const { return v; }
};

// f, psi (poles <= k), phi (poles > k) and derivatives at tau, for poles
// shifted by the origin pole: dd[t] = d_j - d_K for the terms j = g + G t
// this lane owns (G lanes share one root and comb adds their partial sums,
// giving every lane of the group the same totals).  dd and z are held by the
// caller (registers on the device: every loop runs over the capacity).
struct Eval {
  double f, psi, dpsi, phi, dphi, erretm;
};
template <int G, class Comb>
RT_HD inline Eval evaluate(const double (&dd)[N / G], const double (&z)[N / G], int m, int k, int g, double tau,
                           Comb comb) {
  Eval e{1.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int t = 0; t < N / G; ++t) {
    const int j = g + G * t;
    if (j < m) {
      const double q = z[t] * rcp(dd[t] - tau);
      const double term = z[t] * q;
      if (j <= k) {
        e.psi += term;
        e.dpsi += q * q;
      } else {
        e.phi += term;
        e.dphi += q * q;
      }
      e.erretm += fabs(term);
    }
  }
  e.psi = comb(e.psi);
  e.dpsi = comb(e.dpsi);
  e.phi = comb(e.phi);
  e.dphi = comb(e.dphi);
  e.erretm = comb(e.erretm);
  e.f = 1.0 + e.psi + e.phi;
  return e;
}

template <int G>
RT_HD inline void shifted_poles(const Problem &P, int K, int g, double (&dd)[N / G]) {
#pragma unroll
  for (int t = 0; t < N / G; ++t) {
    const int j = g + G * t;
    dd[t] = (j < P.m) ? pole_diff(P.s[j], P.s[K]) : 0.0;
  }
}

// Root k of the secular equation (k < m): returns the origin pole K and the
// shift tau, lambda_k = s_K^2 + tau.  Safeguarded two-pole rational Newton
// iteration inside a bracket that shrinks with every evaluation.  G lanes
// (g = 0..G-1) may work on one root, each summing every G-th term; all of
// them take the same steps and return the same root.
template <int G, class Comb>
RT_HD inline void root_g(const Problem &P, int k, int g, Comb comb, int &K_out, double &tau_out) {
  static_assert(N % G == 0, "terms split evenly over the group");
  const int m = P.m;
  if (m == 1) {  // one pole: lambda = d_0 + z_0^2
    K_out = 0;
    tau_out = P.z[0] * P.z[0];
    return;
  }
  double z[N / G], dd[N / G];
  double z2 = 0.0;
#pragma unroll
  for (int t = 0; t < N / G; ++t) {
    const int j = g + G * t;
    z[t] = (j < m) ? P.z[j] : 0.0;
    z2 += z[t] * z[t];
  }
  z2 = comb(z2);
  int K;
  double lo, hi;  // bracket in tau around the root, f(lo) < 0 < f(hi)
  if (k < m - 1) {
    const double gap = pole_diff(P.s[k + 1], P.s[k]);
    // f at the midpoint, shifted by the lower pole
    shifted_poles<G>(P, k, g, dd);
    const Eval mid = evaluate<G>(dd, z, m, k, g, 0.5 * gap, comb);
    if (mid.f >= 0.0) {
      K = k;
      lo = 0.0;
      hi = 0.5 * gap;
    } else {
      K = k + 1;
      lo = -0.5 * gap;
      hi = 0.0;
      shifted_poles<G>(P, K, g, dd);
    }
  } else {
    K = m - 1;
    lo = 0.0;
    hi = z2;
    shifted_poles<G>(P, K, g, dd);
  }
  // the two poles around the root, shifted by K
  const double da = pole_diff(P.s[k], P.s[K]);
  const double db = (k < m - 1) ? pole_diff(P.s[k + 1], P.s[K]) : 0.0;
  // the pole ends of the bracket are never evaluated: start inside
  double tau = 0.5 * (lo + hi);
  const double eps = 2.220446049250313e-16;
  for (int it = 0; it < 200; ++it) {
    const Eval e = evaluate<G>(dd, z, m, k, g, tau, comb);
    if (e.f == 0.0) break;
    if (e.f < 0.0) lo = tau;
    else hi = tau;
    // converged when |f| is at the level of its own rounding error (about two
    // ulps per term) or the bracket can no longer shrink
    if (fabs(e.f) <= 2.0 * eps * (1.0 + e.erretm)) break;
    if (hi - lo <= 4.0 * eps * fmax(fabs(lo), fabs(hi))) break;
    // two-pole model: c + S1 / (da - x) + S2 / (db - x), fitted to value and
    // derivatives of psi (poles <= k) and phi (poles > k) at tau
    double x;
    if (k < m - 1) {
      const double ra = da - tau, rb = db - tau;
      const double S1 = e.dpsi * ra * ra, S2 = e.dphi * rb * rb;
      const double c = e.f - S1 / ra - S2 / rb;
      // c (da - x)(db - x) + S1 (db - x) + S2 (da - x) = 0, in y = x - tau:
      // c (ra - y)(rb - y) + S1 (rb - y) + S2 (ra - y) = 0
      const double A = c;
      const double B = -(c * (ra + rb) + S1 + S2);
      const double C = c * ra * rb + S1 * rb + S2 * ra;
      double y;
      if (A == 0.0) {
        y = -C / B;
      } else {
        const double disc = fmax(B * B - 4.0 * A * C, 0.0);
        const double q = -0.5 * (B + (B >= 0.0 ? sqrt(disc) : -sqrt(disc)));
        const double y1 = q / A, y2 = (q != 0.0) ? C / q : y1;
        // the root of the model between the poles
        const bool in1 = (tau + y1 > lo) && (tau + y1 < hi);
        const bool in2 = (tau + y2 > lo) && (tau + y2 < hi);
        y = in1 ? y1 : (in2 ? y2 : 0.5 * (lo + hi) - tau);
      }
      x = tau + y;
    } else {
      // last root: c + S1 / (da - x) = 0
      const double ra = da - tau;
      const double S1 = e.dpsi * ra * ra;
      const double c = e.f - S1 / ra;
      x = (c > 0.0) ? da + S1 / c : 0.5 * (lo + hi);
    }
    if (!(x > lo && x < hi)) x = 0.5 * (lo + hi);
    if (x == tau) break;
    tau = x;
  }
  K_out = K;
  tau_out = tau;
}

// Root k by one lane.
RT_HD inline void root(const Problem &P, int k, int &K_out, double &tau_out) {
  root_g<1>(P, k, 0, Whole(), K_out, tau_out);
}

// lambda_k - d_j = (d_K - d_j) + tau_k
RT_HD inline double lam_minus_pole(const Problem &P, int K, double tau, int j) {
  return pole_diff(P.s[K], P.s[j]) + tau;
}

// Recomputed coupling for pole j from all the roots (Gu-Eisenstat), sign of z_j.
RT_HD inline double zhat(const Problem &P, int j, const int *K, const double *tau) {
  double prod = lam_minus_pole(P, K[P.m - 1], tau[P.m - 1], j);
#pragma unroll
  for (int i = 0; i < N - 1; ++i) {
    if (i < P.m - 1) {
      // pair the root below/above pole j with the pole difference of the same side
      const int dpole = i < j ? i : i + 1;
      prod *= lam_minus_pole(P, K[i], tau[i], j) * rcp(pole_diff(P.s[dpole], P.s[j]));
    }
  }
  const double mag = sqrt(fabs(prod));
  return P.z[j] >= 0.0 ? mag : -mag;
}

// Builds the secular problem of the core from S (r values, descending), a (r)
// and nu (used when rows == r + 1).  defl[j] = 1 marks a deflated row j < r.
// Returns false when the secular equation would be degenerate.
RT_HD inline bool build(Problem &P, int *defl, const double *S, const double *a, double nu, int r, int rows,
                        int cols) {
  const double eps = 2.220446049250313e-16;
  double z2 = rows > r ? nu * nu : 0.0;
  for (int j = 0; j < r; ++j) z2 += a[j] * a[j];
  const double scale = fmax(r > 0 ? S[0] : 0.0, sqrt(z2));
  const double tolz = 8.0 * eps * scale;
  bool ok = (rows == r || nu > tolz);
  int m = 0;
  if (rows > r) {  // the nu row: pole 0
    P.s[m] = 0.0;
    P.z[m] = nu;
    P.row[m] = r;
    ++m;
  }
  for (int j = r - 1; j >= 0; --j) {  // ascending poles
    defl[j] = fabs(a[j]) <= tolz;
    if (!defl[j]) {
      if (m > 0 && S[j] - P.s[m - 1] <= 8.0 * eps * S[j]) ok = false;  // coinciding poles
      P.s[m] = S[j];
      P.z[m] = a[j];
      P.row[m] = j;
      ++m;
    }
  }
  P.m = m;
  P.rows = rows;
  P.cols = cols;
  P.scale = scale;
  return ok;
}

// Singular triplet of root k: u (rows entries, stride us), v (cols entries,
// stride vs), returns sigma.  r = number of S values.
RT_HD inline double vectors(const Problem &P, int k, const int *K, const double *tau, const double *zh, int r,
                            double *u, int us, double *v, int vs) {
  const int Kk = K[k];
  const double tk = tau[k];
  // components in registers first (loops over the capacity), then every
  // store at once: zeros for the deflated rows, the normalised entries
  double ur[N], vr[N];
  double un = 0.0, vn = 1.0;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    ur[i] = vr[i] = 0.0;
    if (i < P.m) {
      const double ui = zh[i] * rcp(pole_diff(P.s[i], P.s[Kk]) - tk);
      ur[i] = ui;
      un += ui * ui;
      if (P.row[i] < r) {
        const double vi = P.s[i] * ui;
        vr[i] = vi;
        vn += vi * vi;
      }
    }
  }
  const double iu = rcp(sqrt(un)), iv = rcp(sqrt(vn));
#pragma unroll
  for (int i = 0; i < N; ++i) {
    if (i < P.rows) u[i * us] = 0.0;
    if (i < P.cols) v[i * vs] = 0.0;
  }
#pragma unroll
  for (int i = 0; i < N; ++i)
    if (i < P.m) {
      const int row = P.row[i];
      u[row * us] = ur[i] * iu;
      if (row < r) v[row * vs] = vr[i] * iv;
    }
  v[r * vs] = -iv;  // z^T (D - lambda)^{-1} z = -1 at a root, normalised
  return sqrt(P.s[Kk] * P.s[Kk] + tk);
}

}  // namespace arrow
