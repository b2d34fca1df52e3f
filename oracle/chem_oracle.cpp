// CPU ORACLE for batched stiff-chemistry integration.  TEST INFRASTRUCTURE ONLY:
// only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may load
// or call this file.  It shares no code with the HIP path.
//
// Plain, slow, FP64.  What it computes, with the passage it follows:
//  * the chemistry IVP dPhi/dt = f(Phi), Phi = (T, Y_1..Y_K) at fixed p
//    (paper section 2.1, Eq. 1; all K mass fractions are carried);
//  * f from Chemkin-form kinetics: NASA-7 thermo, Arrhenius forward rates,
//    reverse rates from equilibrium constants, third-body and Troe falloff
//    (the species production rates that section 2.3 delegates to pyJac);
//  * the dense Jacobian J = df/dPhi (section 2.3): by its definition through
//    forward-mode dual numbers (jac_ad), and by the hand-derived analytic
//    formulas (jac_analytic) the integrator uses, as pyJac does;
//  * dense LU with partial pivoting and forward/back substitution (section
//    2.3, LAPACK getrf/getrs semantics);
//  * the linearised implicit step of Eq. 2 as the 1-stage special case of a
//    Rosenbrock method, and the 4-stage Rosenbrock methods ROS4 and Rodas3
//    (Hairer & Wanner, Solving ODEs II, section IV.7) with adaptive step
//    control over one CFD time step (section 2.3: rtol/atol, a sub-step that
//    persists between calls);
//  * the tangent-linear model of the integration with its accepted step
//    sequence frozen (forward-mode duals through every step);
//  * the Seulex-family integrator of section 2.3 (extrapolated linearly
//    implicit Euler with order control);
//  * the ablation options of section 2.3 (one-sided finite-difference
//    Jacobian, LU without pivoting);
//  * reference-cell mapping of low-reactivity cells (section 2.2).
//
// Units: CGS inside (p in dyn/cm^2, R in erg/mol/K, C in mol/cm^3); the C API
// takes p in Pa.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <algorithm>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

constexpr double RU = 8.314462618e7;   // erg / (mol K)
constexpr double PATM = 1.01325e6;      // standard-state pressure, dyn/cm^2
constexpr double LN10 = 2.302585092994045684;

// ---------------------------------------------------------------- dual numbers
template <class T> struct Dual {
  T v, d;
  Dual() : v(0.0), d(0.0) {}
  Dual(double x) : v(x), d(0.0) {}
  Dual(const T& a, const T& b) : v(a), d(b) {}
};
inline double val(double x) { return x; }
template <class T> double val(const Dual<T>& x) { return val(x.v); }

template <class T> Dual<T> operator+(const Dual<T>& a, const Dual<T>& b) { return {a.v + b.v, a.d + b.d}; }
template <class T> Dual<T> operator-(const Dual<T>& a, const Dual<T>& b) { return {a.v - b.v, a.d - b.d}; }
template <class T> Dual<T> operator*(const Dual<T>& a, const Dual<T>& b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
template <class T> Dual<T> operator/(const Dual<T>& a, const Dual<T>& b) {
  T q = a.v / b.v;
  return {q, (a.d - q * b.d) / b.v};
}
template <class T> Dual<T> operator-(const Dual<T>& a) { return {-a.v, -a.d}; }
template <class T> Dual<T> operator+(const Dual<T>& a, double b) { return a + Dual<T>(b); }
template <class T> Dual<T> operator+(double a, const Dual<T>& b) { return Dual<T>(a) + b; }
template <class T> Dual<T> operator-(const Dual<T>& a, double b) { return a - Dual<T>(b); }
template <class T> Dual<T> operator-(double a, const Dual<T>& b) { return Dual<T>(a) - b; }
template <class T> Dual<T> operator*(const Dual<T>& a, double b) { return {a.v * b, a.d * b}; }
template <class T> Dual<T> operator*(double a, const Dual<T>& b) { return {a * b.v, a * b.d}; }
template <class T> Dual<T> operator/(const Dual<T>& a, double b) { return {a.v / b, a.d / b}; }
template <class T> Dual<T> operator/(double a, const Dual<T>& b) { return Dual<T>(a) / b; }
template <class T, class U> Dual<T>& operator+=(Dual<T>& a, const U& b) { a = a + b; return a; }
template <class T, class U> Dual<T>& operator-=(Dual<T>& a, const U& b) { a = a - b; return a; }
template <class T, class U> Dual<T>& operator*=(Dual<T>& a, const U& b) { a = a * b; return a; }
template <class T, class U> Dual<T>& operator/=(Dual<T>& a, const U& b) { a = a / b; return a; }

using std::exp;
using std::log;
template <class T> Dual<T> exp(const Dual<T>& a) { T e = exp(a.v); return {e, e * a.d}; }
template <class T> Dual<T> log(const Dual<T>& a) { return {log(a.v), a.d / a.v}; }
template <class T> Dual<T> sqrt(const Dual<T>& a) { using std::sqrt; T s = sqrt(a.v); return {s, a.d / (2.0 * s)}; }
// ------------------------------------------------- operation-counting scalar
// Counts the floating-point operations that f and J perform, for the
// algorithmic FLOP figures of the roofline: additions/subtractions,
// multiplications, divisions, exponentials and logarithms separately.  A
// value known to be exactly zero (a zero constant or input, or a product
// with one) makes an operation free: adding it or multiplying by it is no
// work, so structurally zero terms of the plain dense loops are not counted.
// One evaluation at a time (global tallies).
struct OpTally {
  double add = 0, mul = 0, div = 0, exp = 0, log = 0;
};
OpTally g_ops;
struct Cnt {
  double v;
  bool zero;
  Cnt() : v(0.0), zero(true) {}
  Cnt(double x) : v(x), zero(x == 0.0) {}
};
inline double val(const Cnt& x) { return x.v; }
inline Cnt cnt_zero() { return Cnt(); }
inline Cnt operator+(const Cnt& a, const Cnt& b) {
  if (a.zero) return b;
  if (b.zero) return a;
  g_ops.add += 1;
  Cnt r(a.v + b.v);
  r.zero = false;
  return r;
}
inline Cnt operator-(const Cnt& a) {
  Cnt r(-a.v);
  r.zero = a.zero;
  return r;
}
inline Cnt operator-(const Cnt& a, const Cnt& b) {
  if (b.zero) return a;
  if (a.zero) return -b;
  g_ops.add += 1;
  Cnt r(a.v - b.v);
  r.zero = false;
  return r;
}
inline Cnt operator*(const Cnt& a, const Cnt& b) {
  if (a.zero || b.zero) return cnt_zero();
  g_ops.mul += 1;
  Cnt r(a.v * b.v);
  r.zero = false;
  return r;
}
inline Cnt operator/(const Cnt& a, const Cnt& b) {
  if (a.zero) return cnt_zero();
  g_ops.div += 1;
  Cnt r(a.v / b.v);
  r.zero = false;
  return r;
}
inline Cnt operator+(const Cnt& a, double b) { return a + Cnt(b); }
inline Cnt operator+(double a, const Cnt& b) { return Cnt(a) + b; }
inline Cnt operator-(const Cnt& a, double b) { return a - Cnt(b); }
inline Cnt operator-(double a, const Cnt& b) { return Cnt(a) - b; }
inline Cnt operator*(const Cnt& a, double b) { return a * Cnt(b); }
inline Cnt operator*(double a, const Cnt& b) { return Cnt(a) * b; }
inline Cnt operator/(const Cnt& a, double b) { return a / Cnt(b); }
inline Cnt operator/(double a, const Cnt& b) { return Cnt(a) / b; }
inline Cnt& operator+=(Cnt& a, const Cnt& b) { a = a + b; return a; }
inline Cnt& operator-=(Cnt& a, const Cnt& b) { a = a - b; return a; }
inline Cnt& operator*=(Cnt& a, const Cnt& b) { a = a * b; return a; }
inline Cnt& operator/=(Cnt& a, const Cnt& b) { a = a / b; return a; }
inline Cnt exp(const Cnt& a) {
  g_ops.exp += 1;
  Cnt r(std::exp(a.v));
  r.zero = false;
  return r;
}
inline Cnt log(const Cnt& a) {
  g_ops.log += 1;
  return Cnt(std::log(a.v));
}

template <class S> S log10_(const S& a) { return log(a) / LN10; }
template <class S> S pow10_(const S& a) { return exp(a * LN10); }
template <class S> S ipow(const S& x, int n) {
  S r(1.0);
  for (int i = 0; i < n; ++i) r = r * x;
  for (int i = 0; i > n; --i) r = r / x;
  return r;
}
template <class S> S sabs(const S& x) { return val(x) < 0.0 ? -x : x; }

// ------------------------------------------------------------------ mechanism
}  // namespace

extern "C" {
struct OracleMech {
  int32_t K, R;
  const double* W;      // [K]
  const double* nasa7;  // [K][15]: Tmid, lo a1..a7, hi a1..a7
  const int32_t* rtype; // [R]: 0 elementary, 1 third-body, 2 Troe
  const int32_t* reac;  // [R][3], -1 = empty slot
  const int32_t* prod;  // [R][3]
  const double* lnA;    // [R]
  const double* b;      // [R]
  const double* theta;  // [R]
  const double* eff;    // [R][K]
  const double* troe;   // [R][4]: alpha, T***, T*, T**
  const double* low;    // [R][3]: lnA0, b0, theta0
};
struct OracleOpts {
  int32_t method;     // 0 ROS4, 1 Rodas3, 2 linearly implicit Euler (Eq. 2)
  int32_t max_steps;  // attempts per cell before TOO_MANY_STEPS
  double fac_safe, fac_min, fac_max, h_min;
  int32_t jac_mode;   // 0 analytic Jacobian, 1 one-sided finite differences (section 2.3's "Standard" case)
  int32_t lu_pivot;   // 0 partial pivoting (LAPACK), 1 no pivoting (a naive LU)
};
}

namespace {

enum { ST_OK = 0, ST_TOO_MANY_STEPS = 1, ST_UNDERFLOW = 2, ST_SINGULAR = 3, ST_NONFINITE = 4 };

// Arrhenius parameters as scalars of type S (duals for the tangent-linear model)
template <class S> struct Params {
  const S* lnA;
  const S* b;
  const S* theta;
};

// NASA-7 polynomials (Chemkin thermodynamic data format):
//   cp/R = a1 + a2 T + a3 T^2 + a4 T^3 + a5 T^4
//   h/RT = a1 + a2 T/2 + a3 T^2/3 + a4 T^3/4 + a5 T^4/5 + a6/T
//   s/R  = a1 ln T + a2 T + a3 T^2/2 + a4 T^3/3 + a5 T^4/4 + a7
template <class S>
void thermo(const OracleMech& m, int k, const S& T, const S& lnT, S& cpR, S& hRT, S& sR, S& dcpRdT) {
  const double* row = m.nasa7 + 15 * k;
  const double* a = (val(T) > row[0]) ? row + 8 : row + 1;
  S T2 = T * T, T3 = T2 * T, T4 = T3 * T;
  cpR = a[0] + a[1] * T + a[2] * T2 + a[3] * T3 + a[4] * T4;
  hRT = a[0] + a[1] * T / 2.0 + a[2] * T2 / 3.0 + a[3] * T3 / 4.0 + a[4] * T4 / 5.0 + a[5] / T;
  sR = a[0] * lnT + a[1] * T + a[2] * T2 / 2.0 + a[3] * T3 / 3.0 + a[4] * T4 / 4.0 + a[6];
  dcpRdT = a[1] + 2.0 * a[2] * T + 3.0 * a[3] * T2 + 4.0 * a[4] * T3;
}

// Everything the rate of one reaction depends on, evaluated at (T, C).
template <class S> struct Mix {
  int K;
  S T, lnT, rho, Wbar, cp, dcpdT;
  std::vector<S> cpR, hRT, sR, gRT, dcpRdT, C;
};

template <class S> void mixture(const OracleMech& m, double p, const S* y, Mix<S>& x) {
  const int K = m.K;
  x.K = K;
  x.T = y[0];
  x.lnT = log(x.T);
  x.cpR.assign(K, S(0.0)); x.hRT.assign(K, S(0.0)); x.sR.assign(K, S(0.0));
  x.gRT.assign(K, S(0.0)); x.dcpRdT.assign(K, S(0.0)); x.C.assign(K, S(0.0));
  for (int k = 0; k < K; ++k) {
    thermo(m, k, x.T, x.lnT, x.cpR[k], x.hRT[k], x.sR[k], x.dcpRdT[k]);
    x.gRT[k] = x.hRT[k] - x.sR[k];
  }
  // 1/Wbar = sum Y_k/W_k ; rho = p Wbar/(R T) ; C_k = rho Y_k / W_k
  S sy(0.0);
  for (int k = 0; k < K; ++k) sy += y[1 + k] / m.W[k];
  x.Wbar = 1.0 / sy;
  x.rho = p * x.Wbar / (RU * x.T);
  for (int k = 0; k < K; ++k) x.C[k] = x.rho * y[1 + k] / m.W[k];
  // mass-specific c_p = sum Y_k cp_k / W_k and its T-derivative
  x.cp = S(0.0);
  x.dcpdT = S(0.0);
  for (int k = 0; k < K; ++k) {
    x.cp += y[1 + k] * x.cpR[k] * RU / m.W[k];
    x.dcpdT += y[1 + k] * x.dcpRdT[k] * RU / m.W[k];
  }
}

// Rate of progress q_r and the pieces the Jacobian needs.
template <class S> struct Rate {
  S q;          // rate of progress, mol/cm^3/s
  S keff;       // effective forward coefficient (incl. [M] or falloff)
  S Kc;         // equilibrium constant in concentration units
  S Rf, Rr;     // products of reactant / product concentrations
  S dkeff_dT;   // d keff / dT at fixed C
  S dkeff_dM;   // d keff / d[M] at fixed T
  S dlnKc_dT;
};

template <class S>
Rate<S> rate(const OracleMech& m, const Params<S>& P, const Mix<S>& x, int r) {
  Rate<S> out;
  const int* re = m.reac + 3 * r;
  const int* pr = m.prod + 3 * r;
  const S& T = x.T;
  // forward rate coefficient k = A T^b exp(-theta/T)
  S kf = exp(P.lnA[r] + P.b[r] * x.lnT - P.theta[r] / T);
  S dlnkf_dT = P.b[r] / T + P.theta[r] / (T * T);
  // Kc = exp(-sum nu g/RT) (p_atm/(R T))^(sum nu)
  int dnu = 0;
  S sum_nu_g(0.0), sum_nu_h(0.0);
  for (int s = 0; s < 3; ++s) {
    if (re[s] >= 0) { dnu -= 1; sum_nu_g -= x.gRT[re[s]]; sum_nu_h -= x.hRT[re[s]]; }
    if (pr[s] >= 0) { dnu += 1; sum_nu_g += x.gRT[pr[s]]; sum_nu_h += x.hRT[pr[s]]; }
  }
  out.Kc = exp(-sum_nu_g) * ipow(PATM / (RU * T), dnu);
  // d(g_k/RT)/dT = -(h_k/RT)/T  =>  d ln Kc/dT = sum nu (h/RT)/T - sum nu / T
  out.dlnKc_dT = sum_nu_h / T - double(dnu) / T;
  out.Rf = S(1.0);
  out.Rr = S(1.0);
  for (int s = 0; s < 3; ++s) {
    if (re[s] >= 0) out.Rf *= x.C[re[s]];
    if (pr[s] >= 0) out.Rr *= x.C[pr[s]];
  }
  const int type = m.rtype[r];
  if (type == 0) {
    out.keff = kf;
    out.dkeff_dT = kf * dlnkf_dT;
    out.dkeff_dM = S(0.0);
  } else {
    S M(0.0);
    for (int k = 0; k < x.K; ++k) M += m.eff[(size_t)r * x.K + k] * x.C[k];
    if (type == 1) {
      out.keff = kf * M;
      out.dkeff_dT = M * kf * dlnkf_dT;
      out.dkeff_dM = kf;
    } else {
      // Troe falloff (Gilbert, Luther & Troe 1983): k_inf = kf, k0 from the
      // low-pressure line, Pr = k0 [M] / k_inf, k = k_inf Pr/(1+Pr) F.
      const double* lo = m.low + 3 * r;
      const double* tr = m.troe + 4 * r;
      const double alpha = tr[0], T3 = tr[1], T1 = tr[2], T2 = tr[3];
      S k0 = exp(lo[0] + lo[1] * x.lnT - lo[2] / T);
      S dlnk0_dT = lo[1] / T + lo[2] / (T * T);
      S Pr = k0 * M / kf;
      S Fcent = (1.0 - alpha) * exp(-T / T3) + alpha * exp(-T / T1) + exp(-T2 / T);
      S dFcent_dT = -(1.0 - alpha) / T3 * exp(-T / T3) - alpha / T1 * exp(-T / T1) +
                    T2 / (T * T) * exp(-T2 / T);
      S xF = log10_(Fcent);
      S L = log10_(Pr);
      S c = -0.4 - 0.67 * xF;
      S n = 0.75 - 1.27 * xF;
      S d = n - 0.14 * (L + c);
      S f1 = (L + c) / d;
      S den = 1.0 + f1 * f1;
      S lgF = xF / den;
      S F = pow10_(lgF);
      out.keff = kf * Pr / (1.0 + Pr) * F;
      // derivatives of log10 F with respect to L = log10 Pr and x = log10 Fcent
      S df1_dL = n / (d * d);
      S df1_dx = (-0.67 * d + 1.1762 * (L + c)) / (d * d);
      S dlgF_dL = -xF * 2.0 * f1 / (den * den) * df1_dL;
      S dlgF_dx = 1.0 / den - xF * 2.0 * f1 / (den * den) * df1_dx;
      // d ln keff / d ln Pr = 1/(1+Pr) + d log10F / d log10 Pr ;  keff/[M] = k0 F/(1+Pr)
      S g = 1.0 / (1.0 + Pr) + dlgF_dL;
      out.dkeff_dM = k0 * F / (1.0 + Pr) * g;
      S dlnkeff_dT = dlnkf_dT + g * (dlnk0_dT - dlnkf_dT) + dlgF_dx * dFcent_dT / Fcent;
      out.dkeff_dT = out.keff * dlnkeff_dT;
    }
  }
  out.q = out.keff * (out.Rf - out.Rr / out.Kc);
  return out;
}

// f(Phi): dT/dt = -sum_k h_k omega_k / (rho c_p), dY_k/dt = W_k omega_k / rho
template <class S>
void rhs(const OracleMech& m, const Params<S>& P, double p, const S* y, S* f) {
  const int K = m.K;
  Mix<S> x;
  mixture(m, p, y, x);
  std::vector<S> omega(K, S(0.0));
  for (int r = 0; r < m.R; ++r) {
    Rate<S> rt = rate(m, P, x, r);
    for (int s = 0; s < 3; ++s) {
      if (m.reac[3 * r + s] >= 0) omega[m.reac[3 * r + s]] -= rt.q;
      if (m.prod[3 * r + s] >= 0) omega[m.prod[3 * r + s]] += rt.q;
    }
  }
  S Q(0.0);
  for (int k = 0; k < K; ++k) Q += x.hRT[k] * RU * x.T * omega[k];
  f[0] = -Q / (x.rho * x.cp);
  for (int k = 0; k < K; ++k) f[1 + k] = m.W[k] * omega[k] / x.rho;
}

// J by its definition: column j is the directional derivative of f along e_j,
// computed with forward-mode dual numbers.
void jac_ad(const OracleMech& m, const Params<double>& P, double p, const double* y, double* J) {
  const int N = m.K + 1;
  using D = Dual<double>;
  std::vector<D> lnA(m.R), b(m.R), th(m.R), yd(N), fd(N);
  for (int r = 0; r < m.R; ++r) { lnA[r] = D(P.lnA[r]); b[r] = D(P.b[r]); th[r] = D(P.theta[r]); }
  Params<D> PD{lnA.data(), b.data(), th.data()};
  for (int j = 0; j < N; ++j) {
    for (int i = 0; i < N; ++i) yd[i] = D(y[i], i == j ? 1.0 : 0.0);
    rhs(m, PD, p, yd.data(), fd.data());
    for (int i = 0; i < N; ++i) J[(size_t)i * N + j] = fd[i].d;
  }
}

// J from the hand-derived formulas.  With d C_i/d Y_j = rho delta_ij / W_i - C_i Wbar / W_j
// and d C_i / dT = -C_i / T:
//   J_kj = (W_k/W_j) dw_k/dC_j + W_k Wbar/(rho W_j) (w_k - sum_i C_i dw_k/dC_i)
//   J_kT = (W_k/rho) (dw_k/dT - (1/T) sum_i C_i dw_k/dC_i + w_k/T)
// and the T row from differentiating sum_k h_k f_k / W_k + c_p f_T = 0.
template <class S>
void jac_analytic(const OracleMech& m, const Params<S>& P, double p, const S* y, S* J, S* f) {
  const int K = m.K, N = K + 1;
  Mix<S> x;
  mixture(m, p, y, x);
  std::vector<S> omega(K, S(0.0)), dwdT(K, S(0.0)), dwdC((size_t)K * K, S(0.0));
  std::vector<S> dRf(K), dRr(K), dqdC(K);
  for (int r = 0; r < m.R; ++r) {
    Rate<S> rt = rate(m, P, x, r);
    const int* re = m.reac + 3 * r;
    const int* pr = m.prod + 3 * r;
    // d Rf / d C_j by the product rule over molecule slots (no division by C)
    for (int j = 0; j < K; ++j) { dRf[j] = S(0.0); dRr[j] = S(0.0); }
    for (int s = 0; s < 3; ++s) {
      if (re[s] >= 0) {
        S prodOther(1.0);
        for (int t = 0; t < 3; ++t)
          if (t != s && re[t] >= 0) prodOther *= x.C[re[t]];
        dRf[re[s]] += prodOther;
      }
      if (pr[s] >= 0) {
        S prodOther(1.0);
        for (int t = 0; t < 3; ++t)
          if (t != s && pr[t] >= 0) prodOther *= x.C[pr[t]];
        dRr[pr[s]] += prodOther;
      }
    }
    S net = rt.Rf - rt.Rr / rt.Kc;
    for (int j = 0; j < K; ++j) {
      dqdC[j] = rt.keff * (dRf[j] - dRr[j] / rt.Kc);
      if (m.rtype[r] != 0) dqdC[j] += rt.dkeff_dM * m.eff[(size_t)r * K + j] * net;
    }
    S dqdT = rt.dkeff_dT * net + rt.keff * rt.Rr / rt.Kc * rt.dlnKc_dT;
    for (int s = 0; s < 3; ++s) {
      const int sp[2] = {re[s], pr[s]};
      const double nu[2] = {-1.0, 1.0};
      for (int side = 0; side < 2; ++side) {
        int k = sp[side];
        if (k < 0) continue;
        omega[k] += nu[side] * rt.q;
        dwdT[k] += nu[side] * dqdT;
        for (int j = 0; j < K; ++j) dwdC[(size_t)k * K + j] += nu[side] * dqdC[j];
      }
    }
  }
  std::vector<S> F(K), hm(K), cpm(K);
  for (int k = 0; k < K; ++k) {
    F[k] = m.W[k] * omega[k] / x.rho;
    hm[k] = RU * x.T * x.hRT[k] / m.W[k];  // mass-specific enthalpy
    cpm[k] = RU * x.cpR[k] / m.W[k];       // mass-specific heat capacity
  }
  S Q(0.0);
  for (int k = 0; k < K; ++k) Q += x.hRT[k] * RU * x.T * omega[k];
  S FT = -Q / (x.rho * x.cp);
  for (int k = 0; k < K; ++k) {
    S sk(0.0);
    for (int i = 0; i < K; ++i) sk += x.C[i] * dwdC[(size_t)k * K + i];
    for (int j = 0; j < K; ++j)
      J[(size_t)(1 + k) * N + 1 + j] = (m.W[k] / m.W[j]) * dwdC[(size_t)k * K + j] +
                                       (m.W[k] * x.Wbar / (x.rho * m.W[j])) * (omega[k] - sk);
    J[(size_t)(1 + k) * N + 0] = (m.W[k] / x.rho) * (dwdT[k] - sk / x.T + omega[k] / x.T);
  }
  for (int j = 0; j < K; ++j) {
    S acc(0.0);
    for (int k = 0; k < K; ++k) acc += hm[k] * J[(size_t)(1 + k) * N + 1 + j];
    J[1 + j] = -(acc + FT * cpm[j]) / x.cp;
  }
  {
    S acc(0.0), acc2(0.0);
    for (int k = 0; k < K; ++k) {
      acc += hm[k] * J[(size_t)(1 + k) * N + 0];
      acc2 += cpm[k] * F[k];
    }
    J[0] = -(acc + acc2 + FT * x.dcpdT) / x.cp;
  }
  if (f) {
    f[0] = FT;
    for (int k = 0; k < K; ++k) f[1 + k] = F[k];
  }
}

// ----------------------------------------------------------------- dense LU
// Right-looking LU with partial pivoting (first index of max |a|), row
// interchanges recorded in piv, unit-lower L stored below the diagonal.
// With pivot = false the rows are taken in their natural order (no search).
template <class S> int lu_factor(S* A, int n, int* piv, bool pivot = true) {
  for (int k = 0; k < n; ++k) {
    int p = k;
    double amax = std::fabs(val(A[(size_t)k * n + k]));
    for (int i = k + 1; pivot && i < n; ++i) {
      double a = std::fabs(val(A[(size_t)i * n + k]));
      if (a > amax) { amax = a; p = i; }
    }
    piv[k] = p;
    if (amax == 0.0 || !std::isfinite(amax)) return k + 1;
    if (p != k)
      for (int j = 0; j < n; ++j) std::swap(A[(size_t)k * n + j], A[(size_t)p * n + j]);
    for (int i = k + 1; i < n; ++i) {
      A[(size_t)i * n + k] /= A[(size_t)k * n + k];
      for (int j = k + 1; j < n; ++j) A[(size_t)i * n + j] -= A[(size_t)i * n + k] * A[(size_t)k * n + j];
    }
  }
  return 0;
}

// Solve A x = b (trans = 0) or A^T x = b (trans = 1) with the factors of lu_factor.
template <class S> void lu_solve(const S* A, int n, const int* piv, S* b, int trans) {
  if (!trans) {
    for (int k = 0; k < n; ++k)
      if (piv[k] != k) std::swap(b[k], b[piv[k]]);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < i; ++j) b[i] -= A[(size_t)i * n + j] * b[j];
    for (int i = n - 1; i >= 0; --i) {
      for (int j = i + 1; j < n; ++j) b[i] -= A[(size_t)i * n + j] * b[j];
      b[i] /= A[(size_t)i * n + i];
    }
  } else {
    // (P^T L U)^T x = U^T L^T P x = b
    for (int i = 0; i < n; ++i) {
      for (int j = 0; j < i; ++j) b[i] -= A[(size_t)j * n + i] * b[j];
      b[i] /= A[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i)
      for (int j = i + 1; j < n; ++j) b[i] -= A[(size_t)j * n + i] * b[j];
    for (int k = n - 1; k >= 0; --k)
      if (piv[k] != k) std::swap(b[k], b[piv[k]]);
  }
}

// ------------------------------------------------------- Rosenbrock tables
// Transformed form (Hairer & Wanner IV.7):  M = I/(gamma h) - J,
//   M K_i = f(y + sum_{j<i} a_ij K_j) + sum_{j<i} (c_ij / h) K_j,
//   y_new = y + sum m_i K_i,   err = sum e_i K_i.
struct Table {
  int s;
  double gamma;
  double a[4][4], c[4][4], m[4], e[4];
  double order_err;  // exponent 1/q of the step-size controller uses q
};

Table ros4() {
  // ROS4 with Shampine's parameters (as tabulated by Sandu et al. 1997)
  Table t{};
  t.s = 4;
  t.gamma = 0.57282;
  t.a[1][0] = 2.0;
  t.a[2][0] = 1.867943637803922;
  t.a[2][1] = 0.2344449711399156;
  t.a[3][0] = 1.867943637803922;
  t.a[3][1] = 0.2344449711399156;
  t.a[3][2] = 0.0;
  t.c[1][0] = -7.137615036412310;
  t.c[2][0] = 2.580708087951457;
  t.c[2][1] = 0.6515950076447975;
  t.c[3][0] = -2.137148994382534;
  t.c[3][1] = -0.3214669691237626;
  t.c[3][2] = -0.6949742501781779;
  const double m[4] = {2.255570073418735, 0.2870493262186792, 0.4353179431840180, 1.093502252409163};
  const double e[4] = {-0.2815431932141155, -0.07276199124938920, -0.1082196201495311, -1.093502252409163};
  for (int i = 0; i < 4; ++i) { t.m[i] = m[i]; t.e[i] = e[i]; }
  t.order_err = 4.0;
  return t;
}

Table rodas3() {
  // Rodas3 (Sandu et al. 1997): stiffly accurate, order 3 with embedded 2
  Table t{};
  t.s = 4;
  t.gamma = 0.5;
  t.a[2][0] = 2.0;
  t.a[3][0] = 2.0;
  t.a[3][2] = 1.0;
  t.c[1][0] = 4.0;
  t.c[2][0] = 1.0;
  t.c[2][1] = -1.0;
  t.c[3][0] = 1.0;
  t.c[3][1] = -1.0;
  t.c[3][2] = -8.0 / 3.0;
  const double m[4] = {2.0, 0.0, 1.0, 1.0};
  const double e[4] = {0.0, 0.0, 0.0, 1.0};
  for (int i = 0; i < 4; ++i) { t.m[i] = m[i]; t.e[i] = e[i]; }
  t.order_err = 3.0;
  return t;
}

Table euler_eq2() {
  // Eq. 2 of the paper: (I - h J)(y_new - y) = h f, i.e. one stage, gamma = 1, m = 1
  Table t{};
  t.s = 1;
  t.gamma = 1.0;
  t.m[0] = 1.0;
  t.e[0] = 0.0;
  t.order_err = 1.0;
  return t;
}

Table table_of(int method) {
  if (method == 1) return rodas3();
  if (method == 2) return euler_eq2();
  return ros4();
}

// Does stage i evaluate f at a point no earlier stage used?
bool stage_needs_f(const Table& t, int i) {
  if (i == 0) return false;
  for (int j = 0; j < i; ++j) {
    bool same = true;
    for (int l = 0; l < 4; ++l)
      if (t.a[i][l] != t.a[j][l]) same = false;
    if (same) return false;
  }
  return true;
}
int stage_source(const Table& t, int i) {
  for (int j = 0; j < i; ++j) {
    bool same = true;
    for (int l = 0; l < 4; ++l)
      if (t.a[i][l] != t.a[j][l]) same = false;
    if (same) return j;
  }
  return i;
}

// One Rosenbrock step of size h from y, given f0 = f(y) and J = J(y).
// Returns 0, or 1 if M is singular.
template <class S, class Rhs>
int ros_step(const Table& t, int N, Rhs&& frhs, const S* y, const S* f0, const S* J, double h, S* ynew,
             S* err, bool pivot = true) {
  std::vector<S> M((size_t)N * N), K((size_t)4 * N), fst((size_t)4 * N), Y(N), rhsv(N);
  std::vector<int> piv(N);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) M[(size_t)i * N + j] = (i == j ? S(1.0 / (t.gamma * h)) : S(0.0)) - J[(size_t)i * N + j];
  if (lu_factor(M.data(), N, piv.data(), pivot)) return 1;
  for (int i = 0; i < t.s; ++i) {
    S* fi = &fst[(size_t)i * N];
    if (i == 0) {
      for (int l = 0; l < N; ++l) fi[l] = f0[l];
    } else if (stage_needs_f(t, i)) {
      for (int l = 0; l < N; ++l) {
        Y[l] = y[l];
        for (int j = 0; j < i; ++j) Y[l] += t.a[i][j] * K[(size_t)j * N + l];
      }
      frhs(Y.data(), fi);
    } else {
      const S* src = &fst[(size_t)stage_source(t, i) * N];
      for (int l = 0; l < N; ++l) fi[l] = src[l];
    }
    for (int l = 0; l < N; ++l) {
      rhsv[l] = fi[l];
      for (int j = 0; j < i; ++j) rhsv[l] += (t.c[i][j] / h) * K[(size_t)j * N + l];
    }
    lu_solve(M.data(), N, piv.data(), rhsv.data(), 0);
    for (int l = 0; l < N; ++l) K[(size_t)i * N + l] = rhsv[l];
  }
  for (int l = 0; l < N; ++l) {
    ynew[l] = y[l];
    err[l] = S(0.0);
    for (int i = 0; i < t.s; ++i) {
      ynew[l] += t.m[i] * K[(size_t)i * N + l];
      err[l] += t.e[i] * K[(size_t)i * N + l];
    }
  }
  return 0;
}

bool all_finite(const double* v, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

struct CellResult {
  int status, steps, rejects;
};

// One-sided finite-difference Jacobian, column j from f(y + d_j e_j):
// d_j = sqrt(eps) max(|y_j|, 1e-10), rounded so that y_j + d_j - y_j = d_j.
constexpr double FD_REL = 1.4901161193847656e-08, FD_FLOOR = 1e-10;
void jac_fd(const OracleMech& m, const Params<double>& P, double p, const double* y, double* J, double* f0) {
  const int N = m.K + 1;
  rhs(m, P, p, y, f0);
  std::vector<double> yp(y, y + N), fp(N);
  for (int j = 0; j < N; ++j) {
    double d = FD_REL * std::max(std::fabs(y[j]), FD_FLOOR);
    d = (y[j] + d) - y[j];
    yp[j] = y[j] + d;
    rhs(m, P, p, yp.data(), fp.data());
    for (int i = 0; i < N; ++i) J[(size_t)i * N + j] = (fp[i] - f0[i]) / d;
    yp[j] = y[j];
  }
}

// ------------------------------------------ extrapolated linearly implicit Euler
// The Seulex family (the paper's integrator, section 2.3; Hairer & Wanner,
// Solving ODEs II, section IV.9): over a step H with J = J(y0) frozen, column
// j (1-based) takes n_j = j linearly implicit Euler substeps of size h = H/n_j,
//   (I/h - J)(y_{m+1} - y_m) = f(y_m),
// and the Aitken-Neville table
//   T_{j,l+1} = T_{j,l} + (T_{j,l} - T_{j-1,l}) / (n_j / n_{j-l} - 1)
// raises the order by one per column (T_{j,j} has order j).  Column j's error
// estimate is ||T_{j,j} - T_{j,j-1}||, which scales as H^j.
constexpr int SX_KMAX = 6;

// Fills T[j][l] (0-based, l <= j < kcols); returns 1 if an iteration matrix is singular.
// With stab, a stability check in the manner of Hairer & Wanner IV.9 (the
// second increment of a column must not exceed the first in the scaled norm
// sc_i = atol + rtol |y0_i|, else return 2); the integrator leaves it off: on
// these mechanisms it rejects sound steps during fast transients.
template <class Rhs>
int seulex_table(int N, Rhs&& frhs, const double* y0, const double* f0, const double* J, double H, int kcols,
                 std::vector<std::vector<std::vector<double>>>& T, bool pivot, double rtol = 0.0,
                 double atol = 0.0, bool stab = false) {
  std::vector<double> M((size_t)N * N), yc(N), f(N), d(N);
  std::vector<int> piv(N);
  auto dnorm = [&](const std::vector<double>& v) {
    double s2 = 0.0;
    for (int i = 0; i < N; ++i) {
      const double e = v[i] / (atol + rtol * std::fabs(y0[i]));
      s2 += e * e;
    }
    return std::sqrt(s2 / N);
  };
  for (int j = 0; j < kcols; ++j) {
    const int nj = j + 1;
    const double h = H / nj;
    for (int a = 0; a < N; ++a)
      for (int b = 0; b < N; ++b) M[(size_t)a * N + b] = (a == b ? 1.0 / h : 0.0) - J[(size_t)a * N + b];
    if (lu_factor(M.data(), N, piv.data(), pivot)) return 1;
    for (int i = 0; i < N; ++i) yc[i] = y0[i];
    double del1 = 0.0;
    for (int mm = 0; mm < nj; ++mm) {
      if (mm == 0) {
        for (int i = 0; i < N; ++i) d[i] = f0[i];
      } else {
        frhs(yc.data(), f.data());
        for (int i = 0; i < N; ++i) d[i] = f[i];
      }
      lu_solve(M.data(), N, piv.data(), d.data(), 0);
      for (int i = 0; i < N; ++i) yc[i] += d[i];
      if (stab) {
        if (mm == 0) del1 = dnorm(d);
        else if (mm == 1 && !(dnorm(d) <= del1)) return 2;
      }
    }
    T[j][0] = yc;
    for (int l = 1; l <= j; ++l) {
      const double r = (double)(j + 1 - l) / l;  // 1 / (n_j / n_{j-l} - 1) for n_j = j
      for (int i = 0; i < N; ++i) T[j][l][i] = T[j][l - 1][i] + (T[j][l - 1][i] - T[j - 1][l - 1][i]) * r;
    }
  }
  return 0;
}

double sx_err(int N, const std::vector<double>& a, const std::vector<double>& b, const double* y0, double rtol,
              double atol) {
  double s2 = 0.0;
  for (int i = 0; i < N; ++i) {
    const double sc = atol + rtol * std::max(std::fabs(y0[i]), std::fabs(a[i]));
    const double e = (a[i] - b[i]) / sc;
    s2 += e * e;
  }
  return std::sqrt(s2 / N);
}

// One record per step attempt, for the controller pins: the step size tried,
// the scaled error norm (NaN when none was formed), the outcome and, for the
// Seulex family, the column count k of the attempt.
enum { AT_ACCEPT = 0, AT_REJECT_ERR = 1, AT_REJECT_NONFINITE = 2, AT_REJECT_SINGULAR = 3, AT_REJECT_UNSTABLE = 4 };
struct Attempt {
  double h, err;
  int outcome, k;
};

// The chemistry system: N = K + 1, f and J at a state (J analytic or by
// one-sided differences, the ablation's jac_mode 1).  A state is valid if it is
// finite with T > 0.
struct ChemSystem {
  const OracleMech& m;
  Params<double> P;
  double p;
  int jac_mode;
  int size() const { return m.K + 1; }
  bool valid(const double* y) const { return all_finite(y, m.K + 1) && y[0] > 0.0; }
  void f(const double* y, double* out) const { rhs(m, P, p, y, out); }
  void jac(const double* y, double* J, double* f0) const {
    if (jac_mode == 1) jac_fd(m, P, p, y, J, f0);
    else jac_analytic(m, P, p, y, J, f0);
  }
};

// Adaptive Seulex integration of one cell over [0, dt].  Order control: the
// target column k starts at 3; after an accepted step the next k among k-1,
// k, k+1 minimises the work per unit step A_j / H_j, with A_j = sum_{i<=j}
// (n_i + 1) (substeps plus one factorisation per column) and H_j the step
// that column j's error proposes, H fac_safe err_j^(-1/j) clamped by
// fac_min / fac_max.  Rejections keep k and take H_k; the controller's other
// rules (clipping to dt, no growth after a rejection, h_out, limits, halving
// on a singular matrix) are those of the Rosenbrock path.
template <class Sys>
CellResult integrate_seulex(const Sys& sys, double dt, double rtol, double atol, const OracleOpts& o, double* y,
                            double* h_io, std::vector<double>* hs_out, std::vector<Attempt>* trace = nullptr) {
  const int N = sys.size();
  auto frhs = [&](const double* yy, double* ff) { sys.f(yy, ff); };
  CellResult res{ST_OK, 0, 0};
  std::vector<double> f0(N), J((size_t)N * N);
  std::vector<std::vector<std::vector<double>>> T(SX_KMAX, std::vector<std::vector<double>>(SX_KMAX,
                                                  std::vector<double>(N)));
  double A[SX_KMAX + 2];
  A[0] = 0.0;
  for (int j = 1; j <= SX_KMAX + 1; ++j) A[j] = A[j - 1] + (j + 1);
  double h_prop = (std::isfinite(*h_io) && *h_io > 0.0) ? std::min(*h_io, dt) : dt;
  if (!sys.valid(y)) {
    res.status = ST_NONFINITE;
    *h_io = h_prop;
    return res;
  }
  int k = 3;
  double tcur = 0.0;
  bool rejected_last = false;
  int attempts = 0;
  auto hopt = [&](double H, double err, int j) {
    return H * std::min(o.fac_max, std::max(o.fac_min, o.fac_safe * std::pow(err, -1.0 / j)));
  };
  auto rec = [&](double H, double err, int outcome) {
    if (trace) trace->push_back(Attempt{H, err, outcome, k});
  };
  while (tcur < dt) {
    sys.jac(y, J.data(), f0.data());
    if (!all_finite(f0.data(), N) || !all_finite(J.data(), N * N)) { res.status = ST_NONFINITE; break; }
    int nsing = 0;
    bool accepted = false;
    while (!accepted) {
      if (attempts >= o.max_steps) { res.status = ST_TOO_MANY_STEPS; break; }
      if (!(h_prop >= o.h_min)) { res.status = ST_UNDERFLOW; break; }
      double H = h_prop;
      bool clipped = false;
      if (H >= dt - tcur) { H = dt - tcur; clipped = true; }
      ++attempts;
      const int rc = seulex_table(N, frhs, y, f0.data(), J.data(), H, k, T, o.lu_pivot == 0, rtol, atol);
      if (rc == 1) {
        rec(H, NAN, AT_REJECT_SINGULAR);
        ++res.rejects;
        if (++nsing > 5) { res.status = ST_SINGULAR; break; }
        h_prop = 0.5 * H;
        rejected_last = true;
        continue;
      }
      if (rc == 2) {  // unstable substeps
        rec(H, NAN, AT_REJECT_UNSTABLE);
        ++res.rejects;
        h_prop = 0.5 * H;
        rejected_last = true;
        continue;
      }
      const std::vector<double>& yk = T[k - 1][k - 1];
      const double errk = sx_err(N, yk, T[k - 1][k - 2], y, rtol, atol);
      if (!std::isfinite(errk) || !all_finite(yk.data(), N)) {
        rec(H, errk, AT_REJECT_NONFINITE);
        ++res.rejects;
        h_prop = o.fac_min * H;
        rejected_last = true;
        continue;
      }
      const double Hk = hopt(H, errk, k);
      // column k-1's proposal (for the order decision), from the same step start
      double Hk1 = 0.0;
      if (k >= 3) {
        const double e1 = sx_err(N, T[k - 2][k - 2], T[k - 2][k - 3], y, rtol, atol);
        if (std::isfinite(e1)) Hk1 = hopt(H, e1, k - 1);
      }
      if (errk <= 1.0) {
        rec(H, errk, AT_ACCEPT);
        accepted = true;
        ++res.steps;
        if (hs_out) hs_out->push_back(H);
        tcur = clipped ? dt : tcur + H;
        for (int i = 0; i < N; ++i) y[i] = yk[i];
        int knew = k;
        double hnew = Hk;
        if (k >= 3 && Hk1 > 0.0 && A[k - 1] / Hk1 < 0.8 * (A[k] / Hk)) {
          knew = k - 1;
          hnew = Hk1;
        } else if (k < SX_KMAX && (k == 2 || Hk1 <= 0.0 || A[k] / Hk < 0.9 * (A[k - 1] / Hk1))) {
          knew = k + 1;
          hnew = Hk * (A[k + 1] / A[k]);
        }
        if (rejected_last) {
          hnew = std::min(hnew, H);
          knew = std::min(knew, k);
        }
        if (clipped) hnew = std::max(hnew, h_prop);
        h_prop = hnew;
        k = knew;
        rejected_last = false;
      } else {
        rec(H, errk, AT_REJECT_ERR);
        ++res.rejects;
        h_prop = Hk;
        rejected_last = true;
      }
    }
    if (res.status != ST_OK) break;
  }
  *h_io = std::min(h_prop, dt);
  return res;
}

// Adaptive Rosenbrock integration of one cell over [0, dt] (controller
// constants in opts; the rules are listed with the C API below).
template <class Sys>
CellResult integrate_ros(const Sys& sys, int method, double dt, double rtol, double atol, const OracleOpts& o,
                         double* y, double* h_io, std::vector<double>* hs_out,
                         std::vector<Attempt>* trace = nullptr) {
  const int N = sys.size();
  const Table t = table_of(method);
  auto frhs = [&](const double* yy, double* ff) { sys.f(yy, ff); };
  CellResult res{ST_OK, 0, 0};
  std::vector<double> f0(N), J((size_t)N * N), yn(N), err(N);
  double h_prop = (std::isfinite(*h_io) && *h_io > 0.0) ? std::min(*h_io, dt) : dt;
  if (!sys.valid(y)) {
    res.status = ST_NONFINITE;
    *h_io = h_prop;
    return res;
  }
  double tcur = 0.0;
  bool rejected_last = false;
  int attempts = 0;
  auto rec = [&](double h, double e, int outcome) {
    if (trace) trace->push_back(Attempt{h, e, outcome, 0});
  };
  while (tcur < dt) {
    sys.jac(y, J.data(), f0.data());
    if (!all_finite(f0.data(), N) || !all_finite(J.data(), N * N)) { res.status = ST_NONFINITE; break; }
    int nsing = 0;
    bool accepted = false;
    while (!accepted) {
      if (attempts >= o.max_steps) { res.status = ST_TOO_MANY_STEPS; break; }
      if (!(h_prop >= o.h_min)) { res.status = ST_UNDERFLOW; break; }
      double h = h_prop;
      bool clipped = false;
      if (h >= dt - tcur) { h = dt - tcur; clipped = true; }
      ++attempts;
      if (ros_step(t, N, frhs, y, f0.data(), J.data(), h, yn.data(), err.data(), o.lu_pivot == 0)) {
        rec(h, NAN, AT_REJECT_SINGULAR);
        ++res.rejects;
        if (++nsing > 5) { res.status = ST_SINGULAR; break; }
        h_prop = 0.5 * h;
        rejected_last = true;
        continue;
      }
      // err = sqrt(mean((err_i / (atol + rtol max(|y_i|, |ynew_i|)))^2))
      double s2 = 0.0;
      for (int i = 0; i < N; ++i) {
        double sc = atol + rtol * std::max(std::fabs(y[i]), std::fabs(yn[i]));
        double e = err[i] / sc;
        s2 += e * e;
      }
      double enorm = std::sqrt(s2 / N);
      if (!std::isfinite(enorm) || !all_finite(yn.data(), N)) {
        rec(h, enorm, AT_REJECT_NONFINITE);
        ++res.rejects;
        h_prop = o.fac_min * h;
        rejected_last = true;
        continue;
      }
      double fac = std::min(o.fac_max, std::max(o.fac_min, o.fac_safe * std::pow(enorm, -1.0 / t.order_err)));
      if (enorm <= 1.0) {
        rec(h, enorm, AT_ACCEPT);
        accepted = true;
        ++res.steps;
        if (hs_out) hs_out->push_back(h);
        tcur = clipped ? dt : tcur + h;
        for (int i = 0; i < N; ++i) y[i] = yn[i];
        double hnew = h * fac;
        if (rejected_last) hnew = std::min(hnew, h);
        if (clipped) hnew = std::max(hnew, h_prop);
        h_prop = hnew;
        rejected_last = false;
      } else {
        rec(h, enorm, AT_REJECT_ERR);
        ++res.rejects;
        h_prop = h * fac;
        rejected_last = true;
      }
    }
    if (res.status != ST_OK) break;
  }
  *h_io = std::min(h_prop, dt);
  return res;
}

// Linear test system for the controller pins: y' = diag(lam) y, J = diag(lam)
// exactly; component i of f is NaN where |y_i| > bound (bound <= 0: none).
// Every step of a Rosenbrock or extrapolation method on it is a rational
// function of h lam_i, so the whole controller trace has a closed form.
struct DiagSystem {
  int n;
  const double* lam;
  double bound;
  int size() const { return n; }
  bool valid(const double* y) const { return all_finite(y, n); }
  void f(const double* y, double* out) const {
    for (int i = 0; i < n; ++i) out[i] = (bound > 0.0 && std::fabs(y[i]) > bound) ? NAN : lam[i] * y[i];
  }
  void jac(const double* y, double* J, double* f0) const {
    f(y, f0);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) J[(size_t)i * n + j] = i == j ? lam[i] : 0.0;
  }
};

// Adaptive integration of one chemistry cell over [0, dt].
CellResult integrate_cell(const OracleMech& m, double p, double dt, double rtol, double atol, const OracleOpts& o,
                          double* y, double* h_io, std::vector<double>* hs_out) {
  const ChemSystem sys{m, Params<double>{m.lnA, m.b, m.theta}, p, o.jac_mode};
  if (o.method == 3) return integrate_seulex(sys, dt, rtol, atol, o, y, h_io, hs_out);
  return integrate_ros(sys, o.method, dt, rtol, atol, o, y, h_io, hs_out);
}

// Replay accepted steps hs[0..n) from y0 without the controller, in scalar type S.
template <class S>
int replay(const OracleMech& m, const Params<S>& P, double p, int method, const S* y0, const double* hs, int n,
           S* yout) {
  const int N = m.K + 1;
  const Table t = table_of(method);
  std::vector<S> y(y0, y0 + N), f0(N), J((size_t)N * N), yn(N), err(N);
  auto frhs = [&](const S* yy, S* ff) { rhs(m, P, p, yy, ff); };
  for (int s = 0; s < n; ++s) {
    jac_analytic(m, P, p, y.data(), J.data(), f0.data());
    if (ros_step(t, N, frhs, y.data(), f0.data(), J.data(), hs[s], yn.data(), err.data())) return 1;
    y = yn;
  }
  for (int i = 0; i < N; ++i) yout[i] = y[i];
  return 0;
}

// Built-in test problems for the tables (Hairer & Wanner style order checks).
//   problem 0: y1' = -y1^2, y2' = y1 y2  (exact 1/(1+t), 1+t from (1,1))
//   problem 1: y' = lambda y with lambda = y0[1] carried as a constant
void test_rhs(int problem, const double* y, double* f, double lam) {
  if (problem == 0) {
    f[0] = -y[0] * y[0];
    f[1] = y[0] * y[1];
  } else {
    f[0] = lam * y[0];
  }
}
void test_jac(int problem, const double* y, double* J, double lam) {
  if (problem == 0) {
    J[0] = -2.0 * y[0]; J[1] = 0.0;
    J[2] = y[1];        J[3] = y[0];
  } else {
    J[0] = lam;
  }
}

}  // namespace

// ====================================================================== C API
extern "C" {

double oracle_gas_constant() { return RU; }

int oracle_rhs(const OracleMech* m, double p_pa, const double* y, double* f) {
  Params<double> P{m->lnA, m->b, m->theta};
  rhs(*m, P, 10.0 * p_pa, y, f);
  return 0;
}

// mode 0: analytic formulas, 1: dual-number AD (the definition)
int oracle_jac(const OracleMech* m, double p_pa, const double* y, double* J, int mode) {
  if (mode == 2) {  // one-sided finite differences (the integrator's jac_mode 1)
    Params<double> P{m->lnA, m->b, m->theta};
    std::vector<double> f0(m->K + 1);
    jac_fd(*m, P, 10.0 * p_pa, y, J, f0.data());
    return 0;
  }
  Params<double> P{m->lnA, m->b, m->theta};
  if (mode == 1) {
    jac_ad(*m, P, 10.0 * p_pa, y, J);
  } else {
    std::vector<double> f(m->K + 1);
    jac_analytic(*m, P, 10.0 * p_pa, y, J, f.data());
  }
  return 0;
}

// Rates of progress of every reaction and species production rates omega.
int oracle_rates(const OracleMech* m, double p_pa, const double* y, double* q, double* kf_eff, double* Kc) {
  Params<double> P{m->lnA, m->b, m->theta};
  Mix<double> x;
  mixture(*m, 10.0 * p_pa, y, x);
  for (int r = 0; r < m->R; ++r) {
    Rate<double> rt = rate(*m, P, x, r);
    if (q) q[r] = rt.q;
    if (kf_eff) kf_eff[r] = rt.keff;
    if (Kc) Kc[r] = rt.Kc;
  }
  return 0;
}

// Operation counts of one f evaluation (out[0..4]: add, mul, div, exp, log)
// and of one analytic Jacobian pass, which also yields f (out[5..9]), at
// state y, on the counting scalar (structurally zero terms are free).
int oracle_op_counts(const OracleMech* m, double p_pa, const double* y, double* out) {
  const int N = m->K + 1, R = m->R;
  std::vector<Cnt> lnA(R), b(R), th(R), yc(N), f(N), J((size_t)N * N);
  for (int r = 0; r < R; ++r) { lnA[r] = Cnt(m->lnA[r]); b[r] = Cnt(m->b[r]); th[r] = Cnt(m->theta[r]); }
  for (int i = 0; i < N; ++i) yc[i] = Cnt(y[i]);
  Params<Cnt> P{lnA.data(), b.data(), th.data()};
  g_ops = OpTally{};
  rhs(*m, P, 10.0 * p_pa, yc.data(), f.data());
  const OpTally a = g_ops;
  g_ops = OpTally{};
  jac_analytic(*m, P, 10.0 * p_pa, yc.data(), J.data(), f.data());
  const OpTally j = g_ops;
  const OpTally* t[2] = {&a, &j};
  for (int q = 0; q < 2; ++q) {
    out[5 * q + 0] = t[q]->add;
    out[5 * q + 1] = t[q]->mul;
    out[5 * q + 2] = t[q]->div;
    out[5 * q + 3] = t[q]->exp;
    out[5 * q + 4] = t[q]->log;
  }
  return 0;
}

// Species thermo at T: cp/R, h/RT, s/R for all K species.
int oracle_thermo(const OracleMech* m, double T, double* cpR, double* hRT, double* sR) {
  for (int k = 0; k < m->K; ++k) {
    double a, b, c, d;
    thermo(*m, k, T, std::log(T), a, b, c, d);
    cpR[k] = a; hRT[k] = b; sR[k] = c;
  }
  return 0;
}

int oracle_lu_factor(int n, double* A, int* piv) { return lu_factor(A, n, piv); }
int oracle_lu_factor_nopivot(int n, double* A, int* piv) { return lu_factor(A, n, piv, false); }
void oracle_lu_solve(int n, const double* A, const int* piv, double* b, int trans) { lu_solve(A, n, piv, b, trans); }

// Batched adaptive integration: state is SoA [N][ld] (row 0 T, rows 1..K Y), in place.
int oracle_integrate(const OracleMech* m, int64_t ncells, int64_t ld, double* state, double* h, double p_pa,
                     double dt, double rtol, double atol, const OracleOpts* o, int32_t* steps, int32_t* rejects,
                     int32_t* status, int nthreads) {
  const int N = m->K + 1;
#ifdef _OPENMP
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
#endif
  for (int64_t c = 0; c < ncells; ++c) {
    std::vector<double> y(N);
    for (int i = 0; i < N; ++i) y[i] = state[(size_t)i * ld + c];
    CellResult r = integrate_cell(*m, 10.0 * p_pa, dt, rtol, atol, *o, y.data(), &h[c], nullptr);
    for (int i = 0; i < N; ++i) state[(size_t)i * ld + c] = y[i];
    if (steps) steps[c] = r.steps;
    if (rejects) rejects[c] = r.rejects;
    if (status) status[c] = r.status;
  }
  (void)nthreads;
  return 0;
}

// Reference-cell mapping.  Section 2.2 describes DLBFoam's zonal reference
// mapping: in low-reactivity (ambient) regions the chemistry solution of one
// reference cell is mapped onto the others instead of integrating each.  The
// paper gives no criterion; the one here is this library's reading:
//  * indicator z_c = z0 + sum_k w_k Y_k (species in index order, each term a
//    fused multiply-add); cell c is in the low-reactivity zone if z_c <= z_max
//    (a linear indicator covers a fuel mass fraction and Bilger's mixture
//    fraction alike);
//  * the reference r is the zone cell of lowest index;
//  * a zone cell c != r is mapped if |T_c - T_r| <= dT: it is not integrated
//    and takes the reference's increment per unit mass,
//    Phi_c(dt) = Phi_c(0) + (Phi_r(dt) - Phi_r(0)), with h_c = h_r after the
//    call, zero steps and rejects, and the reference's status;
//  * every other cell, r included, is integrated.
// ref_of[c] receives r for a mapped cell, -1 otherwise.
int oracle_integrate_refmap(const OracleMech* m, int64_t ncells, int64_t ld, double* state, double* h, double p_pa,
                            double dt, double rtol, double atol, const OracleOpts* o, const double* w, double z0,
                            double z_max, double dT, int32_t* ref_of, int32_t* steps, int32_t* rejects,
                            int32_t* status, int nthreads) {
  const int N = m->K + 1;
  std::vector<char> zone(ncells, 0);
  int64_t r = -1;
  for (int64_t c = 0; c < ncells; ++c) {
    double z = z0;
    for (int k = 0; k < m->K; ++k) z = std::fma(w[k], state[(size_t)(k + 1) * ld + c], z);
    zone[c] = z <= z_max;
    if (zone[c] && r < 0) r = c;
  }
  std::vector<int64_t> active;
  for (int64_t c = 0; c < ncells; ++c) {
    const bool mapped = r >= 0 && c != r && zone[c] && std::fabs(state[c] - state[r]) <= dT;
    ref_of[c] = mapped ? (int32_t)r : -1;
    if (!mapped) active.push_back(c);
  }
  std::vector<double> y0r(N);
  if (r >= 0)
    for (int i = 0; i < N; ++i) y0r[i] = state[(size_t)i * ld + r];
  // the unmapped cells, gathered into a dense SoA block and integrated
  const int64_t na = (int64_t)active.size();
  std::vector<double> sub((size_t)N * na), hsub(na);
  std::vector<int32_t> ssub(na), rsub(na), stsub(na);
  for (int64_t j = 0; j < na; ++j) {
    for (int i = 0; i < N; ++i) sub[(size_t)i * na + j] = state[(size_t)i * ld + active[j]];
    hsub[j] = h[active[j]];
  }
  oracle_integrate(m, na, na, sub.data(), hsub.data(), p_pa, dt, rtol, atol, o, ssub.data(), rsub.data(),
                   stsub.data(), nthreads);
  int32_t st_r = 0;
  double h_r = 0.0;
  for (int64_t j = 0; j < na; ++j) {
    const int64_t c = active[j];
    for (int i = 0; i < N; ++i) state[(size_t)i * ld + c] = sub[(size_t)i * na + j];
    h[c] = hsub[j];
    if (steps) steps[c] = ssub[j];
    if (rejects) rejects[c] = rsub[j];
    if (status) status[c] = stsub[j];
    if (c == r) {
      st_r = stsub[j];
      h_r = hsub[j];
    }
  }
  for (int64_t c = 0; c < ncells; ++c) {
    if (ref_of[c] < 0) continue;
    for (int i = 0; i < N; ++i)
      state[(size_t)i * ld + c] = state[(size_t)i * ld + c] + (state[(size_t)i * ld + r] - y0r[i]);
    h[c] = h_r;
    if (steps) steps[c] = 0;
    if (rejects) rejects[c] = 0;
    if (status) status[c] = st_r;
  }
  return 0;
}

// One cell, also returning the accepted step sizes (capacity cap).
int oracle_integrate_record(const OracleMech* m, double p_pa, double dt, double rtol, double atol,
                            const OracleOpts* o, double* y, double* h, double* hs, int cap, int32_t* nsteps,
                            int32_t* nrejects) {
  std::vector<double> rec;
  CellResult r = integrate_cell(*m, 10.0 * p_pa, dt, rtol, atol, *o, y, h, &rec);
  *nsteps = r.steps;
  if (nrejects) *nrejects = r.rejects;
  for (int i = 0; i < (int)rec.size() && i < cap; ++i) hs[i] = rec[i];
  return r.status;
}

int oracle_replay(const OracleMech* m, double p_pa, int method, const double* y0, const double* hs, int n,
                  double* yout) {
  Params<double> P{m->lnA, m->b, m->theta};
  return replay(*m, P, 10.0 * p_pa, method, y0, hs, n, yout);
}

// Tangent-linear model of the replayed integration: derivative of the final
// state along the direction (dy0, dlnA, db, dtheta); any direction pointer may be NULL.
int oracle_tlm(const OracleMech* m, double p_pa, int method, const double* y0, const double* hs, int n,
               const double* dy0, const double* dlnA, const double* db, const double* dth, double* yout,
               double* dyout) {
  using D = Dual<double>;
  const int N = m->K + 1, R = m->R;
  std::vector<D> lnA(R), b(R), th(R), y(N), yo(N);
  for (int r = 0; r < R; ++r) {
    lnA[r] = D(m->lnA[r], dlnA ? dlnA[r] : 0.0);
    b[r] = D(m->b[r], db ? db[r] : 0.0);
    th[r] = D(m->theta[r], dth ? dth[r] : 0.0);
  }
  for (int i = 0; i < N; ++i) y[i] = D(y0[i], dy0 ? dy0[i] : 0.0);
  Params<D> P{lnA.data(), b.data(), th.data()};
  int rc = replay(*m, P, 10.0 * p_pa, method, y.data(), hs, n, yo.data());
  for (int i = 0; i < N; ++i) {
    yout[i] = yo[i].v;
    dyout[i] = yo[i].d;
  }
  return rc;
}

// The adaptive integrators on the linear test system DiagSystem (n components,
// rates lam, NaN bound), with every step attempt recorded: trace[a] = (h, err,
// outcome, k) for a < min(attempts, cap); outcome 0 accepted, 1 rejected on
// the error, 2 rejected on a non-finite error, 3 singular matrix, 4 unstable
// substeps.  method 0 ROS4, 1 Rodas3, 2 Eq. 2, 3 Seulex family.  Returns the
// cell status; y and h_io are updated as for a chemistry cell.
int oracle_controller_test(int method, int n, const double* lam, double bound, double* y, double dt, double rtol,
                           double atol, const OracleOpts* o, double* h_io, double* trace, int cap,
                           int32_t* nattempts, int32_t* steps, int32_t* rejects) {
  const DiagSystem sys{n, lam, bound};
  std::vector<Attempt> tr;
  CellResult r = method == 3 ? integrate_seulex(sys, dt, rtol, atol, *o, y, h_io, nullptr, &tr)
                             : integrate_ros(sys, method, dt, rtol, atol, *o, y, h_io, nullptr, &tr);
  for (int a = 0; a < (int)tr.size() && a < cap; ++a) {
    trace[4 * a + 0] = tr[a].h;
    trace[4 * a + 1] = tr[a].err;
    trace[4 * a + 2] = tr[a].outcome;
    trace[4 * a + 3] = tr[a].k;
  }
  *nattempts = (int32_t)tr.size();
  *steps = r.steps;
  *rejects = r.rejects;
  return r.status;
}

// The full forward-sensitivity matrix of the replayed integration: column j
// of S ([N][N + 3R], row-major) is the derivative of the final state with
// respect to z_j, z = (y0, lnA, b, theta), each from its own tangent-linear
// replay (columns in parallel).  Returns the first nonzero replay code.
int oracle_tlm_matrix(const OracleMech* m, double p_pa, int method, const double* y0, const double* hs, int n,
                      double* S, int nthreads) {
  const int N = m->K + 1, R = m->R, NZ = N + 3 * R;
  int rc_all = 0;
#ifdef _OPENMP
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
#endif
  for (int j = 0; j < NZ; ++j) {
    std::vector<double> dy0(N, 0.0), dl(R, 0.0), db(R, 0.0), dt(R, 0.0), yo(N), dyo(N);
    if (j < N) dy0[j] = 1.0;
    else if (j < N + R) dl[j - N] = 1.0;
    else if (j < N + 2 * R) db[j - N - R] = 1.0;
    else dt[j - N - 2 * R] = 1.0;
    const int rc = oracle_tlm(m, p_pa, method, y0, hs, n, dy0.data(), dl.data(), db.data(), dt.data(), yo.data(),
                              dyo.data());
    if (rc) {
#ifdef _OPENMP
#pragma omp critical
#endif
      rc_all = rc;
    }
    for (int i = 0; i < N; ++i) S[(size_t)i * NZ + j] = dyo[i];
  }
  (void)nthreads;
  return rc_all;
}

// Fixed-step integration of a built-in test problem; errout gets the embedded
// error estimate of the last step.
int oracle_ros_test(int method, int problem, double h, int nsteps, const double* y0, double* yout, double* errout) {
  const Table t = table_of(method);
  const int N = problem == 0 ? 2 : 1;
  const double lam = problem == 0 ? 0.0 : y0[1];
  std::vector<double> y(y0, y0 + N), f0(N), J((size_t)N * N), yn(N), err(N);
  auto frhs = [&](const double* yy, double* ff) { test_rhs(problem, yy, ff, lam); };
  for (int s = 0; s < nsteps; ++s) {
    test_rhs(problem, y.data(), f0.data(), lam);
    test_jac(problem, y.data(), J.data(), lam);
    if (ros_step(t, N, frhs, y.data(), f0.data(), J.data(), h, yn.data(), err.data())) return 1;
    y = yn;
  }
  for (int i = 0; i < N; ++i) {
    yout[i] = y[i];
    errout[i] = err[i];
  }
  return 0;
}

// Fixed-column extrapolated linearly implicit Euler on the built-in test
// problems (order checks): nsteps steps of size H, result T_{k,k} each step.
int oracle_sx_test(int problem, double H, int nsteps, int kcols, const double* y0, double* yout) {
  const int N = problem == 0 ? 2 : 1;
  const double lam = problem == 0 ? 0.0 : y0[1];
  std::vector<double> y(y0, y0 + N), f0(N), J((size_t)N * N);
  std::vector<std::vector<std::vector<double>>> T(SX_KMAX, std::vector<std::vector<double>>(SX_KMAX,
                                                  std::vector<double>(N)));
  auto frhs = [&](const double* yy, double* ff) { test_rhs(problem, yy, ff, lam); };
  if (kcols < 1 || kcols > SX_KMAX) return 2;
  for (int s = 0; s < nsteps; ++s) {
    test_rhs(problem, y.data(), f0.data(), lam);
    test_jac(problem, y.data(), J.data(), lam);
    if (seulex_table(N, frhs, y.data(), f0.data(), J.data(), H, kcols, T, true)) return 1;
    y = T[kcols - 1][kcols - 1];
  }
  for (int i = 0; i < N; ++i) yout[i] = y[i];
  return 0;
}

int oracle_num_threads() {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

}  // extern "C"
