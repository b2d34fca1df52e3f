// Discrete adjoint of the Rosenbrock integration (device side).
//
// The forward pass records every accepted step size and a checkpoint of the
// state every `ckpt` accepted steps.  The reverse sweep walks the segments
// last to first: it replays a segment forward with the recorded step sizes,
// then walks its steps backwards.  For one step y_{n+1} = y_n + sum_i m_i K_i
// with (I/(gamma h) - J(y_n)) K_i = f(Y_src(i)) + sum_{j<i} (c_ij/h) K_j and
// Y_i = y_n + sum_{j<i} a_ij K_j, and lambda = dPsi/dy_{n+1}:
//   Kbar_i = m_i lambda;  for i = s..1:
//     u_i = M^{-T} Kbar_i
//     Kbar_j += (c_ij/h) u_i                       (j < i)
//     Ubar_src(i) += u_i
//     if src(i) == i:  g = J(Y_i)^T Ubar_i,  Kbar_j += a_ij g (j < i),  lambda_n += g
//     lambda_n += (J'[K_i])^T u_i                   (J(y_n) inside M)
//   lambda_n += lambda
// and the same terms with df/dp for the Arrhenius parameters.  J(Y)^T u is a
// hand-written reverse pass through f; the second-order terms are that
// reverse pass evaluated on dual numbers seeded with y_n + eps K_i.
#pragma once
#include "chem_cell.hpp"

namespace chem {

// ---------------------------------------------------------------- dual numbers
struct Dd {
  double v, d;
};
__device__ __forceinline__ Dd mk(double v, double d = 0.0) { return Dd{v, d}; }
__device__ __forceinline__ Dd operator+(Dd a, Dd b) { return {a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ Dd operator-(Dd a, Dd b) { return {a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ Dd operator*(Dd a, Dd b) { return {a.v * b.v, fma(a.d, b.v, a.v * b.d)}; }
__device__ __forceinline__ Dd operator/(Dd a, Dd b) {
  const double q = a.v / b.v;
  return {q, (a.d - q * b.d) / b.v};
}
__device__ __forceinline__ Dd operator-(Dd a) { return {-a.v, -a.d}; }
__device__ __forceinline__ Dd operator+(Dd a, double b) { return {a.v + b, a.d}; }
__device__ __forceinline__ Dd operator+(double a, Dd b) { return {a + b.v, b.d}; }
__device__ __forceinline__ Dd operator-(Dd a, double b) { return {a.v - b, a.d}; }
__device__ __forceinline__ Dd operator-(double a, Dd b) { return {a - b.v, -b.d}; }
__device__ __forceinline__ Dd operator*(Dd a, double b) { return {a.v * b, a.d * b}; }
__device__ __forceinline__ Dd operator*(double a, Dd b) { return {a * b.v, a * b.d}; }
__device__ __forceinline__ Dd operator/(Dd a, double b) { return {a.v / b, a.d / b}; }
__device__ __forceinline__ Dd operator/(double a, Dd b) {
  const double q = a / b.v;
  return {q, -q * b.d / b.v};
}
__device__ __forceinline__ Dd& operator+=(Dd& a, Dd b) { return a = a + b; }
__device__ __forceinline__ Dd& operator-=(Dd& a, Dd b) { return a = a - b; }

__device__ __forceinline__ double sexp(double x) { return exp(x); }
__device__ __forceinline__ Dd sexp(Dd x) {
  const double e = exp(x.v);
  return {e, e * x.d};
}
__device__ __forceinline__ double slog(double x) { return log(x); }
__device__ __forceinline__ Dd slog(Dd x) { return {log(x.v), x.d / x.v}; }
__device__ __forceinline__ double slog10(double x) { return log10(x); }
__device__ __forceinline__ Dd slog10(Dd x) { return {log10(x.v), x.d / (x.v * 2.302585092994045684)}; }
__device__ __forceinline__ double sexp10(double x) { return exp10(x); }
__device__ __forceinline__ Dd sexp10(Dd x) {
  const double e = exp10(x.v);
  return {e, e * 2.302585092994045684 * x.d};
}
__device__ __forceinline__ double rl(double x, int l) { return readlane(x, l); }
__device__ __forceinline__ Dd rl(Dd x, int l) { return {readlane(x.v, l), readlane(x.d, l)}; }
__device__ __forceinline__ double wsum(double x) { return wave_sum(x); }
__device__ __forceinline__ Dd wsum(Dd x) { return {wave_sum(x.v), wave_sum(x.d)}; }
// the part of a value that a pass contributes: the value itself in the
// first-order pass, the derivative part in the dual (second-order) pass
__device__ __forceinline__ double sval(double x) { return x; }
__device__ __forceinline__ double sval(Dd x) { return x.v; }
__device__ __forceinline__ double part(double x) { return x; }
__device__ __forceinline__ double part(Dd x) { return x.d; }
template <class S>
__device__ __forceinline__ S zero();
template <>
__device__ __forceinline__ double zero<double>() { return 0.0; }
template <>
__device__ __forceinline__ Dd zero<Dd>() { return Dd{0.0, 0.0}; }
template <class S>
__device__ __forceinline__ S one();
template <>
__device__ __forceinline__ double one<double>() { return 1.0; }
template <>
__device__ __forceinline__ Dd one<Dd>() { return Dd{1.0, 0.0}; }

// Adjoint workspace in LDS (arrays of S; the double pass uses the same bytes).
// The adjoint of sum nu g/RT of reaction r is aP[r] R_r, recomputed where it
// is needed, so it takes no array.
template <class S>
struct AdjView {
  S* C;   // [66] concentrations (padding species 1)
  S* g;   // [66] g/RT
  S* hR;  // [66] h/RT
  S* ob;  // [66] adjoint of omega (padding 0)
  S* aR;  // [R] q in the forward part, then adjoint of R_f
  S* aP;  // [R] adjoint of R_r
  S* Mb;  // [R - R0] adjoint of [M] of the third-body and Troe reactions
};

// Doubles of the workspace: room for the dual-number (two-double) pass.
__host__ __device__ inline int adj_ws_doubles(int R, int R0) { return 2 * (4 * 66 + 2 * R + (R - R0)); }

template <class S>
__device__ inline AdjView<S> make_adj(double* base, int R) {
  AdjView<S> v;
  S* b = (S*)base;
  v.C = b;
  v.g = b + 66;
  v.hR = b + 132;
  v.ob = b + 198;
  v.aR = b + 264;
  v.aP = v.aR + R;
  v.Mb = v.aP + R;
  return v;
}

// Species -> (reaction, slot) and species -> (reaction, efficiency entry)
// incidence lists used to gather the adjoints of the concentrations.
struct AdjMech {
  const int32_t* sptr;  // [K+1]
  const uint32_t* sent; // (r << 3) | slot, slot 0..2 reactants, 3..5 products
  const int32_t* tptr;  // [K+1]
  const uint32_t* tent; // (r << 12) | efficiency entry
};

template <class S>
struct RateLoc {
  S kf, dlnkf, iKc, Rf, Rr, net, keff, dkM, dlnk, gg;
};

// Rate of progress of reaction r with the local derivatives the reverse pass needs.
template <class S>
__device__ inline RateLoc<S> rate_loc(const MechView& m, const AdjView<S>& v, int r, S T, S lnT, S iT, S Ctot,
                                      S lnPRT) {
  const Slots s = unpack(m.sp[r]);
  RateLoc<S> o;
  const S lnkf = m.lnA[r] + m.b[r] * lnT - m.th[r] * iT;
  o.kf = sexp(lnkf);
  o.dlnkf = m.b[r] * iT + m.th[r] * iT * iT;
  o.Rf = v.C[s.r0] * v.C[s.r1] * v.C[s.r2];
  o.Rr = v.C[s.p0] * v.C[s.p1] * v.C[s.p2];
  const S sng = v.g[s.p0] + v.g[s.p1] + v.g[s.p2] - v.g[s.r0] - v.g[s.r1] - v.g[s.r2];
  o.iKc = sexp(sng - (double)s.dnu * lnPRT);
  o.net = o.Rf - o.iKc * o.Rr;
  o.keff = o.kf;
  o.dkM = zero<S>();
  o.dlnk = o.dlnkf;
  o.gg = zero<S>();
  if (r >= m.d.R0) {
    S M = Ctot;
    const int e1 = m.tbp[r - m.d.R0 + 1];
    for (int e = m.tbp[r - m.d.R0]; e < e1; ++e) M += m.tbd[e] * v.C[m.tbs[e]];
    if (r < m.d.R1) {
      o.keff = o.kf * M;
      o.dkM = o.kf;
    } else {
      const double* t = m.troe + TROE_STRIDE * (r - m.d.R1);
      const double alpha = t[0], iT3 = t[1], iT1 = t[2], T2 = t[3];
      const S k0 = sexp(t[4] + t[5] * lnT - t[6] * iT);
      const S Pr = k0 * M / o.kf;
      const S e3 = sexp(-T * iT3), e1x = sexp(-T * iT1), e2 = sexp(-T2 * iT);
      const S Fc = (1.0 - alpha) * e3 + alpha * e1x + e2;
      const S xF = slog10(Fc);
      const S L = slog10(Pr);
      const S c = -0.4 - 0.67 * xF;
      const S n = 0.75 - 1.27 * xF;
      const S d = n - 0.14 * (L + c);
      const S f1 = (L + c) / d;
      const S den = 1.0 + f1 * f1;
      const S F = sexp10(xF / den);
      const S ipr = 1.0 / (1.0 + Pr);
      o.keff = k0 * M * ipr * F;
      const S id2 = 1.0 / (d * d);
      const S dlgF_dL = -xF * 2.0 * f1 / (den * den) * n * id2;
      const S dlgF_dx = 1.0 / den - xF * 2.0 * f1 / (den * den) * (-0.67 * d + 1.1762 * (L + c)) * id2;
      o.gg = ipr + dlgF_dL;
      o.dkM = k0 * F * ipr * o.gg;
      const S dFc = -(1.0 - alpha) * iT3 * e3 - alpha * iT1 * e1x + T2 * iT * iT * e2;
      const S dlnk0 = t[5] * iT + t[6] * iT * iT;
      o.dlnk = o.dlnkf + o.gg * (dlnk0 - o.dlnkf) + dlgF_dx * dFc / Fc;
    }
  }
  return o;
}

// u^T f(y) differentiated in reverse mode: returns (J(y)^T u)_lane and adds
// part((df/dp)^T u) to pg[3r + {0,1,2}] = d/dlnA, d/db, d/dtheta.  u is the
// lane-local weight on f_lane; y may be dual (then the returned derivative part
// is (J'[dy])^T u and pg receives the derivative parts).
template <class S>
__device__ S vjp_f(const MechView& m, const AdjMech& am, const AdjView<S>& v, double* pg, S y, double u, double p,
                   int lane) {
  const int K = m.d.K, R = m.d.R;
  const bool isSp = lane >= 1 && lane <= K;
  const int k = isSp ? lane - 1 : 0;
  if (lane == 0) {  // padding species
    v.C[K] = one<S>();
    v.g[K] = zero<S>();
    v.hR[K] = zero<S>();
    v.ob[K] = zero<S>();
  }
  // ---- forward part
  const S T = rl(y, 0);
  const S lnT = slog(T);
  const S iT = 1.0 / T;
  const double* row = m.nasa + 16 * k;
  const double* a = (sval(T) > row[0]) ? row + 8 : row + 1;
  const S cpR = a[0] + T * (a[1] + T * (a[2] + T * (a[3] + T * a[4])));
  const S hRT = a[0] + T * (a[1] * 0.5 + T * (a[2] * (1.0 / 3.0) + T * (a[3] * 0.25 + T * a[4] * 0.2))) + a[5] * iT;
  const S sR = a[0] * lnT + T * (a[1] + T * (a[2] * 0.5 + T * (a[3] * (1.0 / 3.0) + T * a[4] * 0.25))) + a[6];
  const S dcpR = a[1] + T * (2.0 * a[2] + T * (3.0 * a[3] + T * 4.0 * a[4]));
  const double Wk = m.W[k], iWk = m.iW[k];
  const S Yk = isSp ? y : zero<S>();
  const S yw = Yk * iWk;
  const S sy = wsum(yw);
  const S rho = p / (RU * T * sy);
  const S Ctot = p * iT / RU;
  const S lnPRT = slog(PATM * iT / RU);
  const S cpm = isSp ? RU * cpR * iWk : zero<S>();
  const S cp = wsum(Yk * cpm);
  if (isSp) {
    v.C[k] = rho * yw;
    v.g[k] = hRT - sR;
    v.hR[k] = hRT;
  }
  wsync();
  for (int r = lane; r < R; r += WAVE) {
    const RateLoc<S> o = rate_loc<S>(m, v, r, T, lnT, iT, Ctot, lnPRT);
    v.aR[r] = o.keff * o.net;
  }
  wsync();
  S om = zero<S>();
  if (isSp) {
    for (int e = m.cptr[k]; e < m.cptr[k + 1]; ++e) {
      const uint32_t cv = m.cent[e];
      om += (double)(int8_t)(cv & 0xFF) * v.aR[cv >> 8];
    }
  }
  const S Q = wsum(isSp ? hRT * om : zero<S>());
  const S fT = -RU * T * Q / (rho * cp);
  const S fk = isSp ? Wk * om / rho : zero<S>();
  // ---- reverse part
  const double uT = readlane(u, 0);
  const S Qb = -uT * RU * T / (rho * cp);
  const S rhob1 = wsum(isSp ? -u * fk / rho : zero<S>()) - uT * fT / rho;
  const S cpb = -uT * fT / cp;
  S Tb = uT * fT * iT;
  S hRTb = isSp ? Qb * om : zero<S>();
  if (isSp) v.ob[k] = u * Wk / rho + Qb * hRT;
  wsync();
  S Tbr = zero<S>();
  for (int r = lane; r < R; r += WAVE) {
    const RateLoc<S> o = rate_loc<S>(m, v, r, T, lnT, iT, Ctot, lnPRT);
    const Slots s = unpack(m.sp[r]);
    const S qb = v.ob[s.p0] + v.ob[s.p1] + v.ob[s.p2] - v.ob[s.r0] - v.ob[s.r1] - v.ob[s.r2];
    const S keffb = qb * o.net;
    const S netb = qb * o.keff;
    const S sngb = -netb * o.Rr * o.iKc;
    Tbr += (double)s.dnu * sngb * iT;
    S lnkb, Mb = zero<S>();
    if (r < m.d.R1) {
      lnkb = keffb * o.keff;
      Tbr += lnkb * o.dlnkf;
      if (r >= m.d.R0) Mb = keffb * o.kf;
    } else {
      Mb = keffb * o.dkM;
      Tbr += keffb * o.keff * o.dlnk;
      lnkb = keffb * o.keff * (1.0 - o.gg);
    }
    if (r >= m.d.R0) Tbr -= Mb * Ctot * iT;
    v.aR[r] = netb;
    v.aP[r] = -netb * o.iKc;
    if (r >= m.d.R0) v.Mb[r - m.d.R0] = Mb;
    pg[3 * r + 0] += part(lnkb);
    pg[3 * r + 1] += part(lnkb * lnT);
    pg[3 * r + 2] -= part(lnkb * iT);
  }
  wsync();
  S Cb = zero<S>(), gb = zero<S>();
  if (isSp) {
    for (int e = am.sptr[k]; e < am.sptr[k + 1]; ++e) {
      const uint32_t ev = am.sent[e];
      const int r = (int)(ev >> 3), slot = (int)(ev & 7);
      const Slots s = unpack(m.sp[r]);
      const S aP = v.aP[r];
      const S sn = aP * (v.C[s.p0] * v.C[s.p1] * v.C[s.p2]);  // adjoint of sum nu g/RT
      if (slot < 3) {
        const int o1 = slot == 0 ? s.r1 : s.r0, o2 = slot == 2 ? s.r1 : s.r2;
        Cb += v.aR[r] * (v.C[o1] * v.C[o2]);
        gb -= sn;
      } else {
        const int o1 = slot == 3 ? s.p1 : s.p0, o2 = slot == 5 ? s.p1 : s.p2;
        Cb += aP * (v.C[o1] * v.C[o2]);
        gb += sn;
      }
    }
    for (int e = am.tptr[k]; e < am.tptr[k + 1]; ++e) {
      const uint32_t ev = am.tent[e];
      Cb += v.Mb[(ev >> 12) - m.d.R0] * m.tbd[ev & 0xFFF];
    }
  }
  hRTb += gb;
  const S sRb = -gb;
  const S cpRb = isSp ? cpb * Yk * RU * iWk : zero<S>();
  const S Tth = isSp ? hRTb * (cpR - hRT) * iT + sRb * cpR * iT + cpRb * dcpR : zero<S>();
  S Yb = isSp ? cpb * cpm : zero<S>();
  const S rhob = rhob1 + wsum(isSp ? Cb * yw : zero<S>());
  S ywb = isSp ? Cb * rho : zero<S>();
  Tb += wsum(Tbr) + wsum(Tth) - rhob * rho * iT;
  const S syb = -rhob * rho / sy;
  ywb += syb;
  Yb += ywb * iWk;
  wsync();
  return lane == 0 ? Tb : (isSp ? Yb : zero<S>());
}

// Solve M^T x = b with the pivot-ordered factors stored row-wise in LDS F
// (row k of P M = L U on lane k): U^T z = b, L^T v = z, x = P^T v.
template <int NP>
__device__ inline double lu_solve_T(const double* F, int N, int S, int lane, int mystep, double myrdiag, double b) {
  // rows >= N of F are not factors: those steps are skipped (uniform branch);
  // padding lanes read column 0 and are masked.  The masks act on the
  // multipliers, off the chain through b (adding -0 leaves b as it is).
  const int col = lane < N ? lane : 0;
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    if (k < N) {
      const double zk = readlane(b * myrdiag, k);
      b = fma((lane > k && lane < N) ? -F[k * S + col] : -0.0, zk, b);
    }
  }
  b *= myrdiag;
#pragma unroll
  for (int k = NP - 1; k >= 0; --k) {
    if (k < N) {
      const double vk = readlane(b, k);
      b = fma(lane < k ? -F[k * S + col] : -0.0, vk, b);
    }
  }
  return __shfl(b, mystep);
}

__device__ __forceinline__ double pick4(double a0, double a1, double a2, double a3, int i) {
  double r = a0;
  r = i == 1 ? a1 : r;
  r = i == 2 ? a2 : r;
  r = i == 3 ? a3 : r;
  return r;
}

}  // namespace chem
