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

// ------------------------------------------------- tangents and their adjoints
// The second-order terms sum_i (J'(y_n)[K_i])^T u_i are taken two stages at a
// time by reverse mode over a two-direction forward mode: forward values F2
// carry the value and its derivatives along K_a and K_b; adjoint values A3
// carry the adjoint of the value (p, which collects the second-order terms),
// the adjoints of the two derivatives (t0, t1, seeded with u_a and u_b: these
// are first-order adjoints for those seeds) and one more first-order adjoint
// (w, seeded with another weight on f).  For z = x * y with x, y forward
// values: xbar.t_j += zbar.t_j y.v, xbar.w += zbar.w y.v and
// xbar.p += zbar.p y.v + sum_j zbar.t_j y.d_j.  At the end p holds
// sum_j (J'[K_j])^T u_j and w holds J^T w_seed; the t parts are not needed.
// Both types view LDS bytes that the other type also uses (the forward rates
// and the reverse adjoints share an array), so they may alias anything.
struct __attribute__((may_alias)) F2 {
  double v, d0, d1;
};
__device__ __forceinline__ F2 operator+(F2 a, F2 b) { return {a.v + b.v, a.d0 + b.d0, a.d1 + b.d1}; }
__device__ __forceinline__ F2 operator-(F2 a, F2 b) { return {a.v - b.v, a.d0 - b.d0, a.d1 - b.d1}; }
__device__ __forceinline__ F2 operator*(F2 a, F2 b) {
  return {a.v * b.v, fma(a.d0, b.v, a.v * b.d0), fma(a.d1, b.v, a.v * b.d1)};
}
__device__ __forceinline__ F2 operator/(F2 a, F2 b) {
  const double q = a.v / b.v, ib = 1.0 / b.v;
  return {q, (a.d0 - q * b.d0) * ib, (a.d1 - q * b.d1) * ib};
}
__device__ __forceinline__ F2 operator-(F2 a) { return {-a.v, -a.d0, -a.d1}; }
__device__ __forceinline__ F2 operator+(F2 a, double b) { return {a.v + b, a.d0, a.d1}; }
__device__ __forceinline__ F2 operator+(double a, F2 b) { return {a + b.v, b.d0, b.d1}; }
__device__ __forceinline__ F2 operator-(F2 a, double b) { return {a.v - b, a.d0, a.d1}; }
__device__ __forceinline__ F2 operator-(double a, F2 b) { return {a - b.v, -b.d0, -b.d1}; }
__device__ __forceinline__ F2 operator*(F2 a, double b) { return {a.v * b, a.d0 * b, a.d1 * b}; }
__device__ __forceinline__ F2 operator*(double a, F2 b) { return {a * b.v, a * b.d0, a * b.d1}; }
__device__ __forceinline__ F2 operator/(F2 a, double b) { return {a.v / b, a.d0 / b, a.d1 / b}; }
__device__ __forceinline__ F2 operator/(double a, F2 b) {
  const double q = a / b.v, s = -q / b.v;
  return {q, s * b.d0, s * b.d1};
}
__device__ __forceinline__ F2& operator+=(F2& a, F2 b) { return a = a + b; }
__device__ __forceinline__ F2& operator-=(F2& a, F2 b) { return a = a - b; }

struct __attribute__((may_alias)) A3 {
  double p, t0, t1, w;
};
__device__ __forceinline__ A3 operator+(A3 a, A3 b) { return {a.p + b.p, a.t0 + b.t0, a.t1 + b.t1, a.w + b.w}; }
__device__ __forceinline__ A3 operator-(A3 a, A3 b) { return {a.p - b.p, a.t0 - b.t0, a.t1 - b.t1, a.w - b.w}; }
__device__ __forceinline__ A3 operator-(A3 a) { return {-a.p, -a.t0, -a.t1, -a.w}; }
__device__ __forceinline__ A3 operator*(A3 a, double b) { return {a.p * b, a.t0 * b, a.t1 * b, a.w * b}; }
__device__ __forceinline__ A3 operator*(double a, A3 b) { return b * a; }
__device__ __forceinline__ A3 operator/(A3 a, double b) { return {a.p / b, a.t0 / b, a.t1 / b, a.w / b}; }
__device__ __forceinline__ A3 operator*(A3 a, F2 x) {
  return {fma(a.t1, x.d1, fma(a.t0, x.d0, a.p * x.v)), a.t0 * x.v, a.t1 * x.v, a.w * x.v};
}
__device__ __forceinline__ A3 operator*(F2 x, A3 a) { return a * x; }
__device__ __forceinline__ A3 operator/(A3 a, F2 x) { return a * (1.0 / x); }
__device__ __forceinline__ A3& operator+=(A3& a, A3 b) { return a = a + b; }
__device__ __forceinline__ A3& operator-=(A3& a, A3 b) { return a = a - b; }

// LDS accumulation, component by component (within one instruction the
// hardware applies conflicting lanes in a fixed order)
__device__ __forceinline__ void atomic_add(double* p, double v) { atomicAdd(p, v); }
__device__ __forceinline__ void atomic_add(F2* p, F2 v) {
  atomicAdd(&p->v, v.v);
  atomicAdd(&p->d0, v.d0);
  atomicAdd(&p->d1, v.d1);
}
__device__ __forceinline__ void atomic_add(A3* p, A3 v) {
  atomicAdd(&p->p, v.p);
  atomicAdd(&p->t0, v.t0);
  atomicAdd(&p->t1, v.t1);
  atomicAdd(&p->w, v.w);
}

__device__ __forceinline__ double sexp(double x) { return exp(x); }
__device__ __forceinline__ F2 sexp(F2 x) {
  const double e = exp(x.v);
  return {e, e * x.d0, e * x.d1};
}
__device__ __forceinline__ double slog(double x) { return log(x); }
__device__ __forceinline__ F2 slog(F2 x) {
  const double i = 1.0 / x.v;
  return {log(x.v), x.d0 * i, x.d1 * i};
}
__device__ __forceinline__ double slog10(double x) { return log10(x); }
__device__ __forceinline__ F2 slog10(F2 x) {
  const double i = 1.0 / (x.v * 2.302585092994045684);
  return {log10(x.v), x.d0 * i, x.d1 * i};
}
__device__ __forceinline__ double sexp10(double x) { return exp10(x); }
__device__ __forceinline__ F2 sexp10(F2 x) {
  const double e = exp10(x.v), s = e * 2.302585092994045684;
  return {e, s * x.d0, s * x.d1};
}
__device__ __forceinline__ double rl(double x, int l) { return readlane(x, l); }
__device__ __forceinline__ F2 rl(F2 x, int l) { return {readlane(x.v, l), readlane(x.d0, l), readlane(x.d1, l)}; }
__device__ __forceinline__ A3 rl(A3 x, int l) {
  return {readlane(x.p, l), readlane(x.t0, l), readlane(x.t1, l), readlane(x.w, l)};
}
__device__ __forceinline__ double wsum(double x) { return wave_sum(x); }
__device__ __forceinline__ F2 wsum(F2 x) { return {wave_sum(x.v), wave_sum(x.d0), wave_sum(x.d1)}; }
__device__ __forceinline__ A3 wsum(A3 x) { return {wave_sum(x.p), wave_sum(x.t0), wave_sum(x.t1), wave_sum(x.w)}; }
__device__ __forceinline__ double sval(double x) { return x; }
__device__ __forceinline__ double sval(F2 x) { return x.v; }
// what a pass contributes to lambda_n and to the parameter gradient: the
// adjoint itself in the first-order pass; the second-order terms plus the
// extra first-order adjoint in the combined pass
__device__ __forceinline__ double part(double x) { return x; }
__device__ __forceinline__ double part(A3 x) { return x.p + x.w; }
template <class S>
__device__ __forceinline__ S zero();
template <>
__device__ __forceinline__ double zero<double>() { return 0.0; }
template <>
__device__ __forceinline__ F2 zero<F2>() { return F2{0.0, 0.0, 0.0}; }
template <>
__device__ __forceinline__ A3 zero<A3>() { return A3{0.0, 0.0, 0.0, 0.0}; }
template <class S>
__device__ __forceinline__ S one();
template <>
__device__ __forceinline__ double one<double>() { return 1.0; }
template <>
__device__ __forceinline__ F2 one<F2>() { return F2{1.0, 0.0, 0.0}; }

// Adjoint workspace in LDS: forward values F, adjoint values A.  The rates of
// progress of the forward part (q) and the adjoints of R_f (aR) share bytes.
// The adjoint of sum nu g/RT of reaction r is aP[r] R_r, recomputed where it
// is needed, so it takes no array.
template <class F, class A>
struct AdjView {
  F* C;   // [66] concentrations (padding species 1)
  F* g;   // [66] g/RT
  F* om;  // [66] production rates omega (accumulated)
  A* ob;  // [66] adjoint of omega (padding 0); then chunk partial sums of the adjoint of C
  A* xb;  // [64] chunk partial sums of the adjoint of g/RT
  F* q;   // [R] rates of progress (forward part)
  A* aR;  // [R] adjoint of R_f (reverse part; same bytes as q)
  A* aP;  // [R] adjoint of R_r
  A* Mb;  // [R - R0 + 1] adjoint of [M] of the third-body and Troe reactions
};

template <class F, class A>
__host__ __device__ inline int adj_doubles(int R, int R0) {
  constexpr int f = (int)(sizeof(F) / sizeof(double)), a = (int)(sizeof(A) / sizeof(double));
  constexpr int qa = f > a ? f : a;
  return 198 * f + 130 * a + R * qa + R * a + (R - R0 + 1) * a;
}

template <class F, class A>
__device__ inline AdjView<F, A> make_adj(double* base, int R) {
  constexpr int f = (int)(sizeof(F) / sizeof(double)), a = (int)(sizeof(A) / sizeof(double));
  constexpr int qa = f > a ? f : a;
  AdjView<F, A> v;
  v.C = (F*)base;
  v.g = v.C + 66;
  v.om = v.g + 66;
  v.ob = (A*)(base + 198 * f);
  v.xb = v.ob + 66;
  double* qb = base + 198 * f + 130 * a;
  v.q = (F*)qb;
  v.aR = (A*)qb;
  v.aP = (A*)(qb + (size_t)R * qa);
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
  // the sent lists cut into chunks: chunk[i][j] is entry i of lane j's chunk
  // (~0 past its end); cspan[k] = first chunk | count << 8 of species k
  const uint32_t* chunk; // [cw][64]
  const int32_t* cspan;  // [K]
  int cw;
};

template <class S>
struct RateLoc {
  S kf, dlnkf, iKc, Rf, Rr, net, keff, dkM, dlnk, gg;
};

// Rate of progress of reaction r with the local derivatives the reverse pass needs.
template <class S, class A>
__device__ inline RateLoc<S> rate_loc(const MechView& m, const AdjView<S, A>& v, int r, S T, S lnT, S iT, S Ctot,
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
// part((df/dp)^T u) to pg[3r + {0,1,2}] = d/dlnA, d/db, d/dtheta (the cell's
// gradient accumulators, lane-owned entries).  u is the lane-local weight on
// f_lane.  With F = F2 and A = A3 (y carries the directions K_a, K_b; u the
// seeds u_a, u_b and w) the returned p part is sum_j (J'[K_j])^T u_j, the w
// part J^T w, and pg receives both parameter parts.
template <class F, class A>
__device__ A vjp_f(const MechView& m, const AdjMech& am, const AdjView<F, A>& v, double* pg, F y, A u, double p,
                   int lane) {
  const int K = m.d.K, R = m.d.R;
  const bool isSp = lane >= 1 && lane <= K;
  const int k = isSp ? lane - 1 : 0;
  if (lane == 0) {  // padding species
    v.C[K] = one<F>();
    v.g[K] = zero<F>();
  }
  for (int i = lane; i < 66; i += WAVE) v.om[i] = zero<F>();
  // ---- forward part
  const F T = rl(y, 0);
  const F lnT = slog(T);
  const F iT = 1.0 / T;
  const double* row = m.nasa + 16 * k;
  const double* a = (sval(T) > row[0]) ? row + 8 : row + 1;
  const F cpR = a[0] + T * (a[1] + T * (a[2] + T * (a[3] + T * a[4])));
  const F hRT = a[0] + T * (a[1] * 0.5 + T * (a[2] * (1.0 / 3.0) + T * (a[3] * 0.25 + T * a[4] * 0.2))) + a[5] * iT;
  const F sR = a[0] * lnT + T * (a[1] + T * (a[2] * 0.5 + T * (a[3] * (1.0 / 3.0) + T * a[4] * 0.25))) + a[6];
  const F dcpR = a[1] + T * (2.0 * a[2] + T * (3.0 * a[3] + T * 4.0 * a[4]));
  const double Wk = m.W[k], iWk = m.iW[k];
  const F Yk = isSp ? y : zero<F>();
  const F yw = Yk * iWk;
  const F sy = wsum(yw);
  const F rho = p / (RU * T * sy);
  const F Ctot = p * iT / RU;
  const F lnPRT = slog(PATM * iT / RU);
  const F cpm = isSp ? RU * cpR * iWk : zero<F>();
  const F cp = wsum(Yk * cpm);
  if (isSp) {
    v.C[k] = rho * yw;
    v.g[k] = hRT - sR;
  }
  wsync();
  for (int r = lane; r < R; r += WAVE) {
    const RateLoc<F> o = rate_loc<F, A>(m, v, r, T, lnT, iT, Ctot, lnPRT);
    v.q[r] = o.keff * o.net;
  }
  wsync();
  // omega_k = sum_r nu_kr q_r on the balanced species schedule
  {
    const uint32_t* js = m.jsched + lane;
    uint32_t ent = js[0];
    for (int it = 0; it < m.jit; ++it) {
      const uint32_t cur = ent;
      if (it + 1 < m.jit) ent = js[(it + 1) * WAVE];
      if (cur != ~0u) atomic_add(&v.om[(cur >> 8) & 0xFF], (double)(int8_t)(cur & 0xFF) * v.q[cur >> 16]);
    }
  }
  lds_wait();
  wsync();
  const F om = isSp ? v.om[k] : zero<F>();
  const F Q = wsum(isSp ? hRT * om : zero<F>());
  const F fT = -RU * T * Q / (rho * cp);
  const F fk = isSp ? Wk * om / rho : zero<F>();
  // ---- reverse part
  const A uT = rl(u, 0);
  const A Qb = -uT * RU * T / (rho * cp);
  const A rhob1 = wsum(isSp ? -u * fk / rho : zero<A>()) - uT * fT / rho;
  const A cpb = -uT * fT / cp;
  A Tb = uT * fT * iT;
  A hRTb = isSp ? Qb * om : zero<A>();
  if (isSp) v.ob[k] = u * Wk / rho + Qb * hRT;
  if (lane == 0) v.ob[K] = zero<A>();
  wsync();
  A Tbr = zero<A>();
  // the gradient accumulators of the lane's next reaction are loaded one
  // iteration ahead (they live in global memory)
  double n0 = 0.0, n1 = 0.0, n2 = 0.0;
  if (lane < R) {
    n0 = pg[3 * lane];
    n1 = pg[3 * lane + 1];
    n2 = pg[3 * lane + 2];
  }
  for (int r = lane; r < R; r += WAVE) {
    double* pgr = pg + 3 * r;
    const double g0 = n0, g1 = n1, g2 = n2;
    if (r + WAVE < R) {
      n0 = pgr[3 * WAVE];
      n1 = pgr[3 * WAVE + 1];
      n2 = pgr[3 * WAVE + 2];
    }
    const RateLoc<F> o = rate_loc<F, A>(m, v, r, T, lnT, iT, Ctot, lnPRT);
    const Slots s = unpack(m.sp[r]);
    const A qb = v.ob[s.p0] + v.ob[s.p1] + v.ob[s.p2] - v.ob[s.r0] - v.ob[s.r1] - v.ob[s.r2];
    const A keffb = qb * o.net;
    const A netb = qb * o.keff;
    const A sngb = -netb * o.Rr * o.iKc;
    Tbr += (double)s.dnu * sngb * iT;
    A lnkb, Mb = zero<A>();
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
    pgr[0] = g0 + part(lnkb);
    pgr[1] = g1 + part(lnkb * lnT);
    pgr[2] = g2 - part(lnkb * iT);
  }
  wsync();
  // adjoints of the concentrations and of g/RT.  The species' incidence
  // lists are cut into at most 64 chunks of at most cw entries (a species'
  // chunks consecutive); lane j sums chunk j in list order, four entries per
  // pass without branches so that their LDS reads are in flight together;
  // then every species lane adds its chunks' partial sums in chunk order.
  A pc = zero<A>(), pgv = zero<A>();
  {
    const uint32_t* cg = am.chunk + lane;
    uint32_t nx[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) nx[u] = u < am.cw ? cg[u * WAVE] : ~0u;
    for (int it = 0; it < am.cw; it += 4) {
      uint32_t cu[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        cu[u] = nx[u];
        nx[u] = it + 4 + u < am.cw ? cg[(it + 4 + u) * WAVE] : ~0u;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const bool live = cu[u] != ~0u;
        const uint32_t ev = live ? cu[u] : 0u;
        const int r = (int)(ev >> 3), slot = (int)(ev & 7);
        const bool reac = slot < 3;
        const Slots s = unpack(m.sp[r]);
        const A aP = v.aP[r];
        const A sn = aP * (v.C[s.p0] * v.C[s.p1] * v.C[s.p2]);  // adjoint of sum nu g/RT
        const int o1 = reac ? (slot == 0 ? s.r1 : s.r0) : (slot == 3 ? s.p1 : s.p0);
        const int o2 = reac ? (slot == 2 ? s.r1 : s.r2) : (slot == 5 ? s.p1 : s.p2);
        const A c = (reac ? v.aR[r] : aP) * (v.C[o1] * v.C[o2]);
        pc += live ? c : zero<A>();
        pgv += live ? (reac ? -sn : sn) : zero<A>();
      }
    }
  }
  v.ob[lane] = pc;  // the adjoints of omega are no longer needed
  v.xb[lane] = pgv;
  wsync();
  A Cb = zero<A>(), gb = zero<A>();
  if (isSp) {
    const int c0 = am.cspan[k] & 0xFF, cn = am.cspan[k] >> 8;
    for (int j = c0; j < c0 + cn; ++j) {
      Cb += v.ob[j];
      gb += v.xb[j];
    }
    for (int e = am.tptr[k]; e < am.tptr[k + 1]; ++e) {
      const uint32_t ev = am.tent[e];
      Cb += v.Mb[(ev >> 12) - m.d.R0] * m.tbd[ev & 0xFFF];
    }
  }
  hRTb += gb;
  const A sRb = -gb;
  const A cpRb = isSp ? cpb * Yk * RU * iWk : zero<A>();
  const A Tth = isSp ? hRTb * (cpR - hRT) * iT + sRb * cpR * iT + cpRb * dcpR : zero<A>();
  A Yb = isSp ? cpb * cpm : zero<A>();
  const A rhob = rhob1 + wsum(isSp ? Cb * yw : zero<A>());
  A ywb = isSp ? Cb * rho : zero<A>();
  Tb += wsum(Tbr) + wsum(Tth) - rhob * rho * iT;
  const A syb = -rhob * rho / sy;
  ywb += syb;
  Yb += ywb * iWk;
  wsync();
  return lane == 0 ? Tb : (isSp ? Yb : zero<A>());
}

// Solve M^T x = b with the pivot-ordered factors P M = L U stored row-wise in
// LDS F (row k of P M = L U at F + k S): U^T z = b, L^T v = z, x = P^T v.
// Lane j first loads column j of the factors into registers (all loads in
// flight together), so the two triangular sweeps run on registers and
// readlane broadcasts only.  Rows >= N are not factors: those steps are
// skipped (uniform branch); padding lanes read column 0 and are masked.  The
// masks act on the multipliers, off the chain through b (adding -0 leaves b
// as it is).
template <int NP>
__device__ inline double lu_solve_T(const double* F, int N, int S, int lane, int mystep, double myrdiag, double b) {
  const int col = lane < N ? lane : 0;
  double cv[NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) cv[k] = k < N ? F[k * S + col] : 0.0;
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    if (k < N) {
      const double zk = readlane(b * myrdiag, k);
      b = fma((lane > k && lane < N) ? -cv[k] : -0.0, zk, b);
    }
  }
  b *= myrdiag;
#pragma unroll
  for (int k = NP - 1; k >= 0; --k) {
    if (k < N) {
      const double vk = readlane(b, k);
      b = fma(lane < k ? -cv[k] : -0.0, vk, b);
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
