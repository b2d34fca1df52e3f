// Device solver for one cell per wavefront (N <= NP <= 64).
//
// Layout: lane i owns component i of every state-sized vector (lane 0 = T,
// lane 1+k = Y_k) and row i of the iteration matrix M = I/(gamma h) - J, held
// in NP registers.  Reaction-level work runs one reaction per lane in rounds
// of 64; species-level work runs one species per lane.  The Jacobian is
// assembled in the wave's LDS workspace, rows owned by lanes, so its
// accumulation is deterministic.
#pragma once
#include "chem_common.hpp"

namespace chem {

struct MechView {
  MechDims d;
  const double* lnA;      // LDS
  const double* b;        // LDS
  const double* th;       // LDS
  const uint64_t* sp;     // LDS: reactant slots in bytes 0..2, products 3..5, n_reac byte 6, n_prod byte 7
  const double* W;        // LDS
  const double* iW;       // LDS
  const int32_t* cptr;    // LDS [K+1]
  const uint32_t* cent;   // LDS [L] (r << 8) | (uint8)nu
  const int32_t* tbp;     // LDS [R - R0 + 1]
  const int32_t* tbs;     // LDS third-body species
  const double* tbd;      // LDS efficiency - 1
  const double* troe;     // LDS [R - R1][8]
  const double* nasa;     // global [K][16]
  const uint32_t* jsched; // global [jit][64] species-scatter schedule: (r << 16) | (k << 8) | (uint8)nu
  int jit;
};

__device__ inline MechView make_view(const uint8_t* lds, const IntArgs& a) {
  MechView m;
  m.d = a.d;
  m.lnA = (const double*)(lds + a.d.o_lnA);
  m.b = (const double*)(lds + a.d.o_b);
  m.th = (const double*)(lds + a.d.o_th);
  m.sp = (const uint64_t*)(lds + a.d.o_sp);
  m.W = (const double*)(lds + a.d.o_W);
  m.iW = (const double*)(lds + a.d.o_iW);
  m.cptr = (const int32_t*)(lds + a.d.o_cptr);
  m.cent = (const uint32_t*)(lds + a.d.o_cent);
  m.tbp = (const int32_t*)(lds + a.d.o_tbp);
  m.tbs = (const int32_t*)(lds + a.d.o_tbs);
  m.tbd = (const double*)(lds + a.d.o_tbd);
  m.troe = (const double*)(lds + a.d.o_troe);
  m.nasa = a.nasa;
  m.jsched = a.jsched;
  m.jit = a.jsched_it;
  return m;
}

// Per-wave LDS workspace.
struct CellWs {
  double* J;    // [N][S]
  double* rk;   // [R] q (RHS) or k_eff (Jacobian)
  double* rkr;  // [R] k_eff / K_c
  double* rdm;  // [R - R0] d q / d[M] of the third-body and falloff reactions
  double* rdt;  // [R] d q / dT at fixed C
  double* C;    // [64+1] concentrations, C[K] = 1 (padding species)
  double* g;    // [64+1] g/RT (reused for mass enthalpy in the Jacobian pass)
  double* hR;   // [64+1] h/RT
  int* slot;    // [64] row permutation scratch
};

// Everything of a wave's workspace but the Jacobian block.
__host__ __device__ inline int wave_rates_doubles(int R, int R0) { return 3 * R + (R - R0 + 1) + 3 * 66 + 32; }
// S = NP + 1, so reads of static columns j < NP + 1 from any row stay inside
// the J block (its last row is followed by the reaction arrays).
__host__ __device__ inline int cell_ws_doubles(int N, int S, int R, int R0) { return N * S + wave_rates_doubles(R, R0); }

// Workspace after base; with_J = false leaves J to be set from a slot.
__device__ inline CellWs make_ws(double* base, const MechDims& d, bool with_J = true) {
  CellWs w;
  w.J = with_J ? base : nullptr;
  w.rk = with_J ? base + d.N * d.S : base;
  w.rkr = w.rk + d.R;
  w.rdt = w.rkr + d.R;
  w.rdm = w.rdt + d.R;
  w.C = w.rdm + (d.R - d.R0 + 1);
  w.g = w.C + 66;
  w.hR = w.g + 66;
  w.slot = (int*)(w.hR + 66);
  return w;
}

// Jacobian slots shared by the waves of a workgroup: a wave holds one from
// the start of the Jacobian's species pass until M is formed in registers, so
// a workgroup can run more cells than it has Jacobian blocks.  flags[s] is 0
// when slot s is free.  Acquisition is bounded: after `limit` sleeping polls a
// wave gives up (the caller marks its cell failed), so no wave can wait
// forever.
struct SlotPool {
  int* flags;
  double* base;
  int nslots;
  int slot_doubles;
  __device__ double* slot(int s) const { return base + (size_t)s * slot_doubles; }
  __device__ int acquire(unsigned limit) const {
    int got = -1;
    for (unsigned spin = 0; spin < limit; ++spin) {
      int v = -1;
      if (lane_id() == 0) {
        for (int s = 0; s < nslots; ++s) {
          int expected = 0;
          if (__hip_atomic_compare_exchange_strong(&flags[s], &expected, 1, __ATOMIC_ACQUIRE, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_WORKGROUP)) {
            v = s;
            break;
          }
        }
      }
      got = __builtin_amdgcn_readlane(v, 0);
      if (got >= 0) break;
      __builtin_amdgcn_s_sleep(4);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    return got;
  }
  __device__ void release(int s) const {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    if (lane_id() == 0) __hip_atomic_store(&flags[s], 0, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
};

// Uniform mixture quantities of one evaluation point.
struct Mix {
  double T, lnT, iT, rho, iRho, Wbar, cp, Ctot, lnPRT;
};

// Per-phase cycle counters of one wave (compiled in only when PROF is true):
// 0 Jacobian pass (with f(y_n)), 1 forming M, 2 LU, 3 stage f evaluations,
// 4 triangular solves, 5 everything, 6 and 7 the reaction and species parts
// of the Jacobian pass.
template <bool PROF>
struct Prof {
  unsigned long long c[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  unsigned long long t = 0;
  __device__ __forceinline__ void start() {
    if (PROF) t = __builtin_readcyclecounter();
  }
  __device__ __forceinline__ void add(int i, unsigned long long since) {
    if (PROF) c[i] += __builtin_readcyclecounter() - since;
  }
  __device__ __forceinline__ unsigned long long now() const { return PROF ? __builtin_readcyclecounter() : 0ull; }
  __device__ __forceinline__ void stop(int i) {
    if (PROF) {
      const unsigned long long n = __builtin_readcyclecounter();
      c[i] += n - t;
      t = n;
    }
  }
};

// Lane-local species thermo: NASA-7 cp/R, h/RT, s/R and d(cp/R)/dT.
struct SpThermo {
  double cpR, hRT, sR, dcpR;
};

__device__ inline SpThermo nasa7(const double* row, double T, double lnT, double iT) {
  // both ranges are loaded before T is known, so the loads overlap the log
  double lo[7], hi[7];
#pragma unroll
  for (int i = 0; i < 7; ++i) {
    lo[i] = row[1 + i];
    hi[i] = row[8 + i];
  }
  const bool high = T > row[0];
  double a[7];
#pragma unroll
  for (int i = 0; i < 7; ++i) a[i] = high ? hi[i] : lo[i];
  SpThermo t;
  t.cpR = a[0] + T * (a[1] + T * (a[2] + T * (a[3] + T * a[4])));
  t.hRT = a[0] + T * (a[1] * 0.5 + T * (a[2] * (1.0 / 3.0) + T * (a[3] * 0.25 + T * a[4] * 0.2))) + a[5] * iT;
  t.sR = a[0] * lnT + T * (a[1] + T * (a[2] * 0.5 + T * (a[3] * (1.0 / 3.0) + T * a[4] * 0.25))) + a[6];
  t.dcpR = a[1] + T * (2.0 * a[2] + T * (3.0 * a[3] + T * 4.0 * a[4]));
  return t;
}

// Species phase shared by f and J: thermo at T, mixture density, and the
// concentrations / g/RT / h/RT the reaction lanes gather.  Returns the lane's
// species thermo (garbage on non-species lanes).
__device__ inline SpThermo species_phase(const MechView& m, const CellWs& w, double y, double p, int lane,
                                         Mix& x, double& Yk) {
  const int K = m.d.K;
  const bool isSp = lane >= 1 && lane <= K;
  const int k = isSp ? lane - 1 : 0;
  x.T = readlane(y, 0);
  x.lnT = log(x.T);
  x.iT = 1.0 / x.T;
  SpThermo t = nasa7(m.nasa + 16 * k, x.T, x.lnT, x.iT);
  Yk = isSp ? y : 0.0;
  const double iWk = m.iW[k];
  const double yw = Yk * iWk;
  const double sy = wave_sum(yw);
  x.Wbar = 1.0 / sy;
  x.rho = p * x.Wbar * x.iT / RU;
  x.iRho = 1.0 / x.rho;
  x.Ctot = p * x.iT / RU;
  x.lnPRT = log(PATM * x.iT / RU);
  x.cp = wave_sum(isSp ? Yk * t.cpR * RU * iWk : 0.0);
  if (isSp) {
    w.C[k] = x.rho * yw;
    w.g[k] = t.hRT - t.sR;
    w.hR[k] = t.hRT;
  }
  wsync();
  return t;
}

// One reaction's slot data from the packed word.
struct Slots {
  int r0, r1, r2, p0, p1, p2, dnu;
};
__device__ __forceinline__ Slots unpack(uint64_t s) {
  Slots o;
  o.r0 = (int)(s & 0xFF);
  o.r1 = (int)((s >> 8) & 0xFF);
  o.r2 = (int)((s >> 16) & 0xFF);
  o.p0 = (int)((s >> 24) & 0xFF);
  o.p1 = (int)((s >> 32) & 0xFF);
  o.p2 = (int)((s >> 40) & 0xFF);
  o.dnu = (int)((s >> 56) & 0xFF) - (int)((s >> 48) & 0xFF);
  return o;
}

__device__ __forceinline__ double third_body(const MechView& m, const CellWs& w, int r, double Ctot) {
  double M = Ctot;
  const int e1 = m.tbp[r - m.d.R0 + 1];
#pragma clang loop unroll(disable)
  for (int e = m.tbp[r - m.d.R0]; e < e1; ++e) M += m.tbd[e] * w.C[m.tbs[e]];
  return M;
}

// Troe falloff: k = kinf Pr/(1+Pr) F, Pr = k0 [M]/kinf.  Returns k and, when
// Deriv, d k / d[M] / net-factor pieces and d ln k / dT.
template <bool Deriv>
__device__ __forceinline__ double troe_k(const MechView& m, int r, const Mix& x, double kf, double dlnkf, double M,
                                         double& dk_dM, double& dlnk_dT) {
  const double* t = m.troe + TROE_STRIDE * (r - m.d.R1);
  const double alpha = t[0], iT3 = t[1], iT1 = t[2], T2 = t[3];
  const double k0 = exp(t[4] + t[5] * x.lnT - t[6] * x.iT);
  const double Pr = k0 * M / kf;
  const double e3 = exp(-x.T * iT3), e1 = exp(-x.T * iT1), e2 = exp(-T2 * x.iT);
  const double Fc = (1.0 - alpha) * e3 + alpha * e1 + e2;
  const double xF = log10(Fc);
  const double L = log10(Pr);
  const double c = -0.4 - 0.67 * xF;
  const double n = 0.75 - 1.27 * xF;
  const double d = n - 0.14 * (L + c);
  const double f1 = (L + c) / d;
  const double den = 1.0 + f1 * f1;
  const double F = exp10(xF / den);
  const double ipr = 1.0 / (1.0 + Pr);
  const double k = k0 * M * ipr * F;
  if (Deriv) {
    const double id2 = 1.0 / (d * d);
    const double dlgF_dL = -xF * 2.0 * f1 / (den * den) * n * id2;
    const double dlgF_dx = 1.0 / den - xF * 2.0 * f1 / (den * den) * (-0.67 * d + 1.1762 * (L + c)) * id2;
    const double gg = ipr + dlgF_dL;
    dk_dM = k0 * F * ipr * gg;
    const double dFc = -(1.0 - alpha) * iT3 * e3 - alpha * iT1 * e1 + T2 * x.iT * x.iT * e2;
    const double dlnk0 = t[5] * x.iT + t[6] * x.iT * x.iT;
    dlnk_dT = dlnkf + gg * (dlnk0 - dlnkf) + dlgF_dx * dFc / Fc;
  }
  return k;
}

// f(Phi) for the wave's cell: lane i gets f_i.
__device__ inline double rhs(const MechView& m, const CellWs& w, double y, double p, int lane) {
  const int K = m.d.K, R = m.d.R;
  Mix x;
  double Yk;
  SpThermo t = species_phase(m, w, y, p, lane, x, Yk);
#pragma clang loop unroll(disable)
  for (int r = lane; r < R; r += WAVE) {
    const Slots s = unpack(m.sp[r]);
    const double lnkf = m.lnA[r] + m.b[r] * x.lnT - m.th[r] * x.iT;
    const double Rf = w.C[s.r0] * w.C[s.r1] * w.C[s.r2];
    const double Rr = w.C[s.p0] * w.C[s.p1] * w.C[s.p2];
    const double sng = w.g[s.p0] + w.g[s.p1] + w.g[s.p2] - w.g[s.r0] - w.g[s.r1] - w.g[s.r2];
    const double kf = exp(lnkf);
    const double iKc = exp(sng - s.dnu * x.lnPRT);  // 1/K_c
    double q = kf * (Rf - iKc * Rr);
    if (r >= m.d.R0) {
      const double M = third_body(m, w, r, x.Ctot);
      if (r < m.d.R1) {
        q *= M;
      } else {
        double dk, dl;
        q = troe_k<false>(m, r, x, kf, 0.0, M, dk, dl) * (Rf - iKc * Rr);
      }
    }
    w.rk[r] = q;
  }
  // omega_k = sum_r nu_kr q_r on the balanced species schedule of the
  // Jacobian pass (every lane takes about L/64 entries), accumulated with LDS
  // atomics in w.hR, which f does not read (the next thermo pass rewrites it)
  const bool isSp = lane >= 1 && lane <= K;
  if (isSp) w.hR[lane - 1] = 0.0;
  wsync();
  {
    const uint32_t* js = m.jsched + lane;
    uint32_t ent = js[0];
#pragma clang loop unroll(disable)
    for (int it = 0; it < m.jit; ++it) {
      const uint32_t cur = ent;
      if (it + 1 < m.jit) ent = js[(it + 1) * WAVE];
      if (cur != ~0u) atomicAdd(w.hR + ((cur >> 8) & 0xFF), (double)(int8_t)(cur & 0xFF) * w.rk[cur >> 16]);
    }
  }
  lds_wait();
  wsync();
  const double om = isSp ? w.hR[lane - 1] : 0.0;
  const double Q = wave_sum(isSp ? t.hRT * om : 0.0);
  const double fT = -RU * x.T * Q * x.iRho / x.cp;
  wsync();
  if (lane == 0) return fT;
  return isSp ? m.W[lane - 1] * om * x.iRho : 0.0;
}

// Analytic Jacobian (section 2.3) into w.J and f(Phi) into the return value.
//   J_kj = (W_k/W_j) dw_k/dC_j + W_k Wbar/(rho W_j) (w_k - s_k),  s_k = sum_i C_i dw_k/dC_i
//   J_kT = (W_k/rho) (dw_k/dT - s_k/T + w_k/T)
//   J_Tj = -(sum_k hm_k J_kj + f_T cpm_j)/c_p,  J_TT = -(sum_k hm_k J_kT + sum_k cpm_k f_k + f_T dc_p/dT)/c_p
// (hm, cpm: mass-specific enthalpy and heat capacity).  `row` is scratch.
// One-sided finite-difference Jacobian (the ablation of section 2.3): column
// j is (f(y + d_j e_j) - f(y)) / d_j with d_j = sqrt(eps) max(|y_j|, 1e-10)
// rounded to a representable step; N + 1 evaluations of f.  Returns f(y).
__device__ inline double jac_fd(const MechView& m, const CellWs& w, double y, double p, int lane) {
  const int N = m.d.N, S = m.d.S;
  const double f0 = rhs(m, w, y, p, lane);
#pragma clang loop unroll(disable)
  for (int j = 0; j < N; ++j) {
    const double yj = readlane(y, j);
    double d = 1.4901161193847656e-08 * fmax(fabs(yj), 1e-10);
    d = (yj + d) - yj;
    const double fj = rhs(m, w, lane == j ? yj + d : y, p, lane);
    if (lane < N) w.J[lane * S + j] = (fj - f0) / d;
  }
  wsync();
  return f0;
}

template <int NP, bool PROF = false>
__device__ inline double jac_pass(const MechView& m, const CellWs& w, double y, double p, int lane,
                                  double (&row)[NP], Prof<PROF>* pf = nullptr, bool fd = false) {
  if (PROF && fd) return jac_fd(m, w, y, p, lane);
  const int K = m.d.K, R = m.d.R, N = m.d.N, S = m.d.S;
  const unsigned long long t0 = PROF ? pf->now() : 0ull;
  Mix x;
  double Yk;
  SpThermo t = species_phase(m, w, y, p, lane, x, Yk);
#pragma clang loop unroll(disable)
  for (int r = lane; r < R; r += WAVE) {
    const Slots s = unpack(m.sp[r]);
    const double lnkf = m.lnA[r] + m.b[r] * x.lnT - m.th[r] * x.iT;
    const double Rf = w.C[s.r0] * w.C[s.r1] * w.C[s.r2];
    const double Rr = w.C[s.p0] * w.C[s.p1] * w.C[s.p2];
    const double sng = w.g[s.p0] + w.g[s.p1] + w.g[s.p2] - w.g[s.r0] - w.g[s.r1] - w.g[s.r2];
    const double snh = w.hR[s.p0] + w.hR[s.p1] + w.hR[s.p2] - w.hR[s.r0] - w.hR[s.r1] - w.hR[s.r2];
    const double kf = exp(lnkf);
    const double iKc = exp(sng - s.dnu * x.lnPRT);
    const double dlnkf = m.b[r] * x.iT + m.th[r] * x.iT * x.iT;
    const double dlnKc = (snh - (double)s.dnu) * x.iT;
    const double net = Rf - iKc * Rr;
    double keff = kf, dkM = 0.0, dqdT;
    if (r < m.d.R0) {
      dqdT = kf * (dlnkf * Rf - iKc * (dlnkf - dlnKc) * Rr);
    } else {
      const double M = third_body(m, w, r, x.Ctot);
      if (r < m.d.R1) {
        keff = kf * M;
        dkM = kf * net;
        dqdT = M * kf * (dlnkf * Rf - iKc * (dlnkf - dlnKc) * Rr);
      } else {
        double dlnk;
        keff = troe_k<true>(m, r, x, kf, dlnkf, M, dkM, dlnk);
        dkM *= net;
        dqdT = keff * (dlnk * net + iKc * Rr * dlnKc);
      }
    }
    w.rk[r] = keff;
    w.rkr[r] = keff * iKc;
    if (r >= m.d.R0) w.rdm[r - m.d.R0] = dkM;
    w.rdt[r] = dqdT;
  }
  if (PROF) pf->add(6, t0);
  const unsigned long long t1 = PROF ? pf->now() : 0ull;
  // species rows of dw/dC (sparse), scattered by the balanced schedule: lane l
  // takes entry it * 64 + l, species k and reaction r, and adds to row k of J.
  // While they are built, omega_k, d omega_k / dT and the row's dense
  // third-body sum are accumulated in J[k+1][0] (column 0, written after this
  // pass), hR[k] (free after the reaction phase) and J[0][k+1] (row 0, written
  // after this pass).  All additions are LDS atomics, in schedule order and,
  // within one instruction, in the hardware's lane order: deterministic.
  const bool isSp = lane >= 1 && lane <= K;
  double* Jr = w.J + lane * S;  // S = NP + 1: every static column index stays in the row
  if (lane < N) {
#pragma unroll
    for (int j = 0; j < NP + 1; ++j) Jr[j] = 0.0;
  }
  if (isSp) w.hR[lane - 1] = 0.0;
  wsync();
  {
    const uint32_t* js = m.jsched + lane;
    uint32_t ent = js[0];
#pragma clang loop unroll(disable)
    for (int it = 0; it < m.jit; ++it) {
      const uint32_t cur = ent;
      if (it + 1 < m.jit) ent = js[(it + 1) * WAVE];
      if (cur != ~0u) {
        const int r = (int)(cur >> 16), k = (int)((cur >> 8) & 0xFF);
        const double nu = (double)(int8_t)(cur & 0xFF);
        const Slots sl = unpack(m.sp[r]);
        const double c0 = w.C[sl.r0], c1 = w.C[sl.r1], c2 = w.C[sl.r2];
        const double d0 = w.C[sl.p0], d1 = w.C[sl.p1], d2 = w.C[sl.p2];
        const double kf = w.rk[r], kr = w.rkr[r], dq = w.rdt[r];
        double* Jk = w.J + (k + 1) * S;
        atomicAdd(Jk, nu * (kf * c0 * c1 * c2 - kr * d0 * d1 * d2));
        atomicAdd(w.hR + k, nu * dq);
        const double a = nu * kf, bb = -nu * kr;
        atomicAdd(Jk + 1 + sl.r0, a * c1 * c2);
        atomicAdd(Jk + 1 + sl.r1, a * c0 * c2);
        atomicAdd(Jk + 1 + sl.r2, a * c0 * c1);
        atomicAdd(Jk + 1 + sl.p0, bb * d1 * d2);
        atomicAdd(Jk + 1 + sl.p1, bb * d0 * d2);
        atomicAdd(Jk + 1 + sl.p2, bb * d0 * d1);
        if (r >= m.d.R0) {
          const double dm = nu * w.rdm[r - m.d.R0];
          atomicAdd(w.J + 1 + k, dm);
          const int t1 = m.tbp[r - m.d.R0 + 1];
#pragma clang loop unroll(disable)
          for (int q = m.tbp[r - m.d.R0]; q < t1; ++q) atomicAdd(Jk + 1 + m.tbs[q], dm * m.tbd[q]);
        }
      }
    }
  }
  lds_wait();
  wsync();
  double om = 0.0, dwdT = 0.0, adense = 0.0;
  if (isSp) {
    om = Jr[0];
    dwdT = w.hR[lane - 1];
    adense = w.J[lane];
  }
  // dense transform of the lane's row: rank-1 density term and W scaling
  // (uniform loop bounds: no per-column branches; padding columns set to 0)
  double fk = 0.0;
  if (isSp) {
    const int k = lane - 1;
    const double Wk = m.W[k];
    double sk = 0.0;
#pragma clang loop unroll_count(4)
    for (int j = 1; j < N; ++j) sk += w.C[j - 1] * (Jr[j] + adense);
    const double gam = Wk * x.Wbar * x.iRho * (om - sk);
#pragma clang loop unroll_count(4)
    for (int j = 1; j < N; ++j) Jr[j] = m.iW[j - 1] * (Wk * (Jr[j] + adense) + gam);
#pragma clang loop unroll(disable)
    for (int j = N; j < NP; ++j) Jr[j] = 0.0;
    Jr[0] = Wk * x.iRho * (dwdT - sk * x.iT + om * x.iT);
    fk = Wk * om * x.iRho;
    // mass-specific enthalpy for the T row (g/RT is no longer needed)
    w.g[k] = RU * x.T * t.hRT * m.iW[k];
  }
  const double Q = wave_sum(isSp ? t.hRT * om : 0.0);
  const double fT = -RU * x.T * Q * x.iRho / x.cp;
  const double cpm = isSp ? RU * t.cpR * m.iW[lane - 1] : 0.0;
  const double s1 = wave_sum(cpm * fk);
  const double dcpdT = wave_sum(isSp ? Yk * RU * t.dcpR * m.iW[lane - 1] : 0.0);
  wsync();
  // T row: column sums of the species rows weighted by mass enthalpy
  if (lane < N) {
    double acc = 0.0;
    double a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int k = 0;
#pragma clang loop unroll(disable)
    for (; k + 4 <= K; k += 4) {
      acc += w.g[k] * w.J[(1 + k) * S + lane];
      a1 += w.g[k + 1] * w.J[(2 + k) * S + lane];
      a2 += w.g[k + 2] * w.J[(3 + k) * S + lane];
      a3 += w.g[k + 3] * w.J[(4 + k) * S + lane];
    }
#pragma clang loop unroll(disable)
    for (; k < K; ++k) acc += w.g[k] * w.J[(1 + k) * S + lane];
    acc = (acc + a1) + (a2 + a3);
    w.J[lane] = (lane == 0) ? -(acc + s1 + fT * dcpdT) / x.cp : -(acc + fT * cpm) / x.cp;
  }
  wsync();
  if (PROF) pf->add(7, t1);
  return lane == 0 ? fT : fk;
}

// 1/x from the hardware estimate refined by two Newton steps (within an ulp
// or two of the correctly rounded quotient for normal x).
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// LU with partial pivoting of the row-per-lane matrix, with getrf's pivot
// rule: at step k the pivot is the unpivoted row of largest |a|, exact ties
// going to the row that comes first in getrf's current row order (the order
// after the interchanges k <-> pivot of the earlier steps).  No rows move: the
// lane chosen at step k records mystep = k, and pos tracks where getrf would
// hold the lane's row.  L multipliers of step k stay in column k of the
// remaining rows.  |a| is compared as an integer key: the upper 32 bits
// (sign cleared) by one wave max; only when several lanes share the largest
// upper half do the lower halves, and then the positions, decide.
// Steps run in static phases of four: phase P only touches columns >= 4P.
// Inside a phase the four columns of chunk P rotate through c0..c3 so that
// the pivot column is always c0; every register index is static.
// Returns the 1-based step of a zero pivot, or 0.  myipiv (lane k) receives
// getrf's ipiv[k]: the position the step-k pivot row held before its interchange.
template <int NP>
__device__ inline int lu_factor(double (&row)[NP], int N, int lane, int& mystep, double& myrdiag,
                                bool nopiv = false, int* myipiv = nullptr) {
  mystep = lane < N ? -1 : (1 << 20);
  myrdiag = 0.0;
  int info = 0;
  int pos = lane;
#pragma clang loop unroll(full)
  for (int P = 0; P < NP / 4; ++P) {
    const int k0 = 4 * P;
    const int k1 = min(k0 + 4, N);
    double c0 = row[k0], c1 = row[k0 + 1], c2 = row[k0 + 2], c3 = row[k0 + 3];
#pragma clang loop unroll(disable)
    for (int k = k0; k < k1; ++k) {
      const int kk = k - k0;
      const bool elig = mystep < 0;
      const unsigned long long mag = __builtin_bit_cast(unsigned long long, c0) & 0x7fffffffffffffffull;
      const unsigned key = elig ? (unsigned)(mag >> 32) : 0u;
      const unsigned kmax = wave_max_u32(key);
      unsigned long long cand = ballot(elig && key == kmax);
      bool sing = kmax == 0u;
      if (!nopiv && (sing || (cand & (cand - 1)) != 0ull)) {  // wave-uniform: rare tie path
        const bool c = elig && key == kmax;
        const unsigned lmax = wave_max_u32(c ? (unsigned)mag : 0u);
        sing = sing && lmax == 0u;
        cand = ballot(c && (unsigned)mag == lmax);
        if ((cand & (cand - 1)) != 0ull) {
          const bool tie = ((cand >> lane) & 1ull) != 0ull;
          const int pmin = 63 - (int)wave_max_u32(tie ? (unsigned)(63 - pos) : 0u);
          cand = ballot(tie && pos == pmin);
        }
      }
      // a zero pivot column is recorded and the factorisation runs on with
      // zero multipliers (no early exit keeps the control flow simple)
      // without pivoting (ablation) the pivot is row k itself
      if (nopiv) sing = !(readlane(c0, k) != 0.0);
      if (sing && info == 0) info = k + 1;
      const int p = sing ? 0 : (nopiv ? k : uniform_int(__builtin_ctzll(cand)));
      {  // getrf interchanges rows k and pos(p)
        const int pp = sing ? k : uniform_int(__builtin_amdgcn_readlane(pos, p));
        if (myipiv && lane == k) *myipiv = pp;
        const int np = pos == k ? pp : pos;
        pos = (lane == p && !sing) ? k : np;
      }
      const double piv = readlane(c0, p);
      const double rp = recip(piv);
      const bool upd = elig && lane != p && !sing;
      if (lane == p && !sing) {
        mystep = k;
        myrdiag = rp;
      }
      const double l = upd ? c0 * rp : 0.0;
      // c1..c3 hold columns k+1.. of the chunk first, then finished columns
      double u1 = readlane(c1, p), u2 = readlane(c2, p), u3 = readlane(c3, p);
      u1 = kk <= 2 ? u1 : 0.0;
      u2 = kk <= 1 ? u2 : 0.0;
      u3 = kk == 0 ? u3 : 0.0;
      c1 = fma(-l, u1, c1);
      c2 = fma(-l, u2, c2);
      c3 = fma(-l, u3, c3);
      c0 = upd ? l : c0;
      // four broadcasts in flight before their four FMAs: the scalar
      // registers differ, so no broadcast waits on the previous FMA
#pragma unroll
      for (int j = k0 + 4; j < NP; j += 4) {
        const double u0 = readlane(row[j], p), v1 = readlane(row[j + 1], p);
        const double v2 = readlane(row[j + 2], p), v3 = readlane(row[j + 3], p);
        __builtin_amdgcn_sched_barrier(0);
        row[j] = fma(-l, u0, row[j]);
        row[j + 1] = fma(-l, v1, row[j + 1]);
        row[j + 2] = fma(-l, v2, row[j + 2]);
        row[j + 3] = fma(-l, v3, row[j + 3]);
      }
      const double t = c0;
      c0 = c1;
      c1 = c2;
      c2 = c3;
      c3 = t;
    }
    // a short final phase re-aligns the rotation
#pragma clang loop unroll(disable)
    for (int r = max(k1 - k0, 0); r < 4; ++r) {
      const double t = c0;
      c0 = c1;
      c1 = c2;
      c2 = c3;
      c3 = t;
    }
    row[k0] = c0;
    row[k0 + 1] = c1;
    row[k0 + 2] = c2;
    row[k0 + 3] = c3;
  }
  return info;
}

// Moves the factored rows into pivot order (lane k receives the row chosen
// at step k), so that L is unit lower and U upper with lane = row; src is the
// lane each lane took its row from.
template <int NP>
__device__ inline int permute_rows(double (&row)[NP], int N, int lane, int mystep, double& myrdiag, int* slot) {
  if (lane < N) slot[mystep] = lane;
  wsync();
  const int src = lane < N ? slot[lane] : lane;
  wsync();
#pragma unroll
  for (int j = 0; j < NP; ++j) row[j] = __shfl(row[j], src);
  myrdiag = __shfl(myrdiag, src);
  return src;
}

// Solve M x = b with the permuted factors; lane i holds b_i and gets x_i.
// The right-hand side is gathered into pivot order, then forward substitution
// with the unit-lower L and back substitution with U (both by columns, the
// value of step k broadcast from lane k).  Every lane applies every column's
// update (a lane past its own step only changes a value it has already
// saved), so no per-element triangle mask is formed: masks of the factors
// would be loop invariants across a step's four solves and would hold two
// masked copies of the row in registers.
template <int NP>
__device__ inline double lu_solve(const double (&row)[NP], int N, int lane, int src, double myrdiag, double b) {
  // padding lanes carry b = 0 and zero rows, so all NP steps run unconditionally
  (void)N;
  b = __shfl(b, src);
  double y = 0.0;
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    const double yk = readlane(b, k);
    y = lane == k ? b : y;  // lane k's value is final at step k
    b = fma(-row[k], yk, b);
  }
  b = y;
  double x = 0.0;
#pragma unroll
  for (int k = NP - 1; k >= 0; --k) {
    const double bk = b * myrdiag;
    const double xk = readlane(bk, k);
    x = lane == k ? bk : x;
    b = fma(-row[k], xk, b);
  }
  return x;
}

// M = I/(gamma h) - J from the LDS Jacobian into row registers.  Returns
// false if a row holds a non-finite value.
template <int NP>
__device__ inline bool form_matrix(const CellWs& w, int N, int S, int lane, double d, double (&row)[NP]) {
  double chk = 0.0;
#pragma unroll
  for (int j = 0; j < NP; ++j) row[j] = 0.0;
  if (lane < N) {
    double* Jr = w.J + lane * S;
    const double jd = Jr[lane];
    Jr[lane] = jd - d;
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    // every load is in the row (j < NP < S) and taken unconditionally; the
    // padding columns are selected away, so the unrolled loop has no branches
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      const double v = Jr[j];
      row[j] = j < N ? -v : 0.0;
      chk += row[j];
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    Jr[lane] = jd;
  }
  return ballot(!__builtin_isfinite(chk)) == 0ull;
}

// One Rosenbrock attempt from y with f0 = f(y) and J(y) in LDS.  Writes ynew
// and err (lane-local); returns 1 if M is singular and 2 if M holds a
// non-finite value.  Stage vectors live in a shift register: after stage i,
// K0 = K_i, K1 = K_{i-1}, ..., so coefficient a_ij multiplies K_{i-1-j}.
template <int NP, bool PROF>
__device__ inline int ros_attempt(const MechView& m, const CellWs& w, const RosTable& tab, double p, int lane,
                                  double y, double f0, double h, double (&row)[NP], double& ynew, double& err,
                                  int& mystep, double& myrdiag, Prof<PROF>& pf, double* kst = nullptr,
                                  int* srcout = nullptr, bool nopiv = false, int formed = -1) {
  const int N = m.d.N;
  // formed: -1 form M here from the LDS Jacobian; 1 / 0: M is already in row
  // (formed by the caller while it held the Jacobian), finite / not finite
  bool okm = formed == 1;
  if (formed < 0) {
    pf.start();
    okm = form_matrix<NP>(w, N, m.d.S, lane, 1.0 / (tab.gamma * h), row);
    pf.stop(1);
  }
  if (!okm) return 2;
  const int info = lu_factor<NP>(row, N, lane, mystep, myrdiag, PROF && nopiv);
  if (info) {
    pf.stop(2);
    return 1;
  }
  const int src = permute_rows<NP>(row, N, lane, mystep, myrdiag, w.slot);
  pf.stop(2);
  const double ih = 1.0 / h;
  const int s = tab.s;
  double K0 = 0.0, K1 = 0.0, K2 = 0.0, K3 = 0.0;
  double fi = f0;
#pragma clang loop unroll(disable)
  for (int i = 0; i < s; ++i) {
    // contributions of K_{i-1}, K_{i-2}, K_{i-3}
    const double a0 = i >= 1 ? tab.a[i][i - 1] : 0.0, c0 = i >= 1 ? tab.c[i][i - 1] : 0.0;
    const double a1 = i >= 2 ? tab.a[i][i - 2] : 0.0, c1 = i >= 2 ? tab.c[i][i - 2] : 0.0;
    const double a2 = i >= 3 ? tab.a[i][i - 3] : 0.0, c2 = i >= 3 ? tab.c[i][i - 3] : 0.0;
    if (i > 0 && tab.newf[i]) {
      const double Yi = y + a0 * K0 + a1 * K1 + a2 * K2;
      pf.start();
      fi = rhs(m, w, lane < N ? Yi : 0.0, p, lane);
      pf.stop(3);
    }
    const double r = fi + ih * (c0 * K0 + c1 * K1 + c2 * K2);
    pf.start();
    const double ki = lu_solve<NP>(row, N, lane, src, myrdiag, lane < N ? r : 0.0);
    pf.stop(4);
    K3 = K2;
    K2 = K1;
    K1 = K0;
    K0 = ki;
  }
  if (kst) {  // stage order: kst[i] = K_i (four-stage tables)
    kst[0] = K3;
    kst[1] = K2;
    kst[2] = K1;
    kst[3] = K0;
    *srcout = src;
  }
  // after s stages K0 = K_{s-1}, K1 = K_{s-2}, ...
  const double m0 = tab.m[s - 1], e0 = tab.e[s - 1];
  const double m1 = s >= 2 ? tab.m[s - 2] : 0.0, e1 = s >= 2 ? tab.e[s - 2] : 0.0;
  const double m2 = s >= 3 ? tab.m[s - 3] : 0.0, e2 = s >= 3 ? tab.e[s - 3] : 0.0;
  const double m3 = s >= 4 ? tab.m[s - 4] : 0.0, e3 = s >= 4 ? tab.e[s - 4] : 0.0;
  ynew = y + (m0 * K0 + m1 * K1 + m2 * K2 + m3 * K3);
  err = e0 * K0 + e1 * K1 + e2 * K2 + e3 * K3;
  return 0;
}

// Adaptive integration of cell c over [0, dt]; the step-size controller
// follows the constants in a.ctl (accept iff err <= 1, no growth right after a
// rejection, non-finite err rejects with fac_min, the last step is clipped to
// dt and h_out is the last unclipped proposal capped at dt).
//
// With a slot pool the Jacobian block is not the wave's own: each attempt
// takes a slot, runs the Jacobian pass (which also yields f(y)), forms M in
// registers and gives the slot back.  A rejected attempt therefore repeats
// the Jacobian pass; the values are the same bits as the first time, so the
// results equal those of a wave that keeps its Jacobian.
template <int NP, bool PROF>
__device__ void integrate_cell(const MechView& m, const CellWs& w0, const IntArgs& a, int64_t c,
                               const SlotPool* pool = nullptr) {
  const int lane = lane_id();
  Prof<PROF> pf;
  const unsigned long long t_begin = PROF ? __builtin_readcyclecounter() : 0ull;
  const int N = m.d.N;
  CellWs w = w0;
  if (lane == 0) {  // padding species: C = 1, g/RT = h/RT = 0
    w.C[m.d.K] = 1.0;
    w.g[m.d.K] = 0.0;
    w.hR[m.d.K] = 0.0;
  }
  wsync();
  double y = lane < N ? a.state[(int64_t)lane * a.ld + c] : 0.0;
  const double dt = a.dt;
  const double hin = a.h[c];
  double hprop = (__builtin_isfinite(hin) && hin > 0.0) ? fmin(hin, dt) : dt;
  int status = ST_OK, steps = 0, rejects = 0, attempts = 0;
  const bool bad = lane < N && (!__builtin_isfinite(y) || (lane == 0 && !(y > 0.0)));
  if (ballot(bad)) status = ST_NONFINITE;
  double t = 0.0;
  bool rej_last = false;
  const int nck = a.tape_y ? a.max_tape / a.ckpt + 1 : 0;
  if (a.tape_y && lane < N) a.tape_y[(c * (int64_t)nck) * N + lane] = y;
  double row[NP];
  int mystep;
  double myrdiag;
  int ntape = 0;
  const RosTable& tab = kTables[a.method];
  while (status == ST_OK && t < dt) {
    double f0 = 0.0;
    if (!pool) {
      pf.start();
      f0 = jac_pass<NP, PROF>(m, w, y, a.p, lane, row, &pf, PROF && a.jac_fd);
      pf.stop(0);
    }
    bool fresh = true;
    int nsing = 0;
    bool accepted = false;
    while (!accepted) {
      if (attempts >= a.ctl.max_steps) { status = ST_TOO_MANY; break; }
      if (!(hprop >= a.ctl.h_min)) { status = ST_UNDERFLOW; break; }
      double h = hprop;
      bool clipped = false;
      if (h >= dt - t) { h = dt - t; clipped = true; }
      ++attempts;
      int formed = -1;
      if (pool) {
        const int sl = pool->acquire(1u << 26);
        if (sl < 0) { status = ST_NONFINITE; break; }  // unreachable unless a slot is never returned
        w.J = pool->slot(sl);
        pf.start();
        f0 = jac_pass<NP, PROF>(m, w, y, a.p, lane, row, &pf, PROF && a.jac_fd);
        pf.stop(0);
        formed = form_matrix<NP>(w, N, m.d.S, lane, 1.0 / (tab.gamma * h), row) ? 1 : 0;
        pf.stop(1);
        pool->release(sl);
        w.J = nullptr;
      }
      if (fresh && ballot(lane < N && !__builtin_isfinite(f0))) { status = ST_NONFINITE; break; }
      double ynew, err;
      int rc = ros_attempt<NP, PROF>(m, w, tab, a.p, lane, y, f0, h, row, ynew, err, mystep, myrdiag, pf, nullptr,
                                     nullptr, PROF && a.lu_nopiv, formed);
      if (rc == 0 && c >= a.fail_lu_lo && c < a.fail_lu_hi) rc = 1;  // testing: as if M were singular
      if (rc == 2 && fresh) { status = ST_NONFINITE; break; }
      fresh = false;
      if (rc) {
        ++rejects;
        if (++nsing > 5) { status = ST_SINGULAR; break; }
        hprop = 0.5 * h;
        rej_last = true;
        continue;
      }
      double e = 0.0;
      if (lane < N) {
        const double sc = a.atol + a.rtol * fmax(fabs(y), fabs(ynew));
        e = err / sc;
      }
      const double en = sqrt(wave_sum(e * e) / N);
      const bool fin = __builtin_isfinite(en) && ballot(lane < N && !__builtin_isfinite(ynew)) == 0ull;
      if (!fin) {
        ++rejects;
        hprop = a.ctl.fac_min * h;
        rej_last = true;
        continue;
      }
      const double fac = fmin(a.ctl.fac_max, fmax(a.ctl.fac_min, a.ctl.fac_safe * pow(en, -1.0 / a.q)));
      if (uniform_int(en <= 1.0)) {
        accepted = true;
        ++steps;
        if (a.tape_h) {
          if (ntape < a.max_tape) {
            if (lane == 0) a.tape_h[c * (int64_t)a.max_tape + ntape] = h;
          }
          ++ntape;
        }
        t = clipped ? dt : t + h;
        y = ynew;
        double hn = h * fac;
        if (rej_last) hn = fmin(hn, h);
        if (clipped) hn = fmax(hn, hprop);
        hprop = hn;
        rej_last = false;
        if (a.tape_y && ntape <= a.max_tape && (ntape % a.ckpt) == 0 && lane < N)
          a.tape_y[(c * (int64_t)nck + ntape / a.ckpt) * N + lane] = y;
      } else {
        ++rejects;
        hprop = h * fac;
        rej_last = true;
      }
    }
  }
  if (a.tape_h && ntape > a.max_tape && status == ST_OK) status = ST_TAPE;
  if (lane < N) a.state[(int64_t)lane * a.ld + c] = y;
  if (lane == 0) {
    a.h[c] = fmin(hprop, dt);
    if (a.steps) a.steps[c] = steps;
    if (a.rejects) a.rejects[c] = rejects;
    if (a.status) a.status[c] = status;
    if (a.failed && status != ST_OK) atomicAdd(a.failed, 1ull);
  }
  if (PROF && a.prof && lane < 8) {
    unsigned long long v = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i)
      if (lane == i) v = pf.c[i];
    if (lane == 5) v = __builtin_readcyclecounter() - t_begin;
    a.prof[c * 8 + lane] = v;
  }
}

}  // namespace chem
