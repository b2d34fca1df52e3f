// Seulex-family integrator, extrapolated linearly implicit Euler, the paper's
// integrator (section 2.3), on both layouts (wavefront path for N <= 64,
// workgroup path above).
//
// Over a step H with J = J(y0) frozen, column j (1-based) takes n_j = j
// linearly implicit Euler substeps of size h = H / n_j,
//   (I/h - J)(y_{m+1} - y_m) = f(y_m)          (Eq. 2 with h = H / n_j),
// and the Aitken-Neville table
//   T_{j,l+1} = T_{j,l} + (T_{j,l} - T_{j-1,l}) (n_{j-l} / (n_j - n_{j-l}))
// gains one order per column.  Column k's error is ||T_{k,k} - T_{k,k-1}||;
// the next column among k-1, k, k+1 minimises the work per unit step
// A_j / H_j with A_j = sum_{i<=j} (n_i + 1).  Every factorisation and solve
// reuses the LU of the Rosenbrock path of the same layout; each lane (thread)
// keeps its component of the last two rows of the table in registers.
#pragma once
#include "chem_cell.hpp"
#include "chem_wg.hpp"

namespace chem {

constexpr int SX_KMAX = 6;

__device__ __forceinline__ double sx_pick(const double (&r)[SX_KMAX], int i) {
  double v = r[0];
#pragma unroll
  for (int l = 1; l < SX_KMAX; ++l) v = i == l ? r[l] : v;
  return v;
}

template <int NP, bool PROF>
__device__ void integrate_cell_sx(const MechView& m, const CellWs& w, const IntArgs& a, int64_t c) {
  const int lane = lane_id();
  const int N = m.d.N;
  Prof<PROF> pf;
  const unsigned long long t_begin = PROF ? __builtin_readcyclecounter() : 0ull;
  if (lane == 0) {
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
  int nlu = 0, nsub = 0;  // work counters of the instrumented kernel
  const bool bad = lane < N && (!__builtin_isfinite(y) || (lane == 0 && !(y > 0.0)));
  if (ballot(bad)) status = ST_NONFINITE;
  double t = 0.0;
  bool rej_last = false;
  int k = 3;
  double row[NP];
  int mystep;
  double myrdiag;
  while (status == ST_OK && t < dt) {
    pf.start();
    const double f0 = jac_pass<NP, PROF>(m, w, y, a.p, lane, row, &pf);
    pf.stop(0);
    bool fresh = true;
    int nsing = 0;
    bool accepted = false;
    while (!accepted) {
      if (attempts >= a.ctl.max_steps) { status = ST_TOO_MANY; break; }
      if (!(hprop >= a.ctl.h_min)) { status = ST_UNDERFLOW; break; }
      double H = hprop;
      bool clipped = false;
      if (H >= dt - t) { H = dt - t; clipped = true; }
      ++attempts;
      if (fresh && ballot(lane < N && !__builtin_isfinite(f0))) { status = ST_NONFINITE; break; }
      // the extrapolation table, row by row: R = current row, P = previous row
      double R[SX_KMAX], P[SX_KMAX];
#pragma unroll
      for (int l = 0; l < SX_KMAX; ++l) R[l] = P[l] = 0.0;
      int rc = 0;
#pragma clang loop unroll(disable)
      for (int j = 0; j < k; ++j) {
        const int nj = j + 1;
        const double h = H / nj;
        pf.start();
        const bool okm = form_matrix<NP>(w, N, m.d.S, lane, 1.0 / h, row);
        pf.stop(1);
        if (!okm) { rc = 2; break; }
        const int info = lu_factor<NP>(row, N, lane, mystep, myrdiag);
        if (info) {
          pf.stop(2);
          rc = 1;
          break;
        }
        const int src = permute_rows<NP>(row, N, lane, mystep, myrdiag, w.slot);
        pf.stop(2);
        if (PROF) {
          ++nlu;
          nsub += nj;
        }
        double yc = y;
#pragma clang loop unroll(disable)
        for (int mm = 0; mm < nj; ++mm) {
          double fv = f0;
          if (mm > 0) {
            pf.start();
            fv = rhs(m, w, lane < N ? yc : 0.0, a.p, lane);
            pf.stop(3);
          }
          pf.start();
          yc += lu_solve<NP>(row, N, lane, src, myrdiag, lane < N ? fv : 0.0);
          pf.stop(4);
        }
        // new row of the table from the previous one
#pragma unroll
        for (int l = 0; l < SX_KMAX; ++l) P[l] = R[l];
        R[0] = yc;
#pragma unroll
        for (int l = 1; l < SX_KMAX; ++l) {
          if (l <= j) R[l] = R[l - 1] + (R[l - 1] - P[l - 1]) * ((double)(j + 1 - l) / l);
        }
      }
      if (rc == 0 && c >= a.fail_lu_lo && c < a.fail_lu_hi) rc = 1;  // testing: as if M were singular
      if (rc == 2 && fresh) { status = ST_NONFINITE; break; }
      fresh = false;
      if (rc) {
        ++rejects;
        if (++nsing > 5) { status = ST_SINGULAR; break; }
        hprop = 0.5 * H;
        rej_last = true;
        continue;
      }
      // column k's value and error; column k-1's error for the order decision
      const double yk = sx_pick(R, k - 1), ykm = sx_pick(R, k - 2);
      double e = 0.0, e1 = 0.0;
      if (lane < N) {
        const double sc = a.atol + a.rtol * fmax(fabs(y), fabs(yk));
        e = (yk - ykm) / sc;
        const double p1 = sx_pick(P, k - 2), p2 = sx_pick(P, k - 3 < 0 ? 0 : k - 3);
        const double sc1 = a.atol + a.rtol * fmax(fabs(y), fabs(p1));
        e1 = (p1 - p2) / sc1;
      }
      const double errk = sqrt(wave_sum(e * e) / N);
      const double errk1 = k >= 3 ? sqrt(wave_sum(e1 * e1) / N) : 0.0;
      const bool fin = __builtin_isfinite(errk) && ballot(lane < N && !__builtin_isfinite(yk)) == 0ull;
      if (!fin) {
        ++rejects;
        hprop = a.ctl.fac_min * H;
        rej_last = true;
        continue;
      }
      const double Hk = H * fmin(a.ctl.fac_max, fmax(a.ctl.fac_min, a.ctl.fac_safe * pow(errk, -1.0 / k)));
      double Hk1 = 0.0;
      if (k >= 3 && __builtin_isfinite(errk1))
        Hk1 = H * fmin(a.ctl.fac_max, fmax(a.ctl.fac_min, a.ctl.fac_safe * pow(errk1, -1.0 / (k - 1))));
      if (uniform_int(errk <= 1.0)) {
        accepted = true;
        ++steps;
        t = clipped ? dt : t + H;
        y = yk;
        // work per column: A_j = sum_{i<=j} (n_i + 1) = j (j + 3) / 2
        const double Ak = 0.5 * k * (k + 3), Ak1 = 0.5 * (k - 1) * (k + 2), Akp = 0.5 * (k + 1) * (k + 4);
        int knew = k;
        double hn = Hk;
        if (k >= 3 && Hk1 > 0.0 && Ak1 / Hk1 < 0.8 * (Ak / Hk)) {
          knew = k - 1;
          hn = Hk1;
        } else if (k < SX_KMAX && (k == 2 || Hk1 <= 0.0 || Ak / Hk < 0.9 * (Ak1 / Hk1))) {
          knew = k + 1;
          hn = Hk * (Akp / Ak);
        }
        if (rej_last) {
          hn = fmin(hn, H);
          knew = min(knew, k);
        }
        if (clipped) hn = fmax(hn, hprop);
        hprop = hn;
        k = knew;
        rej_last = false;
      } else {
        ++rejects;
        hprop = Hk;
        rej_last = true;
      }
    }
  }
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
    if (lane == 6) v = (unsigned long long)nlu;
    if (lane == 7) v = (unsigned long long)nsub;
    a.prof[c * 8 + lane] = v;
  }
}

// The same integrator on the workgroup path (64 < N <= 255): thread t owns
// component t, every column forms and factors M = I/h - J in the
// workgroup's scratch slot (the Jacobian's sparse part and rank-1 vectors
// stay intact across columns), norms are workgroup sums, so every control
// value is identical in all threads.
template <bool PROF>
__device__ void wg_integrate_cell_sx(const MechView& m, const WgWs& w, const WgTerms& tl, double* Sx, double* Mx,
                                     int NP, const IntArgs& a, int64_t c) {
  const int t = threadIdx.x, N = m.d.N;
  Prof<PROF> pf;
  const unsigned long long t_begin = PROF ? __builtin_readcyclecounter() : 0ull;
  double y = t < N ? a.state[(int64_t)t * a.ld + c] : 0.0;
  const double dt = a.dt;
  const double hin = a.h[c];
  double hprop = (__builtin_isfinite(hin) && hin > 0.0) ? fmin(hin, dt) : dt;
  int status = ST_OK, steps = 0, rejects = 0, attempts = 0;
  int nlu = 0, nsub = 0;  // work counters of the instrumented kernel
  const bool bad = t < N && (!__builtin_isfinite(y) || (t == 0 && !(y > 0.0)));
  if (block_any(bad, w.flag + 1)) status = ST_NONFINITE;
  double tt = 0.0;
  bool rej_last = false;
  int k = 3;
  while (status == ST_OK && tt < dt) {
    pf.start();
    const double f0 = wg_jac(m, w, tl, Sx, NP, y, a.p);
    pf.stop(0);
    bool fresh = true;
    int nsing = 0;
    bool accepted = false;
    while (!accepted) {
      if (attempts >= a.ctl.max_steps) { status = ST_TOO_MANY; break; }
      if (!(hprop >= a.ctl.h_min)) { status = ST_UNDERFLOW; break; }
      double H = hprop;
      bool clipped = false;
      if (H >= dt - tt) { H = dt - tt; clipped = true; }
      ++attempts;
      if (fresh && block_any(t < N && !__builtin_isfinite(f0), w.flag + 1)) { status = ST_NONFINITE; break; }
      double R[SX_KMAX], P[SX_KMAX];
#pragma unroll
      for (int l = 0; l < SX_KMAX; ++l) R[l] = P[l] = 0.0;
      int rc = 0;
#pragma clang loop unroll(disable)
      for (int j = 0; j < k; ++j) {
        const int nj = j + 1;
        const double h = H / nj;
        pf.start();
        const bool okm = wg_form(m, w, Sx, Mx, NP, 1.0 / h);
        pf.stop(1);
        if (!okm) { rc = 2; break; }
        const int info = wg_lu<PROF>(w, Mx, NP, &pf);
        pf.stop(2);
        if (info) { rc = 1; break; }
        if (PROF) {
          ++nlu;
          nsub += nj;
        }
        double yc = y;
#pragma clang loop unroll(disable)
        for (int mm = 0; mm < nj; ++mm) {
          double fv = f0;
          if (mm > 0) {
            pf.start();
            fv = wg_rhs(m, w, t < N ? yc : 0.0, a.p);
            pf.stop(3);
          }
          pf.start();
          yc += wg_solve(w, Mx, NP, t < N ? fv : 0.0);
          pf.stop(4);
        }
#pragma unroll
        for (int l = 0; l < SX_KMAX; ++l) P[l] = R[l];
        R[0] = yc;
#pragma unroll
        for (int l = 1; l < SX_KMAX; ++l) {
          if (l <= j) R[l] = R[l - 1] + (R[l - 1] - P[l - 1]) * ((double)(j + 1 - l) / l);
        }
      }
      if (rc == 0 && c >= a.fail_lu_lo && c < a.fail_lu_hi) rc = 1;  // testing: as if M were singular
      if (rc == 2 && fresh) { status = ST_NONFINITE; break; }
      fresh = false;
      if (rc) {
        ++rejects;
        if (++nsing > 5) { status = ST_SINGULAR; break; }
        hprop = 0.5 * H;
        rej_last = true;
        continue;
      }
      const double yk = sx_pick(R, k - 1), ykm = sx_pick(R, k - 2);
      double e = 0.0, e1 = 0.0;
      if (t < N) {
        const double sc = a.atol + a.rtol * fmax(fabs(y), fabs(yk));
        e = (yk - ykm) / sc;
        const double p1 = sx_pick(P, k - 2), p2 = sx_pick(P, k - 3 < 0 ? 0 : k - 3);
        const double sc1 = a.atol + a.rtol * fmax(fabs(y), fabs(p1));
        e1 = (p1 - p2) / sc1;
      }
      const double errk = sqrt(block_sum(e * e, w.red) / N);
      const double errk1 = k >= 3 ? sqrt(block_sum(e1 * e1, w.red) / N) : 0.0;
      const bool fin = __builtin_isfinite(errk) && !block_any(t < N && !__builtin_isfinite(yk), w.flag + 1);
      if (!fin) {
        ++rejects;
        hprop = a.ctl.fac_min * H;
        rej_last = true;
        continue;
      }
      const double Hk = H * fmin(a.ctl.fac_max, fmax(a.ctl.fac_min, a.ctl.fac_safe * pow(errk, -1.0 / k)));
      double Hk1 = 0.0;
      if (k >= 3 && __builtin_isfinite(errk1))
        Hk1 = H * fmin(a.ctl.fac_max, fmax(a.ctl.fac_min, a.ctl.fac_safe * pow(errk1, -1.0 / (k - 1))));
      if (errk <= 1.0) {
        accepted = true;
        ++steps;
        tt = clipped ? dt : tt + H;
        y = yk;
        const double Ak = 0.5 * k * (k + 3), Ak1 = 0.5 * (k - 1) * (k + 2), Akp = 0.5 * (k + 1) * (k + 4);
        int knew = k;
        double hn = Hk;
        if (k >= 3 && Hk1 > 0.0 && Ak1 / Hk1 < 0.8 * (Ak / Hk)) {
          knew = k - 1;
          hn = Hk1;
        } else if (k < SX_KMAX && (k == 2 || Hk1 <= 0.0 || Ak / Hk < 0.9 * (Ak1 / Hk1))) {
          knew = k + 1;
          hn = Hk * (Akp / Ak);
        }
        if (rej_last) {
          hn = fmin(hn, H);
          knew = min(knew, k);
        }
        if (clipped) hn = fmax(hn, hprop);
        hprop = hn;
        k = knew;
        rej_last = false;
      } else {
        ++rejects;
        hprop = Hk;
        rej_last = true;
      }
    }
  }
  if (t < N) a.state[(int64_t)t * a.ld + c] = y;
  if (t == 0) {
    a.h[c] = fmin(hprop, dt);
    if (a.steps) a.steps[c] = steps;
    if (a.rejects) a.rejects[c] = rejects;
    if (a.status) a.status[c] = status;
    if (a.failed && status != ST_OK) atomicAdd(a.failed, 1ull);
  }
  if (PROF && a.prof && t < 8) {
    unsigned long long v = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i)
      if (t == i) v = pf.c[i];
    if (t == 5) v = __builtin_readcyclecounter() - t_begin;
    if (t == 6) v = (unsigned long long)nlu;
    if (t == 7) v = (unsigned long long)nsub;
    a.prof[c * 8 + t] = v;
  }
  __syncthreads();
}

}  // namespace chem
