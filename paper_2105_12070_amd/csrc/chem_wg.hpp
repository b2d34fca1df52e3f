// Device solver for one cell per 256-thread workgroup (64 < N <= 256).
//
// Thread t owns component t of every state-sized vector (t = 0 is T, t = 1+k
// is Y_k).  The iteration matrix M = I/(gamma h) - J of a 151-species cell
// (182 KB) does not fit in LDS, so each workgroup keeps two NP x NP FP64
// matrices in a global scratch slot (L2/MALL resident while the cell is
// worked on): Sx, the sparse part of d omega/dC at its structural positions,
// and Mx, the matrix being factored.  The LU is blocked by 16 columns: the
// panel is staged in LDS and factored by one wave (in registers up to 192
// rows; partial pivoting, first largest |a|), its row interchanges are
// applied to the other columns, the 16 rows of U are formed by a triangular
// solve, and the trailing matrix takes one rank-16 update per panel on FP64
// MFMA (16 x 16 output tiles, operands from LDS).  The Jacobian
// is assembled without atomics: every species row walks a host-built list of
// its nonzero columns, each with the reaction terms that contribute to it, in
// a fixed order (the longest rows in two segments, the second one on a thread
// that owns no row).  All sums over threads are fixed-order, so results are
// bitwise reproducible.
#pragma once
#include "chem_cell.hpp"

namespace chem {

constexpr int WG = 256;  // threads per workgroup (4 waves)
constexpr int WNB = 16;  // panel width of the blocked LU

// Jacobian term lists of the workgroup path (global memory, built by the
// loader).  Row k (species k) owns groups [gptr[k], gptr[k+1]); group g covers
// terms [grp[g] >> 8, grp[g+1] >> 8) and column species (grp[g] & 0xFF).  A
// term is packed as: bits 0-15 reaction, 16-18 kind (0-2 reactant slot, 3-5
// product slot, 6 third-body efficiency), 19 last term of its column group,
// 20-23 and 60-63 the group's column species (low and high nibble), 24-31 nu
// (int8), 32-39 and 40-47 the two other molecules of that side (K =
// padding), 48-59 efficiency entry.
struct WgTerms {
  const int32_t* gptr;  // [K+1]
  const uint32_t* grp;  // [G+1] (sentinel at G)
  const uint64_t* term; // [T]
  // [WG][4] the term segment of thread t: first term, end, row (-1: none) and,
  // for the thread that owns a row, the thread holding the row's second
  // segment (-1: the row is not split).  Rows are split at a column group, so
  // each Sx entry comes from one segment.
  const int32_t* seg;
};

// Per-workgroup LDS workspace (beyond the staged mechanism blob); NP = N
// rounded up to a multiple of 16.
typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef double dbl2 __attribute__((ext_vector_type(2)));

struct WgWs {
  double* C;     // [NP] concentrations, C[K] = 1
  double* g;     // [NP] g/RT
  double* hR;    // [NP] h/RT
  double* rk;    // [R]
  double* rkr;   // [R]
  double* rdm;   // [R]
  double* rdt;   // [R]
  double* vec;   // [NP] state-sized exchange vector (y for thermo, b for solves)
  double* ad;    // [NP] adense_k per state row (row 1+k)
  double* gam;   // [NP]
  double* jT0;   // [NP] column 0 of J (J_iT)
  double* jTr;   // [NP] row 0 of J (J_Tj)
  double* Pn;    // [NP * 16] panel
  double* Ub;    // [16 * NP] rows of U of the panel
  double* rdg;   // [NP] 1 / U_kk
  double* red;   // [16] block reduction scratch
  int* piv;      // [NP] row interchanges of the LU
  int* perm;     // [NP] their composition (row i of P M is row perm[i] of M)
  int* flag;     // [4] flags and the queue broadcast; [4] interchange count of the panel
  int* sdst;     // [32] rows written by the panel's interchanges
  int* ssrc;     // [32] the rows they take their values from
  double* skp;   // [WG] partial sums C . S_row of the term segments
  double* tbd;   // [ntb] third-body efficiencies - 1 (a copy of the mechanism's)
};

// Doubles of the mechanism's efficiency table (as laid out in the blob).
__host__ __device__ inline int wg_ntb(const MechDims& d) { return (d.o_troe - d.o_tbd) / 8; }

// The Jacobian's rate arrays rkr, rdm, rdt and the LU's panel buffers Pn, Ub
// are never live at the same time, so they share one region.  ntb: doubles of
// the efficiency table copied to the end (0 where no Jacobian is formed).
__host__ __device__ inline int wg_ws_doubles(int R, int NP, int ntb) {
  const int shared = 2 * WNB * NP > 3 * R ? 2 * WNB * NP : 3 * R;
  return 3 * NP + R + 5 * NP + shared + NP + 16 + NP / 2 + NP / 2 + 40 + WG + ntb;
}

__device__ inline WgWs make_wg_ws(double* base, int R, int NP) {
  WgWs w;
  w.C = base;
  w.g = w.C + NP;
  w.hR = w.g + NP;
  w.rk = w.hR + NP;
  w.vec = w.rk + R;
  w.ad = w.vec + NP;
  w.gam = w.ad + NP;
  w.jT0 = w.gam + NP;
  w.jTr = w.jT0 + NP;
  double* shared = w.jTr + NP;
  w.Pn = shared;
  w.Ub = w.Pn + NP * WNB;
  w.rkr = shared;
  w.rdm = w.rkr + R;
  w.rdt = w.rdm + R;
  const int sh = 2 * WNB * NP > 3 * R ? 2 * WNB * NP : 3 * R;
  w.rdg = shared + sh;
  w.red = w.rdg + NP;
  w.piv = (int*)(w.red + 16);
  w.perm = w.piv + NP;
  w.flag = w.perm + NP;
  w.sdst = w.flag + 8;
  w.ssrc = w.sdst + 32;
  w.skp = (double*)w.piv + NP + 40;  // past the 2 NP + 72 ints above
  w.tbd = w.skp + WG;
  return w;
}

// CellWs view of the workgroup workspace for the shared rate helpers.
__device__ inline CellWs wg_cellws(const WgWs& w) {
  CellWs c{};
  c.rk = w.rk;
  c.rkr = w.rkr;
  c.rdm = w.rdm;
  c.rdt = w.rdt;
  c.C = w.C;
  c.g = w.g;
  c.hR = w.hR;
  return c;
}

// Sum over the workgroup in a fixed order (wave sums, then the four partials
// in wave order); every thread gets the result.
__device__ inline double block_sum(double v, double* red) {
  const double s = wave_sum(v);
  const int wv = threadIdx.x / WAVE;
  if ((threadIdx.x & (WAVE - 1)) == 0) red[wv] = s;
  __syncthreads();
  const double r = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return r;
}

__device__ inline bool block_any(bool p, int* flag) {
  if (threadIdx.x == 0) flag[0] = 0;
  __syncthreads();
  if (p) flag[0] = 1;  // benign race: every writer stores 1
  __syncthreads();
  const bool r = flag[0] != 0;
  __syncthreads();
  return r;
}

// Thermo and mixture of the state in w.vec; fills C, g, hR; returns the
// thread's species thermo (species k = t - 1 for 1 <= t <= K).
__device__ inline SpThermo wg_species(const MechView& m, const WgWs& w, double p, Mix& x, double& Yk) {
  const int K = m.d.K, t = threadIdx.x;
  const bool isSp = t >= 1 && t <= K;
  const int k = isSp ? t - 1 : 0;
  x.T = w.vec[0];
  x.lnT = log(x.T);
  x.iT = 1.0 / x.T;
  const SpThermo th = nasa7(m.nasa + 16 * k, x.T, x.lnT, x.iT);
  Yk = isSp ? w.vec[t] : 0.0;
  const double iWk = m.iW[k];
  const double yw = Yk * iWk;
  const double sy = block_sum(yw, w.red);
  x.Wbar = 1.0 / sy;
  x.rho = p * x.Wbar * x.iT / RU;
  x.iRho = 1.0 / x.rho;
  x.Ctot = p * x.iT / RU;
  x.lnPRT = log(PATM * x.iT / RU);
  x.cp = block_sum(isSp ? Yk * th.cpR * RU * iWk : 0.0, w.red);
  if (isSp) {
    w.C[k] = x.rho * yw;
    w.g[k] = th.hRT - th.sR;
    w.hR[k] = th.hRT;
  }
  if (t == 0) {
    w.C[K] = 1.0;
    w.g[K] = 0.0;
    w.hR[K] = 0.0;
  }
  __syncthreads();
  return th;
}

// f(y) with y_t held by thread t; returns f_t.
__device__ inline double wg_rhs(const MechView& m, const WgWs& w, double y, double p) {
  const int K = m.d.K, R = m.d.R, N = m.d.N, t = threadIdx.x;
  if (t < N) w.vec[t] = y;
  __syncthreads();
  Mix x;
  double Yk;
  const SpThermo th = wg_species(m, w, p, x, Yk);
  const CellWs cw = wg_cellws(w);
#pragma clang loop unroll(disable)
  for (int r = t; r < R; r += WG) {
    const Slots s = unpack(m.sp[r]);
    const double lnkf = m.lnA[r] + m.b[r] * x.lnT - m.th[r] * x.iT;
    const double Rf = w.C[s.r0] * w.C[s.r1] * w.C[s.r2];
    const double Rr = w.C[s.p0] * w.C[s.p1] * w.C[s.p2];
    const double sng = w.g[s.p0] + w.g[s.p1] + w.g[s.p2] - w.g[s.r0] - w.g[s.r1] - w.g[s.r2];
    const double kf = exp(lnkf);
    const double iKc = exp(sng - s.dnu * x.lnPRT);
    double q = kf * (Rf - iKc * Rr);
    if (r >= m.d.R0) {
      const double M = third_body(m, cw, r, x.Ctot);
      if (r < m.d.R1) {
        q *= M;
      } else {
        double dk, dl;
        q = troe_k<false>(m, r, x, kf, 0.0, M, dk, dl) * (Rf - iKc * Rr);
      }
    }
    w.rk[r] = q;
  }
  __syncthreads();
  const bool isSp = t >= 1 && t <= K;
  double om = 0.0;
  if (isSp) {
    // the incidence list is in global memory: eight entries per pass, loaded
    // together, then summed in list order
    const int k = t - 1, e0 = m.cptr[k], e1 = m.cptr[k + 1];
#pragma clang loop unroll(disable)
    for (int eb = e0; eb < e1; eb += 8) {
      uint32_t v8[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v8[u] = eb + u < e1 ? m.cent[eb + u] : 0u;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (eb + u >= e1) break;
        om += (double)(int8_t)(v8[u] & 0xFF) * w.rk[v8[u] >> 8];
      }
    }
  }
  const double Q = block_sum(isSp ? th.hRT * om : 0.0, w.red);
  const double fT = -RU * x.T * Q * x.iRho / x.cp;
  if (t == 0) return fT;
  return isSp ? m.W[t - 1] * om * x.iRho : 0.0;
}

// Analytic Jacobian (the same formulas as the wavefront path): the sparse
// part of d omega/dC goes to Sx at its structural positions (row 1+k, column
// 1+l), the dense row/column pieces to LDS vectors.  Returns f_t.
__device__ inline double wg_jac(const MechView& m, const WgWs& w, const WgTerms& tl, double* Sx, int NP, double y,
                                double p) {
  const int K = m.d.K, R = m.d.R, N = m.d.N, t = threadIdx.x;
  if (t < N) w.vec[t] = y;
  __syncthreads();
  Mix x;
  double Yk;
  const SpThermo th = wg_species(m, w, p, x, Yk);
  const CellWs cw = wg_cellws(w);
#pragma clang loop unroll(disable)
  for (int r = t; r < R; r += WG) {
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
      const double M = third_body(m, cw, r, x.Ctot);
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
    w.rdm[r] = dkM;
    w.rdt[r] = dqdT;
  }
  __syncthreads();
  const bool isSp = t >= 1 && t <= K;
  double om = 0.0, dwdT = 0.0, adense = 0.0, sk = 0.0;
  if (isSp) {
    const int k = t - 1, e0 = m.cptr[k], e1 = m.cptr[k + 1];
    // incidence entries and their reactions' slots come from global memory:
    // eight per pass, loaded together, then summed in list order
#pragma clang loop unroll(disable)
    for (int eb = e0; eb < e1; eb += 8) {
      uint32_t v8[8];
      uint64_t sp8[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v8[u] = eb + u < e1 ? m.cent[eb + u] : 0u;
#pragma unroll
      for (int u = 0; u < 8; ++u) sp8[u] = eb + u < e1 ? m.sp[v8[u] >> 8] : 0ull;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (eb + u >= e1) break;
        const int r = (int)(v8[u] >> 8);
        const double nu = (double)(int8_t)(v8[u] & 0xFF);
        const Slots s = unpack(sp8[u]);
        om += nu * (w.rk[r] * w.C[s.r0] * w.C[s.r1] * w.C[s.r2] - w.rkr[r] * w.C[s.p0] * w.C[s.p1] * w.C[s.p2]);
        dwdT += nu * w.rdt[r];
        if (r >= m.d.R0) adense += nu * w.rdm[r];
      }
    }
  }
  // structural nonzeros, one group per column, terms in a fixed order: thread
  // t sums its segment of a row's terms (the loader splits the longest rows
  // in two at a column group and gives the second halves to the threads that
  // own no row)
  {
    typedef int int4v __attribute__((ext_vector_type(4)));
    const int4v sg = *(const int4v*)(tl.seg + 4 * t);
    const int tb = sg[0], te = sg[1], srow = sg[2];
    double skt = 0.0;
    if (srow >= 0) {
      double* Srow = Sx + (size_t)(1 + srow) * NP + 1;
      // the last term of each column group carries the column and closes it
      double acc = 0.0;
      // software-pipelined: the next pass's term words are in flight while
      // this pass is summed; the pass itself has no branch except the column
      // store
      uint64_t nx[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) nx[u] = tb + u < te ? tl.term[tb + u] : 0ull;
#pragma clang loop unroll(disable)
      for (int ti = tb; ti < te; ti += 8) {
        uint64_t tw8[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          tw8[u] = nx[u];
          nx[u] = ti + 8 + u < te ? tl.term[ti + 8 + u] : 0ull;
        }
        // the efficiencies of third-body terms (from the LDS copy)
        double ef8[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
          ef8[u] = (ti + u < te && ((tw8[u] >> 16) & 7) == 6) ? w.tbd[(tw8[u] >> 48) & 0xFFF] : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const bool in = ti + u < te;  // past the segment's end the word is 0: indices 0, no store
          const uint64_t tw = tw8[u];
          const int r = (int)(tw & 0xFFFF);
          const int kind = (int)((tw >> 16) & 7);
          const double nu = (double)(int8_t)((tw >> 24) & 0xFF);
          const double co = w.C[(tw >> 32) & 0xFF] * w.C[(tw >> 40) & 0xFF];
          // one rate load per term: the array is picked by the kind
          const double rv = (kind < 3 ? w.rk : (kind < 6 ? w.rkr : w.rdm))[r];
          const double v = (kind >= 3 && kind < 6 ? -rv : rv) * (kind < 6 ? co : ef8[u]);
          const double an = acc + nu * v;
          acc = in ? an : acc;
          if (in && ((tw >> 19) & 1)) {
            const int col = (int)(((tw >> 20) & 0xF) | (((tw >> 60) & 0xF) << 4));
            Srow[col] = acc;
            skt += w.C[col] * acc;
            acc = 0.0;
          }
        }
      }
    }
    w.skp[t] = skt;
    __syncthreads();
    // a split row's two partial sums, first segment first
    if (isSp) sk = sg[3] >= 0 ? w.skp[t] + w.skp[sg[3]] : w.skp[t];
  }
  // sk = sum_l C_l (S_kl + adense_k); C sums to Ctot
  if (isSp) {
    double csum = 0.0;
    for (int l = 0; l < K; ++l) csum += w.C[l];  // same order on every thread
    sk += adense * csum;
  }
  double fk = 0.0, gam = 0.0, hmW = 0.0, jkT = 0.0;
  if (isSp) {
    const int k = t - 1;
    const double Wk = m.W[k];
    gam = Wk * x.Wbar * x.iRho * (om - sk);
    jkT = Wk * x.iRho * (dwdT - sk * x.iT + om * x.iT);
    fk = Wk * om * x.iRho;
    hmW = RU * x.T * th.hRT;  // mass enthalpy times W_k
  }
  if (t < NP) {
    w.ad[t] = isSp ? adense : 0.0;
    w.gam[t] = gam;
    w.jT0[t] = jkT;
  }
  const double Q = block_sum(isSp ? th.hRT * om : 0.0, w.red);
  const double fT = -RU * x.T * Q * x.iRho / x.cp;
  const double cpm = isSp ? RU * th.cpR * m.iW[t - 1] : 0.0;
  const double s1 = block_sum(cpm * fk, w.red);
  const double dcpdT = block_sum(isSp ? Yk * RU * th.dcpR * m.iW[t - 1] : 0.0, w.red);
  const double sA = block_sum(hmW * adense, w.red);
  const double sG = block_sum(isSp ? hmW * m.iW[t - 1] * gam : 0.0, w.red);
  const double sT = block_sum(isSp ? hmW * m.iW[t - 1] * jkT : 0.0, w.red);
  // Sx rows are complete (the block sums above synchronised the workgroup)
  __threadfence_block();
  __syncthreads();
  // row 0 of J: column sums of the species rows weighted by mass enthalpy
  if (isSp) {
    const int l = t - 1;
    const double* Sc = Sx + NP + 1 + l;
    const double RT = RU * x.T;
    double ps[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int k = 0;
#pragma clang loop unroll(disable)
    for (; k + 8 <= K; k += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = Sc[(size_t)(k + u) * NP];
#pragma unroll
      for (int u = 0; u < 8; ++u) ps[u] = fma(RT * w.hR[k + u], v[u], ps[u]);
    }
    for (; k < K; ++k) ps[0] = fma(RT * w.hR[k], Sc[(size_t)k * NP], ps[0]);
    const double cs = ((ps[0] + ps[1]) + (ps[2] + ps[3])) + ((ps[4] + ps[5]) + (ps[6] + ps[7]));
    const double colsum = m.iW[l] * (cs + sA + sG);
    w.jTr[t] = -(colsum + fT * cpm) / x.cp;
  } else if (t == 0) {
    w.jTr[0] = -(sT + s1 + fT * dcpdT) / x.cp;
  }
  __syncthreads();
  return t == 0 ? fT : fk;
}

// M = I/(gamma h) - J into Mx (NP x NP, identity on the padding); returns
// false if an entry is not finite.
__device__ inline bool wg_form(const MechView& m, const WgWs& w, const double* Sx, double* Mx, int NP, double d) {
  const int N = m.d.N, tot = NP * NP;
  // Thread t forms the element pairs (idx, idx + 1), idx = 2t + 2 WG u (NP is
  // even, so a pair never leaves its row).  Row and column follow idx by
  // additions; eight pairs per pass have their scratch loads in flight
  // together.
  constexpr int STEP = 2 * WG;
  const int di = STEP / NP, dj = STEP - di * NP;
  int i = (2 * (int)threadIdx.x) / NP, j = 2 * (int)threadIdx.x - i * NP;
  bool bad = false;
#pragma clang loop unroll(disable)
  for (int base = 2 * (int)threadIdx.x; base < tot; base += 8 * STEP) {
    dbl2 sv[8];
    int ri[8], cj[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = base + u * STEP;
      ri[u] = i;
      cj[u] = j;
      sv[u] = idx < tot ? *(const dbl2*)(Sx + idx) : dbl2{0.0, 0.0};
      j += dj;
      i += di;
      if (j >= NP) {
        j -= NP;
        ++i;
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = base + u * STEP;
      if (idx >= tot) break;
      const int r = ri[u];
      double v[2];
      const double sr[2] = {sv[u][0], sv[u][1]};
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int c = cj[u] + e;
        if (r >= N || c >= N) {
          v[e] = r == c ? 1.0 : 0.0;
        } else {
          double J;
          if (r == 0) J = w.jTr[c];
          else if (c == 0) J = w.jT0[r];
          else J = m.iW[c - 1] * (m.W[r - 1] * (sr[e] + w.ad[r]) + w.gam[r]);
          v[e] = (r == c ? d : 0.0) - J;
          bad |= !__builtin_isfinite(v[e]);
        }
      }
      *(dbl2*)(Mx + idx) = dbl2{v[0], v[1]};
    }
  }
  return !block_any(bad, w.flag + 1);
}

// Factors the panel (rows p0..NP-1, columns p0..p0+15, staged in Pn) in the
// registers of wave 0: relative row r sits in lane r % 64, slot r / 64.  The
// pivot is the first row with the largest |a| (exact comparison of the
// non-negative doubles as integers, then the smallest row index); the pivot
// row is broadcast with readlane and swapped into row kk.  Records piv, 1/U_kk
// and a zero-pivot step in flag[2]; leaves the factored panel in Pn.
template <int NS>
__device__ inline void wg_panel(const WgWs& w, int p0, int NP, int lane) {
  const int nrow = NP - p0;
  double P[NS][WNB];
#pragma unroll
  for (int sl = 0; sl < NS; ++sl) {
    const int rel = sl * WAVE + lane;
#pragma unroll
    for (int c = 0; c < WNB; ++c) P[sl][c] = rel < nrow ? w.Pn[rel * WNB + c] : 0.0;
  }
#pragma clang loop unroll(full)
  for (int kk = 0; kk < WNB; ++kk) {
    double best = -1.0;
    int brel = 1 << 20;
#pragma unroll
    for (int sl = 0; sl < NS; ++sl) {
      const int rel = sl * WAVE + lane;
      const double v = fabs(P[sl][kk]);
      if (rel >= kk && rel < nrow && v > best) {
        best = v;
        brel = rel;
      }
    }
    const unsigned long long key = __builtin_bit_cast(unsigned long long, best < 0.0 ? 0.0 : best);
    const unsigned hi = (unsigned)(key >> 32), lo = (unsigned)key;
    const unsigned mh = wave_max_u32(best < 0.0 ? 0u : hi);
    // the low halves decide only between lanes that tie on the high half
    const bool top = best >= 0.0 && hi == mh;
    bool holder = top;
    if (__builtin_popcountll(ballot(top)) > 1) {
      const unsigned ml = wave_max_u32(top ? lo : 0u);
      holder = top && lo == ml;
    }
    // first row holding the maximum: the lowest slot with a holder, then the
    // lowest lane in it (one ballot per slot)
    int pr = kk;
#pragma unroll
    for (int sl = NS - 1; sl >= 0; --sl) {
      const unsigned long long bm = ballot(holder && brel / WAVE == sl);
      if (bm) pr = sl * WAVE + (int)__builtin_ctzll(bm);
    }
    pr = pr < nrow ? pr : kk;
    const int lp = pr & (WAVE - 1), sp = pr / WAVE;
    // the pivot row's slot is wave-uniform: a scalar branch picks it.  The
    // update needs columns kk.. of the pivot row; the columns left of kk only
    // move with a row interchange, so they are broadcast only then.
    double b[WNB];
#pragma unroll
    for (int sl = 0; sl < NS; ++sl) {
      if (sp == sl) {
#pragma unroll
        for (int c = kk; c < WNB; ++c) b[c] = readlane(P[sl][c], lp);
      }
    }
    const double pv = b[kk];
    const bool sing = !(pv != 0.0);
    if (!sing && pr != kk) {
#pragma unroll
      for (int sl = 0; sl < NS; ++sl) {
        if (sp == sl) {
#pragma unroll
          for (int c = 0; c < kk; ++c) b[c] = readlane(P[sl][c], lp);
        }
      }
#pragma unroll
      for (int c = 0; c < WNB; ++c) {
        const double a = readlane(P[0][c], kk);
#pragma unroll
        for (int sl = 0; sl < NS; ++sl) P[sl][c] = (lane == lp && sp == sl) ? a : P[sl][c];
        P[0][c] = lane == kk ? b[c] : P[0][c];
      }
    }
    const double rp = sing ? 0.0 : recip(pv);
    if (lane == 0) {
      w.piv[p0 + kk] = (sing ? kk : pr) + p0;
      w.rdg[p0 + kk] = rp;
      if (sing && w.flag[2] == 0) w.flag[2] = p0 + kk + 1;
    }
#pragma unroll
    for (int sl = 0; sl < NS; ++sl) {
      const int rel = sl * WAVE + lane;
      if (rel > kk && rel < nrow) {
        const double l = P[sl][kk] * rp;
        P[sl][kk] = l;
#pragma clang loop unroll(full)
        for (int c = kk + 1; c < WNB; ++c) P[sl][c] = fma(-l, b[c], P[sl][c]);
      }
    }
  }
#pragma unroll
  for (int sl = 0; sl < NS; ++sl) {
    const int rel = sl * WAVE + lane;
    if (rel < nrow) {
#pragma unroll
      for (int c = 0; c < WNB; ++c) w.Pn[rel * WNB + c] = P[sl][c];
    }
  }
  wsync();
}

// Panel factorization in LDS by wave 0 (any panel height; used above 192 rows,
// where the register version would not fit).  Same pivot rule and records.
__device__ inline void wg_panel_lds(const WgWs& w, int p0, int NP, int lane) {
#pragma clang loop unroll(disable)
  for (int kk = 0; kk < WNB; ++kk) {
    const int k = p0 + kk;
    double best = -1.0;
    int bi = NP;
    for (int i = k + lane; i < NP; i += WAVE) {
      const double v = fabs(w.Pn[(i - p0) * WNB + kk]);
      if (v > best) {
        best = v;
        bi = i;
      }
    }
    const unsigned long long key = __builtin_bit_cast(unsigned long long, best < 0.0 ? 0.0 : best);
    const unsigned hi = (unsigned)(key >> 32), lo = (unsigned)key;
    const unsigned mh = wave_max_u32(best < 0.0 ? 0u : hi);
    const unsigned ml = wave_max_u32((best >= 0.0 && hi == mh) ? lo : 0u);
    int cand = (best >= 0.0 && hi == mh && lo == ml) ? bi : NP;
    for (int o = 32; o >= 1; o >>= 1) cand = min(cand, __shfl_xor(cand, o));
    const int pr = uniform_int(cand);
    const double pv = (pr < NP) ? w.Pn[(pr - p0) * WNB + kk] : 0.0;
    const bool sing = !(pv != 0.0);
    if (lane == 0) {
      w.piv[k] = sing ? k : pr;
      if (sing && w.flag[2] == 0) w.flag[2] = k + 1;
    }
    const int prow = sing ? k : pr;
    if (lane < WNB && prow != k) {
      const double a = w.Pn[(k - p0) * WNB + lane], b = w.Pn[(prow - p0) * WNB + lane];
      w.Pn[(k - p0) * WNB + lane] = b;
      w.Pn[(prow - p0) * WNB + lane] = a;
    }
    wsync();
    const double rp = sing ? 0.0 : 1.0 / pv;
    if (lane == 0) w.rdg[k] = rp;
    for (int i = k + 1 + lane; i < NP; i += WAVE) {
      double* Pr = w.Pn + (i - p0) * WNB;
      const double l = Pr[kk] * rp;
      Pr[kk] = l;
      for (int c = kk + 1; c < WNB; ++c) Pr[c] = fma(-l, w.Pn[(k - p0) * WNB + c], Pr[c]);
    }
    wsync();
  }
}

// Blocked LU with partial pivoting of Mx in place.  Returns the 1-based step
// of a zero pivot column, or 0.  Leaves piv, perm and 1/U_kk in LDS.
template <bool PROF = false>
__device__ inline int wg_lu(const WgWs& w, double* Mx, int NP, Prof<PROF>* pf = nullptr) {
  const int t = threadIdx.x, lane = t & (WAVE - 1), wv = t / WAVE;
  unsigned long long tp = 0;
  if (t == 0) w.flag[2] = 0;
#pragma clang loop unroll(disable)
  for (int p0 = 0; p0 < NP; p0 += WNB) {
    const int nrow = NP - p0;
    // panel to LDS
    {
      double pv[WNB];
#pragma unroll
      for (int u = 0; u < WNB; ++u) {
        const int idx = t + u * WG;
        pv[u] = idx < nrow * WNB ? Mx[(size_t)(p0 + idx / WNB) * NP + p0 + (idx % WNB)] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < WNB; ++u) {
        const int idx = t + u * WG;
        if (idx < nrow * WNB) w.Pn[idx] = pv[u];
      }
    }
    __syncthreads();
    if (PROF) tp = pf->now();
    if (wv == 0) {
      // as many 64-row register slots as the panel has rows
      if (nrow <= WAVE) wg_panel<1>(w, p0, NP, lane);
      else if (nrow <= 2 * WAVE) wg_panel<2>(w, p0, NP, lane);
      else if (nrow <= 3 * WAVE) wg_panel<3>(w, p0, NP, lane);
      else wg_panel_lds(w, p0, NP, lane);
      // the panel's 16 interchanges composed on the rows they touch (at most
      // 32, one per lane): afterwards row sdst[i] holds old row ssrc[i]
      int myrow = -1, mysrc = -1, nt = 0;
#pragma clang loop unroll(disable)
      for (int kk = 0; kk < WNB; ++kk) {
        const int k = p0 + kk, q = w.piv[k];
        if (q == k) continue;
        const unsigned long long bk = ballot(myrow == k);
        int sk = nt;
        if (bk) sk = (int)__builtin_ctzll(bk);
        else {
          if (lane == nt) myrow = mysrc = k;
          ++nt;
        }
        const unsigned long long bq = ballot(myrow == q);
        int sq = nt;
        if (bq) sq = (int)__builtin_ctzll(bq);
        else {
          if (lane == nt) myrow = mysrc = q;
          ++nt;
        }
        const int srck = __builtin_amdgcn_readlane(mysrc, sk), srcq = __builtin_amdgcn_readlane(mysrc, sq);
        if (lane == sk) mysrc = srcq;
        if (lane == sq) mysrc = srck;
      }
      if (lane < nt) {
        w.sdst[lane] = myrow;
        w.ssrc[lane] = mysrc;
      }
      if (lane == 0) w.flag[4] = nt;
    }
    __syncthreads();
    if (PROF) {
      pf->add(6, tp);
      tp = pf->now();
    }
    // row interchanges on the columns outside the panel: each thread owns a
    // column, loads every source row first, then stores
    const int nsw = w.flag[4];
#pragma clang loop unroll(disable)
    for (int j = t; j < NP; j += WG) {
      if (j >= p0 && j < p0 + WNB) continue;
      double v[2 * WNB];
#pragma unroll
      for (int i = 0; i < 2 * WNB; ++i) v[i] = i < nsw ? Mx[(size_t)w.ssrc[i] * NP + j] : 0.0;
#pragma unroll
      for (int i = 0; i < 2 * WNB; ++i)
        if (i < nsw) Mx[(size_t)w.sdst[i] * NP + j] = v[i];
      // rows of U of this panel: U12 = L11^-1 A12 (column j, forward substitution)
      if (j >= p0 + WNB) {
        double u[WNB];
#pragma unroll
        for (int r = 0; r < WNB; ++r) u[r] = Mx[(size_t)(p0 + r) * NP + j];
#pragma unroll
        for (int r = 1; r < WNB; ++r) {
#pragma unroll
          for (int c = 0; c < r; ++c) u[r] = fma(-w.Pn[r * WNB + c], u[c], u[r]);
        }
#pragma unroll
        for (int r = 0; r < WNB; ++r) {
          w.Ub[r * NP + j] = u[r];
          Mx[(size_t)(p0 + r) * NP + j] = u[r];
        }
      }
    }
    // factored panel back to Mx
#pragma clang loop unroll(disable)
    for (int idx = t; idx < nrow * WNB; idx += WG) Mx[(size_t)(p0 + idx / WNB) * NP + p0 + (idx % WNB)] = w.Pn[idx];
    __syncthreads();
    if (PROF) pf->add(7, tp);
    // trailing update A22 -= L21 U12 on FP64 MFMA (v_mfma_f64_16x16x4f64):
    // 16 x 16 output tiles; wave wv takes tile rows wv, wv + 4, ... and keeps
    // the row's L21 operand (16 x 16, negated) in registers across its tile
    // columns, two of which are in flight.  Lane layouts of the instruction:
    // lane l holds A[l % 16][l / 16], B[l / 16][l % 16] and D[l / 16 + 4 v][l % 16].
    const int m0 = p0 + WNB, nt = (NP - m0) / 16;
    const int li = lane & 15, lk = lane >> 4;
#pragma clang loop unroll(disable)
    for (int bi = uniform_int(wv); bi < nt; bi += WG / WAVE) {
      const int i0 = m0 + 16 * bi;
      double am[4];
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) am[s4] = -w.Pn[(i0 - p0 + li) * WNB + 4 * s4 + lk];
      double* rowp = Mx + (size_t)(i0 + lk) * NP + m0 + li;
      const double* ub = w.Ub + (size_t)lk * NP + m0 + li;
#pragma clang loop unroll(disable)
      for (int bj = 0; bj < nt; bj += 2) {
        const bool two = bj + 1 < nt;
        double* r0 = rowp + 16 * bj;
        const double* u0 = ub + 16 * bj;
        dbl4 c0, c1;
#pragma unroll
        for (int v = 0; v < 4; ++v) c0[v] = r0[(size_t)4 * v * NP];
        if (two) {
#pragma unroll
          for (int v = 0; v < 4; ++v) c1[v] = r0[(size_t)4 * v * NP + 16];
        }
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(am[s4], u0[(size_t)4 * s4 * NP], c0, 0, 0, 0);
          if (two) c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(am[s4], u0[(size_t)4 * s4 * NP + 16], c1, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) r0[(size_t)4 * v * NP] = c0[v];
        if (two) {
#pragma unroll
          for (int v = 0; v < 4; ++v) r0[(size_t)4 * v * NP + 16] = c1[v];
        }
      }
    }
    __syncthreads();
  }
  // composition of the interchanges: row i of P M is row perm[i] of M.
  // Thread i follows its row back through the interchanges, last first.
  if (t < NP) {
    int pos = t;
#pragma clang loop unroll(disable)
    for (int k0 = NP - WNB; k0 >= 0; k0 -= WNB) {
      int q[WNB];
#pragma unroll
      for (int u = 0; u < WNB; ++u) q[u] = w.piv[k0 + u];
#pragma unroll
      for (int u = WNB - 1; u >= 0; --u) pos = pos == k0 + u ? q[u] : (pos == q[u] ? k0 + u : pos);
    }
    w.perm[t] = pos;
  }
  __syncthreads();
  const int info = w.flag[2];
  __syncthreads();
  return info;
}

// Solve M x = b with the factors in Mx; thread t holds b_t and gets x_t.
// Thread t also owns row t of the factors: at each 16-column block it holds
// that block's 16 entries of its row in registers and has the next block's
// entries in flight, so the global-memory latency is paid once per solve.  The
// 16 x 16 diagonal block is solved by the wave that owns its rows (rows
// p0..p0+15 are 16 consecutive lanes of one wave).
__device__ inline double wg_solve(const WgWs& w, const double* Mx, int NP, double b) {
  const int t = threadIdx.x, wv = t / WAVE;
  const double* Mrow = Mx + (size_t)(t < NP ? t : 0) * NP;
  double seg[WNB], nxt[WNB];
  // first forward block (columns 0..15) in flight while b is permuted
#pragma unroll
  for (int c = 0; c < WNB; ++c) nxt[c] = t < NP ? Mrow[c] : 0.0;
  if (t < NP) w.vec[t] = b;
  __syncthreads();
  double y = t < NP ? w.vec[w.perm[t]] : 0.0;
  __syncthreads();
  // forward substitution with unit-lower L
#pragma clang loop unroll(disable)
  for (int p0 = 0; p0 < NP; p0 += WNB) {
#pragma unroll
    for (int c = 0; c < WNB; ++c) seg[c] = nxt[c];
    const int pn = p0 + WNB;
    if (pn < NP && t >= pn) {
#pragma unroll
      for (int c = 0; c < WNB; ++c) nxt[c] = Mrow[pn + c];
    }
    if (wv == p0 / WAVE) {  // diagonal block: lanes l0 .. l0+15 of this wave
      const int l0 = p0 & (WAVE - 1);
      const bool inb = t >= p0 && t < pn;
#pragma unroll
      for (int c = 0; c < WNB - 1; ++c) {
        const double yc = readlane(y, l0 + c);
        y = fma((inb && t > p0 + c) ? -seg[c] : -0.0, yc, y);  // mask off the chain
      }
      if (inb) w.vec[t] = y;
    }
    __syncthreads();
    // no barrier after this update: the next block's diagonal wave writes
    // other entries of vec, and it updates its own rows here first
    if (t >= pn && t < NP) {
#pragma unroll
      for (int c = 0; c < WNB; ++c) y = fma(-seg[c], w.vec[p0 + c], y);
    }
  }
  // back substitution with U, last block first
  const int last = NP - WNB;
#pragma unroll
  for (int c = 0; c < WNB; ++c) nxt[c] = t < NP ? Mrow[last + c] : 0.0;
#pragma clang loop unroll(disable)
  for (int p0 = last; p0 >= 0; p0 -= WNB) {
#pragma unroll
    for (int c = 0; c < WNB; ++c) seg[c] = nxt[c];
    const int pp = p0 - WNB;
    if (pp >= 0 && t < p0) {
#pragma unroll
      for (int c = 0; c < WNB; ++c) nxt[c] = Mrow[pp + c];
    }
    if (wv == p0 / WAVE) {
      const int l0 = p0 & (WAVE - 1);
      const bool inb = t >= p0 && t < p0 + WNB;
      const double rd = inb ? w.rdg[t] : 0.0;
#pragma unroll
      for (int c = WNB - 1; c >= 0; --c) {
        const double xc = readlane(y * rd, l0 + c);
        y = fma((inb && t < p0 + c) ? -seg[c] : -0.0, xc, y);
      }
      if (inb) {
        y *= rd;
        w.vec[t] = y;
      }
    }
    __syncthreads();
    if (t < p0) {
#pragma unroll
      for (int c = 0; c < WNB; ++c) y = fma(-seg[c], w.vec[p0 + c], y);
    }
  }
  return t < NP ? y : 0.0;
}

}  // namespace chem

namespace chem {

// One Rosenbrock attempt of the workgroup path (the same stage recurrence as
// the wavefront path).  Returns 0, 1 (singular M) or 2 (non-finite M).
template <bool PROF>
__device__ inline int wg_attempt(const MechView& m, const WgWs& w, const double* Sx, double* Mx, int NP,
                                 const RosTable& tab, double p, double y, double f0, double h, double& ynew,
                                 double& err, Prof<PROF>& pf) {
  const int N = m.d.N, t = threadIdx.x;
  pf.start();
  const bool okm = wg_form(m, w, Sx, Mx, NP, 1.0 / (tab.gamma * h));
  pf.stop(1);
  if (!okm) return 2;
  const int info = wg_lu<PROF>(w, Mx, NP, &pf);
  pf.stop(2);
  if (info) return 1;
  const double ih = 1.0 / h;
  const int s = tab.s;
  double K0 = 0.0, K1 = 0.0, K2 = 0.0, K3 = 0.0;
  double fi = f0;
#pragma clang loop unroll(disable)
  for (int i = 0; i < s; ++i) {
    const double a0 = i >= 1 ? tab.a[i][i - 1] : 0.0, c0 = i >= 1 ? tab.c[i][i - 1] : 0.0;
    const double a1 = i >= 2 ? tab.a[i][i - 2] : 0.0, c1 = i >= 2 ? tab.c[i][i - 2] : 0.0;
    const double a2 = i >= 3 ? tab.a[i][i - 3] : 0.0, c2 = i >= 3 ? tab.c[i][i - 3] : 0.0;
    if (i > 0 && tab.newf[i]) {
      const double Yi = y + a0 * K0 + a1 * K1 + a2 * K2;
      pf.start();
      fi = wg_rhs(m, w, t < N ? Yi : 0.0, p);
      pf.stop(3);
    }
    const double r = fi + ih * (c0 * K0 + c1 * K1 + c2 * K2);
    pf.start();
    const double ki = wg_solve(w, Mx, NP, t < N ? r : 0.0);
    pf.stop(4);
    K3 = K2;
    K2 = K1;
    K1 = K0;
    K0 = ki;
  }
  const double m0 = tab.m[s - 1], e0 = tab.e[s - 1];
  const double m1 = s >= 2 ? tab.m[s - 2] : 0.0, e1 = s >= 2 ? tab.e[s - 2] : 0.0;
  const double m2 = s >= 3 ? tab.m[s - 3] : 0.0, e2 = s >= 3 ? tab.e[s - 3] : 0.0;
  const double m3 = s >= 4 ? tab.m[s - 4] : 0.0, e3 = s >= 4 ? tab.e[s - 4] : 0.0;
  ynew = y + (m0 * K0 + m1 * K1 + m2 * K2 + m3 * K3);
  err = e0 * K0 + e1 * K1 + e2 * K2 + e3 * K3;
  return 0;
}

// Adaptive integration of cell c over [0, dt] by the whole workgroup, with the
// controller of the wavefront path.  Every control value is computed
// identically by all threads (from workgroup sums), so branches are uniform.
template <bool PROF>
__device__ inline void wg_integrate_cell(const MechView& m, const WgWs& w, const WgTerms& tl, double* Sx, double* Mx,
                                         int NP, const IntArgs& a, int64_t c) {
  const int t = threadIdx.x, N = m.d.N;
  Prof<PROF> pf;
  const unsigned long long t_begin = PROF ? __builtin_readcyclecounter() : 0ull;
  double y = t < N ? a.state[(int64_t)t * a.ld + c] : 0.0;
  const double dt = a.dt;
  const double hin = a.h[c];
  double hprop = (__builtin_isfinite(hin) && hin > 0.0) ? fmin(hin, dt) : dt;
  int status = ST_OK, steps = 0, rejects = 0, attempts = 0;
  const bool bad = t < N && (!__builtin_isfinite(y) || (t == 0 && !(y > 0.0)));
  if (block_any(bad, w.flag + 1)) status = ST_NONFINITE;
  double tt = 0.0;
  bool rej_last = false;
  const RosTable& tab = kTables[a.method];
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
      double h = hprop;
      bool clipped = false;
      if (h >= dt - tt) { h = dt - tt; clipped = true; }
      ++attempts;
      if (fresh && block_any(t < N && !__builtin_isfinite(f0), w.flag + 1)) { status = ST_NONFINITE; break; }
      double ynew, err;
      int rc = wg_attempt<PROF>(m, w, Sx, Mx, NP, tab, a.p, y, f0, h, ynew, err, pf);
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
      if (t < N) {
        const double sc = a.atol + a.rtol * fmax(fabs(y), fabs(ynew));
        e = err / sc;
      }
      const double en = sqrt(block_sum(e * e, w.red) / N);
      const bool fin = __builtin_isfinite(en) && !block_any(t < N && !__builtin_isfinite(ynew), w.flag + 1);
      if (!fin) {
        ++rejects;
        hprop = a.ctl.fac_min * h;
        rej_last = true;
        continue;
      }
      const double fac = fmin(a.ctl.fac_max, fmax(a.ctl.fac_min, a.ctl.fac_safe * pow(en, -1.0 / a.q)));
      if (en <= 1.0) {
        accepted = true;
        ++steps;
        tt = clipped ? dt : tt + h;
        y = ynew;
        double hn = h * fac;
        if (rej_last) hn = fmin(hn, h);
        if (clipped) hn = fmax(hn, hprop);
        hprop = hn;
        rej_last = false;
      } else {
        ++rejects;
        hprop = h * fac;
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
  if (PROF && t < 8) {
    unsigned long long v = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i)
      if (t == i) v = pf.c[i];
    if (t == 5) v = __builtin_readcyclecounter() - t_begin;
    a.prof[c * 8 + t] = v;
  }
  __syncthreads();
}

}  // namespace chem
