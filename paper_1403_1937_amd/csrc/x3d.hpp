// x3d.hpp -- passes along the contiguous axis of the 3D solve.
//   X_GHAT  kernel table lines (nega-cyclic extension), forward real FFT;
//           also reduces f into the reference forcing and publishes it
//   X_PHI0  phi_0 from the sources (eq. phi_0Solution), first forcing term,
//           forward real FFT
//   X_TERM  term `term` < T: inverse real FFT, rescale, store the term; then
//           the next forcing term and its FFT
//   X_LAST  term T: inverse real FFT, the float64 sum of all terms and
//           S = -hbar ln phi
//   X_ADJ0  adjoint start: lambda = -hbar dL/dS / phi, a_T = (-1)^T lambda,
//           forward real FFT (gamma formed from f again)
//   X_ADJ   adjoint step `term` = i: inverse real FFT of b_i = kappa (*) a_i,
//           dL/dgamma += phi_{i-1} b_i, a_{i-1} = (-1)^(i-1) lambda + gamma
//           b_i and its FFT; at i = 1, dL/df = dL/dgamma 2 f / ftilde^2
//   X_DGHAT  the kernel's beta-derivative table lines, forward real FFT
//            (scalars from the checkpoint)
//   X_ADJ0_B, X_ADJ_B  X_ADJ0 and X_ADJ for the full gradient: also the
//            per-work-group partial sums of the scalar derivatives (slots
//            G_*), X_ADJ_B from the second spectrum c_i = dkappa/dbeta (*) a_i
//   X_ETAB   phi_0 by FFT: table lines of exp(-beta |m|), forward real FFT
//   X_SEED   phi_0 by FFT: forward real FFT of the source grid (held in gamma)
//   X_PHI0F  X_PHI0 with phi_0 the inverse real FFT of the convolved source
//            grid instead of the sum over the sources
#pragma once

#include "common3d.hpp"

namespace sweik {

// Odd-frequency real transform of a line of M = 2H real samples held by a
// team as u(m) = x(2m) + i x(2m+1), m = t + P j.  With w(q) = exp(-2 pi i q /
// 2M) (the LDS table holds the even ones, we[m] = w(2m) for m < H; an odd one
// is w(2k+1) = we[k] w(1)):
//   forward  U = FFT_H(u(m) w(2m));  X(k) = E(k) + w(2k+1) O(k) with
//            2E = U(k) + conj U(H-1-k), 2iO = U(k) - conj U(H-1-k)
//            -> returns 2 X(k) = sum_j x(j) exp(-2 pi i j (k + 1/2) / M)
//   inverse  the same steps backwards; returns 2M times the real line.
template <typename R, int H>
__device__ __forceinline__ void odd_r2c(cplx<R> (&v)[16], int t, cplx<R> *line,
                                        const cplx<R> *twl, const cplx<R> *tws, cplx<R> w1) {
  using C = cplx<R>;
  constexpr int P = H / 16;
#pragma unroll
  for (int j = 0; j < 16; ++j) v[j] = cmul(v[j], twl[t + P * j]);
  team_fft<H, false>(v, t, line, tws, true);
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 16; ++j) line[lpad(t + P * j)] = v[j];
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int k = t + P * j;
    const C up = cconj(line[lpad(H - 1 - k)]);
    const C e = cadd(v[j], up);
    const C d = csub(v[j], up);
    const C o = cmake<C>(d.y, -d.x);  // -i d = 2 O
    v[j] = cadd(e, cmul(o, cmul(twl[k], w1)));
  }
}

template <typename R, int H>
__device__ __forceinline__ void odd_c2r(cplx<R> (&v)[16], int t, cplx<R> *line,
                                        const cplx<R> *twl, const cplx<R> *tws, cplx<R> w1) {
  using C = cplx<R>;
  constexpr int P = H / 16;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 16; ++j) line[lpad(t + P * j)] = v[j];
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int k = t + P * j;
    const C xp = cconj(line[lpad(H - 1 - k)]);
    const C e = cadd(v[j], xp);                         // 2E
    const C o = cmulc(csub(v[j], xp), cmul(twl[k], w1));  // 2O
    v[j] = cmake<C>(e.x - o.y, e.y + o.x);              // 2(E + iO)
  }
  team_fft<H, true>(v, t, line, tws, true);
#pragma unroll
  for (int j = 0; j < 16; ++j) v[j] = cmulc(v[j], twl[t + P * j]);
}

// FULL: every line of the group exists and n2 == H2 (no bounds checks).
template <typename R, int MODE, int H, bool FULL>
__device__ __forceinline__ void x_pass(const Args3<R> &a, int term, unsigned char *smem_raw,
                                       const int bid) {
  using C = cplx<R>;
  constexpr int P = H / 16, LPW = x_lpw(H), LL = x_line_len<R>(H);
  constexpr int TWLOG = ilog2c(4 * H);
  constexpr int NTW = (H + kThreads - 1) / kThreads;
  C *twl = reinterpret_cast<C *>(smem_raw);  // exp(-2 pi i 2m / 4H), m < H
  C *tws = twl + H;                          // stage tables of the length-H FFT
  C *lines = tws + stage_tw_len(H, 16);
  __shared__ double s_par[1];

  const int tid = threadIdx.x, team = tid / P, t = tid - team * P;
  const int r = bid * LPW + team;  // line index i0 n1 + i1
  const bool line_ok = FULL || r < a.nlines;
  const int rs = line_ok ? r : 0;
  const int i0 = rs / a.n1, i1 = rs - i0 * a.n1;
  C *line = lines + team * LL;
  const size_t rowoff = (size_t)rs * a.n2;
  constexpr bool TERMLIKE = MODE == X_TERM || MODE == X_LAST;
  constexpr bool PHI0 = MODE == X_PHI0 || MODE == X_PHI0F;
  constexpr bool ADJ0 = MODE == X_ADJ0 || MODE == X_ADJ0_B;
  constexpr bool ADJ = MODE == X_ADJ || MODE == X_ADJ_B;
  constexpr bool FULLG = MODE == X_ADJ0_B || MODE == X_ADJ_B;  // full gradient
  constexpr bool TABLE = MODE == X_GHAT || MODE == X_DGHAT || MODE == X_ETAB;
  const bool last = MODE == X_LAST || (PHI0 && a.T == 0);
  auto col_ok = [&](int c) { return FULL ? true : (line_ok && c < a.n2); };
  const bool vec = FULL || (a.n2 & 1) == 0;  // column pairs aligned: vector access

  // ---- 1. issue the global reads ---------------------------------------------
  C twr[NTW];
#pragma unroll
  for (int u = 0; u < NTW; ++u) {
    const int k = tid + u * kThreads;
    twr[u] = a.tw[(2 * min(k, H - 1)) << (a.lmax_log - TWLOG)];  // stored only if k < H
  }
  constexpr int NSR = (stage_tw_len(H, 16) + kThreads - 1) / kThreads;
  C tsr[NSR > 0 ? NSR : 1];
  stage_tw_issue<H, 16>(tsr, a.tw, a.lmax_log, tid, kThreads);
  const C w1 = a.tw[1 << (a.lmax_log - TWLOG)];  // w(1) = exp(-2 pi i / 4H)
  C v[16];
  if constexpr (TERMLIKE || ADJ || MODE == X_PHI0F) {
    const C *sl = a.s1 + (size_t)rs * H;
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = line_ok ? sl[t + P * j] : cmake<C>((R)0, (R)0);
  }
  // full gradient: the spectrum of c_i = dkappa/dbeta (*) a_i
  C vc[MODE == X_ADJ_B ? 16 : 1];
  if constexpr (MODE == X_ADJ_B) {
    const C *sl = a.s1b + (size_t)rs * H;
#pragma unroll
    for (int j = 0; j < 16; ++j) vc[j] = line_ok ? sl[t + P * j] : cmake<C>((R)0, (R)0);
  }
  // pointwise operands of columns c = 2m, 2m+1, m = t + P j (only j < 8
  // can lie in the grid since n2 <= H)
  R o1[16];
  double od[16];
  if constexpr (TERMLIKE || PHI0 || MODE == X_SEED) {
    // f (phi_0), gamma (terms) or the source grid (held in gamma)
    const R *p1 = last ? nullptr : (PHI0 ? a.f : a.gam);
    const double *pd = nullptr;  // no operand in float64
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int c0 = 2 * (t + P * j);
      if (vec) {
        using V = cplx<R>;
        V x1 = cmake<V>((R)0, (R)0);
        double2 xd = make_double2(0.0, 0.0);
        if (col_ok(c0)) {
          if (p1) x1 = *reinterpret_cast<const V *>(p1 + rowoff + c0);
          if (pd) xd = *reinterpret_cast<const double2 *>(pd + rowoff + c0);
        }
        o1[2 * j] = x1.x;
        o1[2 * j + 1] = x1.y;
        od[2 * j] = xd.x;
        od[2 * j + 1] = xd.y;
      } else {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const bool ok = col_ok(c0 + e);
          o1[2 * j + e] = (ok && p1) ? p1[rowoff + c0 + e] : (R)0;
          od[2 * j + e] = (ok && pd) ? pd[rowoff + c0 + e] : 0.0;
        }
      }
    }
  }

  // ---- 2. scalars ------------------------------------------------------------
  double beta, inv_ft2, ft;
  if constexpr (MODE == X_GHAT) {
    double lo, hi;
    int fl;
    reduce_forcing(a.red, a.ft_mode, a.ftilde_given, &lo, &hi, &fl);
    ft = a.ft_mode == SWEIK_FT_NU ? sqrt(0.5 * (lo * lo + hi * hi))
         : a.ft_mode == SWEIK_FT_FMAX ? hi : a.ftilde_given;
    beta = ft * a.h / a.hbar;
    inv_ft2 = 1.0 / (ft * ft);
    if (tid == 0) {
      // the origin value is used only by the group of line 0
      s_par[0] = bid == 0 ? kappa0_3d(beta) : 0.0;
      if (bid == 0) {
        const double c0 = fmax((hi - ft) * (hi + ft), (ft - lo) * (ft + lo)) * inv_ft2;
        if (!(c0 < 1.0)) fl |= SWEIK_FLAG_C0_GE_1;
        for (int k = 0; k < a.n_src; ++k) {
          const int y0 = a.src[3 * k], y1 = a.src[3 * k + 1], y2 = a.src[3 * k + 2];
          if (y0 < 0 || y0 >= a.n0 || y1 < 0 || y1 >= a.n1 || y2 < 0 || y2 >= a.n2)
            fl |= SWEIK_FLAG_BAD_SOURCE;
        }
        Params p;
        p.ftilde = ft;
        p.beta = beta;
        p.hbar = a.hbar;
        p.inv_ft2 = inv_ft2;
        p.kappa0 = s_par[0];
        p.fmin = lo;
        p.fmax = hi;
        p.c0 = c0;
        p.flags = fl;
        p.pad_ = 0;
        *a.par = p;
        if (a.info) {
          a.info->f_min = lo;
          a.info->f_max = hi;
          a.info->ftilde = ft;
          a.info->beta = beta;
          a.info->c0_bound = c0;
          a.info->n_nonpositive_phi = 0;
          a.info->flags = fl;
          a.info->T = a.T;
        }
      }
    }
    __syncthreads();
  } else {
    beta = a.par->beta;
    inv_ft2 = a.par->inv_ft2;
    ft = a.par->ftilde;
  }
  int dstep = 0, E = 0;
  if (TERMLIKE) {
    dstep = exp_step(a.mu_red[term - 1]);
    E = a.expo[term - 1] + dstep;
  }
  if ((TERMLIKE || PHI0) && bid == 0 && tid == 0) {
    const int slot = TERMLIKE ? term : 0;
    a.expo[slot] = E;
    if (a.info) a.info->scale_exp[slot] = E;
    if (a.ck_expo) a.ck_expo[slot] = E;
  }
  // adjoint: lambda's exponent (from the partial maxima of |lambda|), and
  // the stored exponent of phi_{i-1}
  int elam = 0, Eprev = 0;
  if constexpr (ADJ0) {
    double mx = 0.0;
    for (int i = tid; i < kRedBlocks; i += kThreads) mx = fmax(mx, a.red[i]);
    mx = block_max(mx);
    elam = exp_step(mx);
    if (bid == 0 && tid == 0) a.expo[0] = elam;
  }
  if constexpr (ADJ) {
    elam = a.expo[0];
    Eprev = a.ck_expo[term - 1];
  }
  // last term: signed scales (-1)^i 2^E_i of the stored terms
  __shared__ double s_sE[MODE == X_LAST ? SWEIK_MAX_TERMS + 1 : 1];
  if (MODE == X_LAST)
    for (int i = tid; i < a.T; i += kThreads) s_sE[i] = ((i & 1) ? -1.0 : 1.0) * ldexp(1.0, a.expo[i]);
  constexpr int kSrcLds = MODE == X_PHI0 ? 512 : 1;
  __shared__ int s_src[3 * kSrcLds];
  __shared__ R s_lw[kSrcLds];
  auto logw = [&](int k) -> double {  // -s_k / hbar (log2 e times that in float32)
    const double l = a.src_s ? -(double)a.src_s[k] / a.hbar : 0.0;
    return sizeof(R) == 4 ? l * 1.4426950408889634 : l;
  };
  if (MODE == X_PHI0) {
    for (int i = tid; i < 3 * min(a.n_src, kSrcLds); i += kThreads) s_src[i] = a.src[i];
    for (int i = tid; i < min(a.n_src, kSrcLds); i += kThreads) s_lw[i] = (R)logw(i);
  }

#pragma unroll
  for (int u = 0; u < NTW; ++u) {
    const int k = tid + u * kThreads;
    if (k < H) twl[k] = twr[u];
  }
  stage_tw_store<H, 16>(tsr, tws, tid, kThreads);
  __syncthreads();

  // ---- 3. kernel table -------------------------------------------------------
  if constexpr (TABLE) {
    // line (d0, d1) = (i0, i1): x(c) = kappa(|d|) for c < n2, -kappa at M2 - c
    // for 0 < c < n2, zero between (the same for dkappa/dbeta)
    const double k0v = MODE == X_GHAT ? s_par[0] : 0.0;
    const long long r01 = (long long)i0 * i0 + (long long)i1 * i1;
    const int M2 = 2 * H;
    auto kv = [&](long long r2) -> R {
      if constexpr (MODE == X_GHAT) return kappa_3d_t<R>(beta, r2, k0v);
      else if constexpr (MODE == X_ETAB) return exp_kernel_t<R>(beta, (int)r2);
      else return (R)dkappa_3d(beta, r2);
    };
    auto tab = [&](int c) -> R {
      if (!line_ok) return (R)0;
      if (c < a.n2) return kv(r01 + (long long)c * c);
      const int d = M2 - c;
      if (d < a.n2) return -kv(r01 + (long long)d * d);
      return (R)0;
    };
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int c0 = 2 * (t + P * j);
      v[j] = cmake<C>(tab(c0), tab(c0 + 1));
    }
  }

  if constexpr (TERMLIKE || ADJ || MODE == X_PHI0F) odd_c2r<R, H>(v, t, line, twl, tws, w1);
  if constexpr (MODE == X_ADJ_B) odd_c2r<R, H>(vc, t, line, twl, tws, w1);

  // full gradient: d phi_0 / d beta and d phi_0 / d hbar (through the
  // weights w_k = exp(-s_k / hbar)) at column cc of this line, in float64
  auto dphi0 = [&](int cc, double &dbeta, double &dhbar) {
    dbeta = 0.0;
    dhbar = 0.0;
    for (int k = 0; k < a.n_src; ++k) {
      const double d0 = (double)(i0 - a.src[3 * k]), d1 = (double)(i1 - a.src[3 * k + 1]);
      const double d2 = (double)(cc - a.src[3 * k + 2]);
      const double dist = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
      const double sk = a.src_s ? (double)a.src_s[k] : 0.0;
      const double e = exp(-sk / a.hbar - beta * dist);
      dbeta -= dist * e;
      dhbar += e * sk / (a.hbar * a.hbar);
    }
  };
  // per-work-group slot of the full gradient's partial sums
  auto gslot = [&](int slot) -> double & { return a.gpart[(size_t)slot * a.nbx + bid]; };

  // ---- 4a. adjoint pointwise steps (columns c = 2m, 2m+1, m = t + P j) --------
  // Each chunk of four column pairs reads its operands before any store (a
  // read after a store would wait for it: the arrays may alias as far as the
  // compiler knows).
  if constexpr (ADJ0) {
    const double lam_scale = ldexp(1.0, -elam);
    const double sgnT = (a.T & 1) ? -1.0 : 1.0;
    double ps[FULLG ? 3 : 1] = {};  // S/hbar, a_0 d phi_0/d beta, a_0 d phi_0/d hbar
#pragma unroll
    for (int j0 = 0; j0 < 8; j0 += 4) {
      R qf[4][2], qs[4][2];
      double qp[4][2];
#pragma unroll
      for (int jj = 0; jj < 4; ++jj)
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int cc = 2 * (t + P * (j0 + jj)) + e;
          const bool ok = col_ok(cc);
          qf[jj][e] = ok ? a.f[rowoff + cc] : (R)1;
          qs[jj][e] = ok ? a.dLdS[rowoff + cc] : (R)0;
          qp[jj][e] = ok ? a.ck_phi[rowoff + cc] : 1.0;
        }
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        R zz[2] = {(R)0, (R)0};
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int cc = 2 * (t + P * (j0 + jj)) + e;
          if (col_ok(cc)) {
            const double fa = (double)qf[jj][e];
            a.gam[rowoff + cc] = (R)((fa - ft) * (fa + ft) * inv_ft2);
            const double ph = qp[jj][e];
            double l = 0.0;
            if (ph > 0.0 && isfinite(ph)) l = -a.hbar * (double)qs[jj][e] / ph * lam_scale;
            const R q = (R)l;
            a.lam[rowoff + cc] = q;
            zz[e] = (R)(sgnT * (double)q);
            if constexpr (FULLG) {
              if (ph > 0.0 && isfinite(ph)) ps[0] += (double)qs[jj][e] * -log(ph);
              if (a.T == 0) {  // phi = phi_0: a_0 = lambda
                double db, dh;
                dphi0(cc, db, dh);
                ps[1] += (double)q * db;
                ps[2] += (double)q * dh;
              }
            }
          }
        }
        v[j0 + jj] = cmake<C>(zz[0], zz[1]);
      }
    }
#pragma unroll
    for (int j = 8; j < 16; ++j) v[j] = cmake<C>((R)0, (R)0);
    if constexpr (FULLG) {
      block_sums_d(ps);
      if (tid == 0) {
        const double sl = ldexp(1.0, elam);
        gslot(G_S) = ps[0];
        gslot(G_C) = 0.0;
        gslot(G_B0) = ps[1] * sl;
        gslot(G_H0) = ps[2] * sl;
        gslot(G_GF) = 0.0;
      }
      if (a.T == 0) return;
    }
  }
  if constexpr (ADJ) {
    const double gscale = ldexp(1.0, Eprev + elam);
    const double sgn_prev = ((term - 1) & 1) ? -1.0 : 1.0;  // (-1)^(i-1)
    const R *mprev = a.terms + (size_t)(term - 1) * ((size_t)a.nlines * a.n2);
    const R *p2 = term > 1 ? a.gam : a.f;  // gamma, or f at the last step
    const bool need3 = term > 1 || FULLG;   // lambda
    // full gradient: <c_i, gamma phi_{i-1}>, and at term 1 a_0 d phi_0 and
    // dL/dgamma f^2 (mantissa sums; scales applied per work-group)
    double ps[FULLG ? 4 : 1] = {};
#pragma unroll
    for (int j0 = 0; j0 < 8; j0 += 4) {
      R q1[4][2], q2[4][2], q3[4][2];
      double qd[4][2];
#pragma unroll
      for (int jj = 0; jj < 4; ++jj)
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int cc = 2 * (t + P * (j0 + jj)) + e;
          const bool ok = col_ok(cc);
          q1[jj][e] = ok ? mprev[rowoff + cc] : (R)0;
          q2[jj][e] = ok ? p2[rowoff + cc] : (R)0;
          q3[jj][e] = (ok && need3) ? a.lam[rowoff + cc] : (R)0;
          qd[jj][e] = (ok && term != a.T) ? a.acc[rowoff + cc] : 0.0;
        }
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int j = j0 + jj;
        R zz[2] = {(R)0, (R)0};
        const double bb[2] = {(double)v[j].x, (double)v[j].y};
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int cc = 2 * (t + P * j) + e;
          if (col_ok(cc)) {
            // dL/dgamma += phi_{i-1} b_i  (true scale 2^(E_{i-1} + e_lam))
            const double mp = (double)q1[jj][e];
            const double g = mp * bb[e] * gscale + qd[jj][e];
            double ga;  // gamma at this point
            if (term > 1) {
              a.acc[rowoff + cc] = g;
              ga = (double)q2[jj][e];
              zz[e] = (R)(sgn_prev * (double)q3[jj][e] + ga * bb[e]);
            } else {
              // dL/df = dL/dgamma * 2 f / ftilde^2
              const double fa = (double)q2[jj][e];
              a.dLdf[rowoff + cc] = (R)(g * 2.0 * fa * inv_ft2);
              ga = (fa - ft) * (fa + ft) * inv_ft2;
            }
            if constexpr (MODE == X_ADJ_B) {
              if (term == 1) {
                const double fa = (double)q2[jj][e];
                const double a0 = (double)q3[jj][e] + ga * bb[e];  // a_0 = lambda + gamma b_1
                double db, dh;
                dphi0(cc, db, dh);
                ps[1] += a0 * db;
                ps[2] += a0 * dh;
                ps[3] += g * fa * fa;
              }
              ps[0] += (double)(e ? vc[j].y : vc[j].x) * ga * mp;
            }
          }
        }
        v[j] = cmake<C>(zz[0], zz[1]);
      }
    }
    if constexpr (MODE == X_ADJ_B) {
      block_sums_d(ps);
      if (tid == 0) {
        gslot(G_C) += ps[0] * gscale;
        if (term == 1) {
          const double sl = ldexp(1.0, elam);
          gslot(G_B0) = ps[1] * sl;
          gslot(G_H0) = ps[2] * sl;
          gslot(G_GF) = ps[3];
        }
      }
    }
    if (term == 1) return;
#pragma unroll
    for (int j = 8; j < 16; ++j) v[j] = cmake<C>((R)0, (R)0);
  }

  // ---- 4. pointwise step -------------------------------------------------------
  if constexpr (MODE == X_SEED) {
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = cmake<C>(o1[2 * j], o1[2 * j + 1]);
#pragma unroll
    for (int j = 8; j < 16; ++j) v[j] = cmake<C>((R)0, (R)0);
  }
  if constexpr (PHI0 || TERMLIKE) {
    long long nbad = 0;
    const R sm = (R)ldexp(1.0, -dstep);
    const double sE = ((TERMLIKE && (term & 1)) ? -1.0 : 1.0) * ldexp(1.0, E);
    R mlr = (R)0;
    R *tout = a.terms + (size_t)(TERMLIKE ? term : 0) * ((size_t)a.nlines * a.n2) + rowoff;
    // last term: the float64 sum of the stored terms 0..T-1 at this thread's
    // columns, in the order of the terms
    double ps[16];
    if constexpr (MODE == X_LAST) {
      using V = cplx<R>;
      const size_t NN = (size_t)a.nlines * a.n2;
      auto pair = [&](const R *q, int c0) -> V {
        V x = cmake<V>((R)0, (R)0);
        if (!col_ok(c0)) return x;
        if (vec) return *reinterpret_cast<const V *>(q + c0);
        x.x = q[c0];
        if (FULL || c0 + 1 < a.n2) x.y = q[c0 + 1];
        return x;
      };
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const V x = pair(a.terms + rowoff, 2 * (t + P * j));
        ps[2 * j] = (double)x.x;
        ps[2 * j + 1] = (double)x.y;
      }
      for (int i0 = 1; i0 < a.T; i0 += 4) {  // four terms of loads in flight
        V q[4][8];
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (i0 + u < a.T) {
#pragma unroll
            for (int j = 0; j < 8; ++j)
              q[u][j] = pair(a.terms + (size_t)(i0 + u) * NN + rowoff, 2 * (t + P * j));
          }
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (i0 + u < a.T) {
            const double sc = s_sE[i0 + u];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
              ps[2 * j] = fma((double)q[u][j].x, sc, ps[2 * j]);
              ps[2 * j + 1] = fma((double)q[u][j].y, sc, ps[2 * j + 1]);
            }
          }
      }
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int c0 = 2 * (t + P * j);
      R z0 = 0, z1 = 0;
      if (col_ok(c0)) {
        const bool ok1 = FULL || c0 + 1 < a.n2;
        double p0, p1 = 0.0;
        R m0, m1;
        if constexpr (MODE == X_PHI0F) {
          // phi_0 = exp(-beta |m|) (*) source grid (Table 1 steps 1-5): the
          // kernel spectrum carries the transforms' scale
          m0 = v[j].x;
          m1 = v[j].y;
          p0 = (double)m0;
          p1 = (double)m1;
        } else if constexpr (MODE == X_PHI0) {
          // phi_0 = sum_k exp(-beta |m - y_k|)  (eq. phi_0Solution, C = 1)
          double s0 = 0.0, s1 = 0.0;
          // the first kSrcLds sources from LDS, the rest from global memory
          // (two loops, so that no load picks its address space at run time)
          const int nl = min(a.n_src, kSrcLds);
          if constexpr (sizeof(R) == 4) {
            const float nb = (float)(-beta * 1.4426950408889634);  // exp(x) = 2^(x log2 e)
            float f0 = 0.0f, f1 = 0.0f;
            auto add = [&](int y0, int y1, int y2, float lw) {
              const float d0 = (float)(i0 - y0), d1 = (float)(i1 - y1);
              const float d2 = (float)(c0 - y2);
              const float q = d0 * d0 + d1 * d1;
              f0 += __builtin_amdgcn_exp2f(nb * __builtin_amdgcn_sqrtf(q + d2 * d2) + lw);
              f1 += __builtin_amdgcn_exp2f(nb * __builtin_amdgcn_sqrtf(q + (d2 + 1.0f) * (d2 + 1.0f)) + lw);
            };
            for (int k = 0; k < nl; ++k) add(s_src[3 * k], s_src[3 * k + 1], s_src[3 * k + 2], (float)s_lw[k]);
            for (int k = nl; k < a.n_src; ++k)
              add(a.src[3 * k], a.src[3 * k + 1], a.src[3 * k + 2], (float)logw(k));
            s0 = f0;
            s1 = f1;
          } else {
            auto add = [&](int y0, int y1, int y2, double lw) {
              const double d0 = (double)(i0 - y0), d1 = (double)(i1 - y1);
              const double d2 = (double)(c0 - y2);
              const double q = d0 * d0 + d1 * d1;
              s0 += exp(lw - beta * sqrt(q + d2 * d2));
              s1 += exp(lw - beta * sqrt(q + (d2 + 1) * (d2 + 1)));
            };
            for (int k = 0; k < nl; ++k) add(s_src[3 * k], s_src[3 * k + 1], s_src[3 * k + 2], (double)s_lw[k]);
            for (int k = nl; k < a.n_src; ++k) add(a.src[3 * k], a.src[3 * k + 1], a.src[3 * k + 2], logw(k));
          }
          m0 = (R)s0;
          m1 = (R)s1;
          p0 = s0;
          p1 = s1;
        } else {
          m0 = v[j].x * sm;  // power-of-two rescale: exact
          m1 = v[j].y * sm;
          p0 = last ? fma((double)m0, sE, ps[2 * j]) : 0.0;
          p1 = (last && ok1) ? fma((double)m1, sE, ps[2 * j + 1]) : 0.0;
        }
        if (last) {
          nbad += write_S(a, rowoff + c0, p0);
          if (a.ck_phi) a.ck_phi[rowoff + c0] = p0;
          if (ok1) {
            nbad += write_S(a, rowoff + c0 + 1, p1);
            if (a.ck_phi) a.ck_phi[rowoff + c0 + 1] = p1;
          }
        } else {
          if (vec)
            *reinterpret_cast<cplx<R> *>(tout + c0) = cmake<cplx<R>>(m0, m1);
          else {
            tout[c0] = m0;
            if (ok1) tout[c0 + 1] = m1;
          }
          R g0, g1 = (R)0;
          if constexpr (PHI0) {
            const double fa = (double)o1[2 * j];
            g0 = (R)((fa - ft) * (fa + ft) * inv_ft2);
            a.gam[rowoff + c0] = g0;
            if (ok1) {
              const double fb = (double)o1[2 * j + 1];
              g1 = (R)((fb - ft) * (fb + ft) * inv_ft2);
              a.gam[rowoff + c0 + 1] = g1;
            }
          } else {
            g0 = o1[2 * j];
            if (ok1) g1 = o1[2 * j + 1];
          }
          z0 = g0 * m0;
          z1 = ok1 ? g1 * m1 : (R)0;
          mlr = fmax(mlr, fabs(m0));
          if (ok1) mlr = fmax(mlr, fabs(m1));
        }
      }
      v[j] = cmake<C>(z0, z1);
    }
    if (last) {
      const long long nb = block_sum_ll(nbad);
      if (tid == 0 && a.info && nb)
        atomicAdd((unsigned long long *)&a.info->n_nonpositive_phi, (unsigned long long)nb);
      return;
    }
    const double bm = block_max((double)mlr);
    if (tid == 0) a.mu[(size_t)(TERMLIKE ? term : 0) * a.nbx + bid] = bm;
#pragma unroll
    for (int j = 8; j < 16; ++j) v[j] = cmake<C>((R)0, (R)0);
  }

  // ---- 5. forward real FFT, store the line's spectrum ------------------------
  odd_r2c<R, H>(v, t, line, twl, tws, w1);
  if (line_ok) {
    C *sl = a.s1 + (size_t)rs * H;
#pragma unroll
    for (int j = 0; j < 16; ++j) sl[t + P * j] = v[j];
  }
}

template <typename R, int MODE, int H>
__global__ void __launch_bounds__(kThreads) k_x3(Args3<R> a, int term) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int bid = blockIdx.x;
  if ((bid + 1) * x_lpw(H) <= a.nlines && a.n2 == H)
    x_pass<R, MODE, H, true>(a, term, smem_raw, bid);
  else
    x_pass<R, MODE, H, false>(a, term, smem_raw, bid);
}

}  // namespace sweik
