// row2d.hpp -- row passes of the 2D solve (forward and adjoint).
//
// One team of P = H/E threads per grid row (E = 16, 8 or 4 elements per
// thread), RPW = max(1, 4096/H) rows and RPW P threads per work-group.  A
// pass (i) reads its spectral tile (RPW contiguous rows of the blocked
// spectrum), the twiddle table and the pointwise operands of its rows,
// (ii) takes the inverse real FFT of each row (complex FFT of length H
// plus a split step), (iii) applies the pointwise step of its mode, and
// (iv) takes the forward real FFT of the new forcing and stores the tile.
// The pass after the last convolution (ROW_LAST) stops after (iii): it sums
// the stored terms in float64 and writes S.
#pragma once

#include "common2d.hpp"

namespace sweik {

// Spectral tile of a row work-group: rows [row0, row0 + rows) of the blocked
// transposed spectrum spec[b][k1][rr], k1 < H (column 0 holds the real DC
// and Nyquist bins of the row as one complex number).  Element e <-> (local
// row, column).
template <typename R, int H, int E> struct RowTile {
  static constexpr int RB = spec_rb<R>(), RPW = row_rpw(H), LDK = H, NT = row_threads(H, E);
  static constexpr int NREG = (RPW * LDK + NT - 1) / NT;  // per thread
  cplx<R> *base;
  int rows;
  __device__ __forceinline__ void init(cplx<R> *spec, int row0, int spec_rows) {
    rows = min(RPW, spec_rows - row0);
    if constexpr (RPW >= RB) {
      base = spec + (size_t)row0 * LDK;
    } else {
      const int b = row0 / RB, rr0 = row0 - b * RB;
      base = spec + ((size_t)b * LDK * RB + rr0);
    }
  }
  __device__ __forceinline__ void map(int e, int &rl, int &k1, int &off) const {
    if constexpr (RPW >= RB) {
      constexpr int PER = LDK * RB;
      const int bl = e / PER, rem = e - bl * PER;
      k1 = rem / RB;
      rl = bl * RB + (rem - k1 * RB);
      off = e;
    } else {
      k1 = e / RPW;
      rl = e - k1 * RPW;
      off = k1 * RB + rl;
    }
  }
};

template <bool FULL, typename R, int H, int E>
__device__ __forceinline__ void tile_issue(const RowTile<R, H, E> &tile, int tid,
                                           cplx<R> (&tl)[RowTile<R, H, E>::NREG]) {
  const int total = tile.rows * H;
#pragma unroll
  for (int u = 0; u < RowTile<R, H, E>::NREG; ++u) {
    const int e = tid + u * RowTile<R, H, E>::NT;
    if (FULL || e < total) {
      int rl, k1, off;
      tile.map(e, rl, k1, off);
      tl[u] = tile.base[off];
    }
  }
}

template <bool FULL, typename R, int H, int E>
__device__ __forceinline__ void tile_to_lds(const RowTile<R, H, E> &tile, int tid,
                                            const cplx<R> (&tl)[RowTile<R, H, E>::NREG],
                                            cplx<R> *lines) {
  constexpr int LL = row_line_len<R>(H);
  const int total = tile.rows * H;
#pragma unroll
  for (int u = 0; u < RowTile<R, H, E>::NREG; ++u) {
    const int e = tid + u * RowTile<R, H, E>::NT;
    if (FULL || e < total) {
      int rl, k1, off;
      tile.map(e, rl, k1, off);
      lines[rl * LL + lslot<cplx<R>>(k1)] = tl[u];
    }
  }
}

template <bool FULL, typename R, int H, int E>
__device__ __forceinline__ void tile_store(const RowTile<R, H, E> &tile, int tid,
                                           const cplx<R> *lines) {
  constexpr int LL = row_line_len<R>(H);
  const int total = tile.rows * H;
  cplx<R> out[RowTile<R, H, E>::NREG];
#pragma unroll
  for (int u = 0; u < RowTile<R, H, E>::NREG; ++u) {
    const int e = tid + u * RowTile<R, H, E>::NT;
    if (FULL || e < total) {
      int rl, k1, off;
      tile.map(e, rl, k1, off);
      out[u] = lines[rl * LL + lslot<cplx<R>>(k1)];
    }
  }
#pragma unroll
  for (int u = 0; u < RowTile<R, H, E>::NREG; ++u) {
    const int e = tid + u * RowTile<R, H, E>::NT;
    if (FULL || e < total) {
      int rl, k1, off;
      tile.map(e, rl, k1, off);
      tile.base[off] = out[u];
    }
  }
}

// Split-step twiddle k from the LDS table(s) (see row_twl_len): the entry
// itself, or beyond 4096 points the product of the coarse entry k >> 6 and
// the fine entry k & 63.  split_tw_k: the twiddle index held by table entry e.
__host__ __device__ constexpr int split_tw_k(int H, int e) {
  return !row_split2(H) ? e
         : e < (H >> kSplitFineBits) ? e << kSplitFineBits
                                     : e - (H >> kSplitFineBits);
}
template <typename R, int H>
__device__ __forceinline__ cplx<R> split_tw(const cplx<R> *twl, int k) {
  if constexpr (!row_split2(H)) {
    return twl[k];
  } else {
    constexpr int NA = H >> kSplitFineBits, MASK = (1 << kSplitFineBits) - 1;
    return cmul(twl[k >> kSplitFineBits], twl[NA + (k & MASK)]);
  }
}

// Inverse real FFT of this team's row (already in LDS): on return
// v[j] = (x[2k], x[2k+1]) * 2 M1, k = t + P j, x the real row (M1 = 2H).
template <typename R, int H, int E>
__device__ __forceinline__ void row_c2r(cplx<R> (&v)[E], int t, cplx<R> *line,
                                        const cplx<R> *twl, const cplx<R> *tws) {
  using C = cplx<R>;
  constexpr int P = H / E;
  // split step: Z = (X_k + conj X_{H-k}) + i (X_k - conj X_{H-k}) conj(w^k);
  // for k = 0 the stored pair (X_0, X_H) gives Z = (X_0 + X_H, X_0 - X_H)
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int k = t + P * j;
    C xk = line[lslot<cplx<R>>(k)];
    C xc = cconj(line[lslot<cplx<R>>((H - k) & (H - 1))]);
    C e = cadd(xk, xc);
    C o = cmulc(csub(xk, xc), split_tw<R, H>(twl, k));
    v[j] = cmake<C>(e.x - o.y, e.y + o.x);
    if (k == 0) v[j] = cmake<C>(xk.x + xk.y, xk.x - xk.y);
  }
  team_fft<H, true, true>(v, t, line, tws, true);
}

// Forward real FFT of this team's row (v[j] = (x[2k], x[2k+1]), k = t + P j)
// into its LDS line as the half spectrum (twice the DFT, bins 0 and H packed
// into column 0), then the store of the work-group's tile.
template <bool FULL, typename R, int H, int E>
__device__ __forceinline__ void row_r2c_store(cplx<R> (&v)[E], int t, int tid,
                                              cplx<R> *line, const cplx<R> *lines,
                                              const cplx<R> *twl, const cplx<R> *tws,
                                              const RowTile<R, H, E> &tile) {
  using C = cplx<R>;
  constexpr int P = H / E;
  team_fft<H, false, true>(v, t, line, tws, true);
  __syncthreads();
#pragma unroll
  for (int j = 0; j < E; ++j) line[lslot<cplx<R>>(t + P * j)] = v[j];
  __syncthreads();
  C x[E];
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int k = t + P * j;
    C zk = line[lslot<cplx<R>>(k)];
    C zc = cconj(line[lslot<cplx<R>>((H - k) & (H - 1))]);
    C e = cadd(zk, zc);
    C d = csub(zk, zc);
    C o = cmake<C>(d.y, -d.x);  // d / i
    x[j] = cadd(e, cmul(split_tw<R, H>(twl, k), o));
    // k = 0: the real bins X_0 and X_H travel together
    if (k == 0) x[j] = cmake<C>((R)2 * (zk.x + zk.y), (R)2 * (zk.x - zk.y));
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < E; ++j) line[lslot<cplx<R>>(t + P * j)] = x[j];
  __syncthreads();
  tile_store<FULL>(tile, tid, lines);
}

// ---------------------------------------------------------------------------
// Row pass, all modes.
//   ROW_GHAT  kernel table rows (evenly extended), forward real FFT
//   ROW_PHI0  phi_0 from the sources, first forcing term, forward real FFT
//   ROW_TERM  term `term` < T: inverse FFT, rescale, store the term, the
//             next forcing term and its FFT
//   ROW_LAST  term T: inverse FFT, the sum of all terms in float64 and
//             S = -hbar ln phi
//   ROW_SEED  transform of the source grid (phi_0 by FFT)
//   ROW_ADJ0  adjoint start: lambda = -hbar dL/dS / phi, a_T = (-1)^T lambda
//   ROW_ADJ   adjoint step `term` = i: b_i = kappa (*) a_i, dL/dgamma +=
//             phi_{i-1} b_i, a_{i-1} = (-1)^{i-1} lambda + gamma b_i; at
//             i = 1, dL/df = dL/dgamma 2 f / ftilde^2
// ---------------------------------------------------------------------------
// FULL: every row of the work-group lies in the grid and n1 == H, so no
// element needs a bounds check (columns >= H are zero padding, known
// statically).
template <typename R, int MODE, int H, int E, bool FULL>
__device__ __forceinline__ void row_pass(const Args2<R> &a, int term, unsigned char *smem_raw,
                                         const int bid) {
  using C = cplx<R>;
  using Tile = RowTile<R, H, E>;
  constexpr int P = H / E, RPW = row_rpw(H), LL = row_line_len<R>(H), NT = row_threads(H, E);
  constexpr int TWLOG = ilog2c(2 * H);
  constexpr bool STG = row_staged<R>(H, MODE);
  constexpr int TWL = row_twl_len(H), NTW = (TWL + NT - 1) / NT;
  constexpr bool LASTLIKE = MODE == ROW_LAST || MODE == ROW_LASTT;
  constexpr bool TERMLIKE = MODE == ROW_TERM || LASTLIKE;
  constexpr bool ADJ = MODE == ROW_ADJ || MODE == ROW_ADJ_B;
  constexpr bool ADJ0 = MODE == ROW_ADJ0 || MODE == ROW_ADJ0_B;
  constexpr bool FULLG = MODE == ROW_ADJ_B || MODE == ROW_ADJ0_B;  // full gradient
  constexpr bool GHATLIKE = MODE == ROW_GHAT || MODE == ROW_DGHAT;
  constexpr bool LOADS_TILE = TERMLIKE || ADJ || MODE == ROW_PHI0;
  // phi_0 reads the spectrum only on its FFT route
  const bool tile_in = MODE != ROW_PHI0 || a.phi0_fft;
  C *twl = reinterpret_cast<C *>(smem_raw);  // exp(-2 pi i k / 2H), k < H (split steps)
  C *tws = twl + TWL;                        // stage tables of the length-H FFT
  C *lines = tws + row_stage_tw<R>(H);
  unsigned char *stg = reinterpret_cast<unsigned char *>(lines + RPW * LL);
  __shared__ double s_par[2];

  const int tid = threadIdx.x, team = tid / P, t = tid - team * P;
  const int row0 = bid * RPW, r = row0 + team;
  C *line = lines + team * LL;
  const bool row_ok = FULL || r < a.n0;
  const size_t rowoff = (size_t)r * a.n1;
  const size_t N = (size_t)a.n0 * a.n1;
  const bool last = LASTLIKE || (MODE == ROW_PHI0 && a.T == 0);
  // column c of this thread's pair j (c = 2(t + P j) + e) lies in the grid
  auto col_ok = [&](int c) { return FULL ? true : (row_ok && c < a.n1); };
  Tile tile;
  tile.init(a.spec, row0, a.nb * spec_rb<R>());

  // staging rows of this team (written and read by the same thread)
  R *sR = reinterpret_cast<R *>(stg) + (size_t)team * H;                   // first R row
  constexpr int NRSTG = ADJ ? 3 : 1;
  double *sD = reinterpret_cast<double *>(reinterpret_cast<R *>(stg) + (size_t)RPW * H * NRSTG) +
               (size_t)team * H;

  // ---- 1. issue the global reads of the pass ------------------------------
  C twr[NTW];
#pragma unroll
  for (int u = 0; u < NTW; ++u) {
    const int e = tid + u * NT;
    twr[u] = a.tw[min(split_tw_k(H, e), H - 1) << (a.lmax_log - TWLOG)];  // stored if e < TWL
  }
  constexpr int NSR = (stage_tw_len(H, E) + NT - 1) / NT;
  C tsr[NSR > 0 ? NSR : 1];
  stage_tw_issue<H, E>(tsr, a.tw, a.lmax_log, tid, NT);
  C tl[Tile::NREG];
  if (LOADS_TILE && tile_in) tile_issue<FULL>(tile, tid, tl);
  // full gradient: the tile of c_i = dkappa/dbeta (*) a_i
  Tile tile2;
  C tl2[MODE == ROW_ADJ_B ? Tile::NREG : 1];
  if constexpr (MODE == ROW_ADJ_B) {
    tile2.init(a.spec2, row0, a.nb * spec_rb<R>());
    tile_issue<FULL>(tile2, tid, tl2);
  }
  // pointwise operands of this thread's columns c = 2(t + P j) + e
  constexpr int NOP = STG ? E : 1;
  R o1[NOP], o2[NOP], o3[NOP];
  double od[NOP];
  if constexpr (STG) {
    const R *p1 = nullptr, *p2 = nullptr, *p3 = nullptr;
    const double *pd = nullptr;
    if (MODE == ROW_PHI0) p1 = last ? nullptr : a.f;
    if (MODE == ROW_SEED) p1 = a.gam;  // the source grid
    if (ADJ) {
      p1 = a.ck_terms + (size_t)(term - 1) * N;
      p2 = term > 1 ? a.gam : a.f;
      p3 = (term > 1 || FULLG) ? a.lam : nullptr;  // the full gradient also needs a_0
      pd = term != a.T ? a.acc : nullptr;
    }
    // columns 2(t + P j) for j >= E/2 are >= H >= n1: zero padding
    if ((a.n1 & 1) == 0) {  // column pairs are aligned: vector loads
#pragma unroll
      for (int j = 0; j < E / 2; ++j) {
        const int c0 = 2 * (t + P * j);
        const bool ok = col_ok(c0);
        using V = cplx<R>;  // a pair of R
        V x1 = cmake<V>((R)0, (R)0), x2 = x1, x3 = x1;
        double2 xd = make_double2(0.0, 0.0);
        if (ok && p1) x1 = *reinterpret_cast<const V *>(p1 + rowoff + c0);
        if (ADJ) {
          if (ok && p2) x2 = *reinterpret_cast<const V *>(p2 + rowoff + c0);
          if (ok && p3) x3 = *reinterpret_cast<const V *>(p3 + rowoff + c0);
        }
        if (ok && pd) xd = *reinterpret_cast<const double2 *>(pd + rowoff + c0);
        o1[2 * j] = x1.x;
        o1[2 * j + 1] = x1.y;
        if (ADJ) {
          o2[2 * j] = x2.x;
          o2[2 * j + 1] = x2.y;
          o3[2 * j] = x3.x;
          o3[2 * j + 1] = x3.y;
        }
        od[2 * j] = xd.x;
        od[2 * j + 1] = xd.y;
      }
    } else {
#pragma unroll
      for (int q = 0; q < E; ++q) {
        const int cc = 2 * (t + P * (q >> 1)) + (q & 1);
        const bool ok = col_ok(cc);
        o1[q] = (ok && p1) ? p1[rowoff + cc] : (R)0;
        if (ADJ) {
          o2[q] = (ok && p2) ? p2[rowoff + cc] : (R)0;
          o3[q] = (ok && p3) ? p3[rowoff + cc] : (R)0;
        }
        od[q] = (ok && pd) ? pd[rowoff + cc] : 0.0;
      }
    }
  }

  // ---- 2. scalars ----------------------------------------------------------
  double beta, inv_ft2, ft;
  if (MODE == ROW_GHAT || MODE == ROW_GHATT) {
    double lo, hi;
    int fl;
    reduce_forcing(a.red, a.ft_mode, a.ftilde_given, &lo, &hi, &fl);
    ft = a.ft_mode == SWEIK_FT_NU ? sqrt(0.5 * (lo * lo + hi * hi))
         : a.ft_mode == SWEIK_FT_FMAX ? hi : a.ftilde_given;
    beta = ft * a.h / a.hbar;
    inv_ft2 = 1.0 / (ft * ft);
    // the first work-group checks the sources, one per thread (a loop in one
    // thread made every work-group wait for n_src dependent reads)
    __shared__ int s_badsrc;
    if (tid == 0) s_badsrc = 0;
    __syncthreads();
    if (bid == 0)
      for (int k = tid; k < a.n_src; k += NT) {
        const int y0 = a.src[2 * k], y1 = a.src[2 * k + 1];
        if (y0 < 0 || y0 >= a.n0 || y1 < 0 || y1 >= a.n1) atomicOr(&s_badsrc, 1);
      }
    __syncthreads();
    if (tid == 0) {
      // the origin value (one float64 Bessel evaluation in one thread) is
      // used only by the tile of row 0
      s_par[0] = bid == 0 ? kappa0_2d(beta) : 0.0;
      const double c0 = fmax((hi - ft) * (hi + ft), (ft - lo) * (ft + lo)) * inv_ft2;
      if (!(c0 < 1.0)) fl |= SWEIK_FLAG_C0_GE_1;
      if (s_badsrc) fl |= SWEIK_FLAG_BAD_SOURCE;
      if (bid == 0) {
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
  } else if (MODE == ROW_PHI0 && a.own_par) {
    // running beside the kernel-table pass: the same reduction and formulas
    // (bit-identical scalars), nothing published
    double lo, hi;
    int fl;
    reduce_forcing(a.red, a.ft_mode, a.ftilde_given, &lo, &hi, &fl);
    ft = a.ft_mode == SWEIK_FT_NU ? sqrt(0.5 * (lo * lo + hi * hi))
         : a.ft_mode == SWEIK_FT_FMAX ? hi : a.ftilde_given;
    beta = ft * a.h / a.hbar;
    inv_ft2 = 1.0 / (ft * ft);
  } else {
    beta = a.par->beta;
    inv_ft2 = a.par->inv_ft2;
    ft = a.par->ftilde;
  }

  // exponents: forward phi_i = 2^E_i m_i; adjoint a_i = 2^e_lam (mantissa)
  int dstep = 0, Ei = 0, elam = 0;
  double term_mu = 0.0;  // ROW_LASTT: max |m_{T-1}|
  // ROW_TERM: gamma at this thread's columns c = 2(t + P j) + e, kept in
  // registers until the pointwise step; issued after the previous term's
  // maxima, so that their reduction (and the inverse FFT) waits only for
  // the loads issued before them, while gamma arrives during the FFT
  R og[MODE == ROW_TERM ? E : 1];
  if (TERMLIKE) {
    // the previous pass's per-work-group maxima: the first four rounds are
    // read before any is folded (one wait instead of one per round)
    const double *mp = a.mu + (size_t)(term - 1) * a.nbr;
    double mr[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = tid + u * NT;
      mr[u] = i < a.nbr ? mp[i] : 0.0;
    }
    if constexpr (MODE == ROW_TERM) {
      if ((a.n1 & 1) == 0) {  // column pairs are aligned: vector loads
        using V = cplx<R>;
#pragma unroll
        for (int j = 0; j < E / 2; ++j) {
          const int c0 = 2 * (t + P * j);
          V x = cmake<V>((R)0, (R)0);
          if (col_ok(c0)) x = *reinterpret_cast<const V *>(a.gam + rowoff + c0);
          og[2 * j] = x.x;
          og[2 * j + 1] = x.y;
        }
      } else {
#pragma unroll
        for (int q = 0; q < E; ++q) {
          const int cc = 2 * (t + P * (q >> 1)) + (q & 1);
          og[q] = col_ok(cc) ? a.gam[rowoff + cc] : (R)0;
        }
      }
    }
    double mu = fmax(fmax(mr[0], mr[1]), fmax(mr[2], mr[3]));
    for (int i = tid + 4 * NT; i < a.nbr; i += NT) mu = fmax(mu, mp[i]);
    mu = block_max(mu);
    dstep = exp_step(mu);
    Ei = a.expo[term - 1] + dstep;
    // tilted solve: max |phi_{term-1}| (its mantissa maximum times its scale)
    if (a.tmax && bid == 0 && tid == 0) a.tmax[term - 1] = mu * ldexp(1.0, a.expo[term - 1]);
    if constexpr (MODE == ROW_LASTT) term_mu = mu;
  }
  if ((TERMLIKE || MODE == ROW_PHI0) && bid == 0 && tid == 0) {
    const int slot = TERMLIKE ? term : 0;
    a.expo[slot] = Ei;
    if (a.info) a.info->scale_exp[slot] = Ei;
    if (a.ck_expo) a.ck_expo[slot] = Ei;
  }
  // last term: signed scales (-1)^i 2^E_i of the stored terms (read after
  // the barrier below)
  __shared__ double s_sE[LASTLIKE ? SWEIK_MAX_TERMS + 1 : 1];
  if (LASTLIKE)
    for (int i = tid; i < a.T; i += NT) s_sE[i] = ((i & 1) ? -1.0 : 1.0) * ldexp(1.0, a.expo[i]);
  if (ADJ0) {
    double mx = 0.0;
    for (int i = tid; i < kRedBlocks; i += NT) mx = fmax(mx, a.red[i]);
    mx = block_max(mx);
    elam = exp_step(mx);
    if (bid == 0 && tid == 0) a.expo[0] = elam;
  }
  if (ADJ) {
    __shared__ int s_e[2];
    if (tid == 0) {
      s_e[0] = a.expo[0];
      s_e[1] = a.ck_expo[term - 1];
    }
    __syncthreads();
    elam = s_e[0];
    Ei = s_e[1];
  }

  // sources of phi_0 and their log-weights -s_k/hbar (the first kSrcLds of
  // them through LDS)
  constexpr int kSrcLds = MODE == ROW_PHI0 ? row_src_lds(H) : 1;
  __shared__ int s_src[2 * kSrcLds];
  __shared__ R s_lw[kSrcLds];
  auto logw = [&](int k) -> double {  // -s_k / hbar (log2 e times that in float32)
    const double l = a.src_s ? -(double)a.src_s[k] / a.hbar : 0.0;
    return sizeof(R) == 4 ? l * 1.4426950408889634 : l;
  };
  if (MODE == ROW_PHI0) {
    for (int i = tid; i < 2 * min(a.n_src, kSrcLds); i += NT) s_src[i] = a.src[i];
    for (int i = tid; i < min(a.n_src, kSrcLds); i += NT) s_lw[i] = (R)logw(i);
  }

  // ---- 3. operands into LDS -------------------------------------------------
#pragma unroll
  for (int u = 0; u < NTW; ++u) {
    const int e = tid + u * NT;
    if (e < TWL) twl[e] = twr[u];
  }
  stage_tw_store<H, E>(tsr, tws, tid, NT);
  if (LOADS_TILE && tile_in) tile_to_lds<FULL>(tile, tid, tl, lines);
  if constexpr (STG) {
#pragma unroll
    for (int q = 0; q < E; ++q) {
      // a staging row holds H >= n1 entries
      const int cc = 2 * (t + P * (q >> 1)) + (q & 1);
      if (FULL || cc < a.n1) {
        sR[cc] = o1[q];
        if (ADJ) {
          sR[(size_t)RPW * H + cc] = o2[q];
          sR[(size_t)2 * RPW * H + cc] = o3[q];
        }
        if (ADJ) sD[cc] = od[q];
      }
    }
  }
  __syncthreads();

  // Pointwise steps that store to global memory read their operands a chunk
  // of kOpChunk column pairs at a time, all before the chunk's stores: the
  // compiler cannot tell the stored arrays from the operand arrays, so a read
  // placed after a store would wait for everything before it (one memory
  // latency per column instead of one per chunk).
  constexpr int kOpChunk = E >= 16 ? 4 : 1;
  // operand access: staged copy or direct global read
  auto op1 = [&](int cc, const R *g) -> R { return STG ? sR[cc] : g[rowoff + cc]; };
  auto op2 = [&](int cc, const R *g) -> R { return STG ? sR[(size_t)RPW * H + cc] : g[rowoff + cc]; };
  auto op3 = [&](int cc, const R *g) -> R { return STG ? sR[(size_t)2 * RPW * H + cc] : g[rowoff + cc]; };
  auto opd = [&](int cc, const double *g) -> double { return STG ? sD[cc] : g[rowoff + cc]; };

  C v[E];

  // ---- 4. kernel table ------------------------------------------------------
  if constexpr (MODE == ROW_GHATT) {
    // Row r of the tilted kernel table for the offsets m0 = tsign r:
    // x[c] = kappa(r, m1) exp(beta (tsign tilt0 r + tilt1 m1)) with m1 = c
    // for c < n1 and m1 = c - 2H for c > 2H - n1 (kappa is even, the tilt is
    // not: both halves are evaluated), zero in between.
    const double k0v = s_par[0];
    const double a0 = (double)a.tsign * a.tilt0 * beta, a1 = a.tilt1 * beta;
    auto tab = [&](int c) -> R {
      const int m1 = c < a.n1 ? c : (c > 2 * H - a.n1 ? c - 2 * H : INT_MIN);
      if (!row_ok || m1 == INT_MIN) return (R)0;
      return kappa_2d_tilt_t<R>(beta, r, m1, a0 * r + a1 * m1, k0v, a.k0tab);
    };
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int c0 = 2 * (t + P * j);
      v[j] = cmake<C>(tab(c0), tab(c0 + 1));
    }
    row_r2c_store<FULL, R, H, E>(v, t, tid, line, lines, twl, tws, tile);
    return;
  }
  if constexpr (GHATLIKE) {
    // Row r of the evenly extended kernel table, x[m] = kappa(r, min(m,
    // 2H - m)) (zero for offsets >= n1): the first half is evaluated, the
    // mirrored half is read back through LDS.
    R *xl = reinterpret_cast<R *>(line);
    const double k0v = MODE == ROW_GHAT ? s_par[0] : 0.0;
#pragma unroll
    for (int j = 0; j < E / 2; ++j) {
      const int c0 = 2 * (t + P * j);
      R z0 = 0, z1 = 0;
      if (row_ok) {
        const int rr = r * r;
        auto tab = [&](int q) -> R {
          if constexpr (MODE == ROW_DGHAT) return (R)dkappa_2d(beta, q, a.k0tab);
          else return a.table ? exp_kernel_t<R>(beta, q) : kappa_2d_t<R>(beta, q, k0v, a.k0tab);
        };
        if (c0 < a.n1) z0 = tab(rr + c0 * c0);
        if (c0 + 1 < a.n1) z1 = tab(rr + (c0 + 1) * (c0 + 1));
      }
      xl[c0] = z0;
      xl[c0 + 1] = z1;
      v[j] = cmake<C>(z0, z1);
    }
    if (t == 0) xl[H] = (R)0;  // offset H >= n1 is never used
    __syncthreads();
#pragma unroll
    for (int j = E / 2; j < E; ++j) {
      const int c0 = 2 * (t + P * j);
      v[j] = cmake<C>(xl[2 * H - c0], xl[2 * H - c0 - 1]);
    }
    row_r2c_store<FULL, R, H, E>(v, t, tid, line, lines, twl, tws, tile);
    return;
  }

  // ---- 4b. transform of the source grid (phi_0 by FFT, Table 1 steps 1-3) ---
  if constexpr (MODE == ROW_SEED) {
#pragma unroll
    for (int j = 0; j < E / 2; ++j) {
      const int c0 = 2 * (t + P * j);
      R z0 = 0, z1 = 0;
      if (col_ok(c0)) {
        z0 = op1(c0, a.gam);
        if (FULL || c0 + 1 < a.n1) z1 = op1(c0 + 1, a.gam);
      }
      v[j] = cmake<C>(z0, z1);
    }
#pragma unroll
    for (int j = E / 2; j < E; ++j) v[j] = cmake<C>((R)0, (R)0);
    row_r2c_store<FULL, R, H, E>(v, t, tid, line, lines, twl, tws, tile);
    return;
  }

  if (LOADS_TILE && tile_in) row_c2r<R, H, E>(v, t, line, twl, tws);
  // full gradient: the inverse transform of c_i's tile through the same lines
  C vc[MODE == ROW_ADJ_B ? E : 1];
  if constexpr (MODE == ROW_ADJ_B) {
    __syncthreads();  // every team is done with its line
    tile_to_lds<FULL>(tile2, tid, tl2, lines);
    __syncthreads();
    row_c2r<R, H, E>(vc, t, line, twl, tws);
  }
  // the forcing of the next FFT is zero in the padding half (columns >= H)
#pragma unroll
  for (int j = E / 2; j < E; ++j) v[j] = cmake<C>((R)0, (R)0);

  // ---- 5. pointwise step over columns 2k, 2k+1 (k = t + P j, j < E/2) -----
  long long nbad = 0;
  if constexpr (MODE == ROW_PHI0 || TERMLIKE) {
    const bool even_n1 = FULL || (a.n1 & 1) == 0;
    // tilted solve (tmax set): the terms are phi_i exp(a . x - A) with
    // a = beta (tilt0, tilt1) and A = max_k (a . y_k - s_k / hbar), so that
    // the tilted phi_0 stays below n_src; phi_0's pass forms A and keeps it
    // for the last pass
    const bool tilted = a.tmax != nullptr && (MODE == ROW_PHI0 || MODE == ROW_LASTT);
    const double ta0 = a.tilt0 * beta, ta1 = a.tilt1 * beta;
    double tA = 0.0;
    if (MODE == ROW_PHI0 && tilted) {
      double m = -__builtin_huge_val();
      for (int k = 0; k < a.n_src; ++k) {
        const int y0 = k < kSrcLds ? s_src[2 * k] : a.src[2 * k];
        const int y1 = k < kSrcLds ? s_src[2 * k + 1] : a.src[2 * k + 1];
        const double lw = a.src_s ? -(double)a.src_s[k] / a.hbar : 0.0;
        m = fmax(m, ta0 * y0 + ta1 * y1 + lw);
      }
      tA = m;
      if (bid == 0 && tid == 0) a.tmax[a.T + 1] = tA;
    }
    if (MODE == ROW_LASTT) tA = a.tmax[a.T + 1];
    const R sm = (R)ldexp(1.0, -dstep);
    const double sE = ((TERMLIKE && (term & 1)) ? -1.0 : 1.0) * ldexp(1.0, Ei);
    R mlr = (R)0;
    const int slot = TERMLIKE ? term : 0;
    R *tout = a.terms + (size_t)slot * N + rowoff;  // this term's mantissas
    // unstaged operand (f for phi_0) of this thread's columns,
    // read before the loop's stores (see kOpChunk)
    constexpr bool PRE = !STG && MODE == ROW_PHI0;
    R opre[PRE ? E : 1];
    if constexpr (PRE) {
      const R *po = MODE == ROW_PHI0 ? a.f : a.gam;
#pragma unroll
      for (int q = 0; q < E; ++q) {
        const int cc = 2 * (t + P * (q >> 1)) + (q & 1);
        opre[q] = (!last && col_ok(cc)) ? po[rowoff + cc] : (R)0;
      }
    }
    auto opr = [&](int q, int cc, const R *g) -> R {
      if constexpr (MODE == ROW_TERM) return og[q];
      else if constexpr (PRE) return opre[q];
      else return op1(cc, g);
    };
    // tilted solve, last pass: the tilt's noise scale B (sum of the terms'
    // maxima over the kernel's tilted mass 1 / (1 - |tilt|^2)) and the scores
    // stored by the earlier tilts at this thread's columns
    double lnB = 0.0;
    float bprev[MODE == ROW_LASTT ? E : 1];
    if constexpr (MODE == ROW_LASTT) {
      double B = term_mu * ldexp(1.0, a.expo[a.T - 1]);
      for (int i = 0; i + 1 < a.T; ++i) B += a.tmax[i];
      B /= 1.0 - (a.tilt0 * a.tilt0 + a.tilt1 * a.tilt1);
      lnB = (B > 0.0 && isfinite(B)) ? log(B) : __builtin_huge_val();
#pragma unroll
      for (int q = 0; q < E; ++q) {
        const int cc = 2 * (t + P * (q >> 1)) + (q & 1);
        bprev[q] = (!a.tfirst && col_ok(cc)) ? a.best[rowoff + cc] : -__builtin_huge_valf();
      }
    }
    // last term: the float64 sum of the stored terms 0..T-1 at this thread's
    // columns, in the order of the terms (as a running accumulation would)
    double ps[E];
    if constexpr (LASTLIKE) {
      using V = cplx<R>;
      auto pair = [&](const R *q, int c0) -> V {
        V x = cmake<V>((R)0, (R)0);
        if (!col_ok(c0)) return x;
        if (even_n1) return *reinterpret_cast<const V *>(q + c0);
        x.x = q[c0];
        if (FULL || c0 + 1 < a.n1) x.y = q[c0 + 1];
        return x;
      };
      const R *t0 = a.terms + rowoff;
#pragma unroll
      for (int j = 0; j < E / 2; ++j) {
        const V x = pair(t0, 2 * (t + P * j));
        ps[2 * j] = (double)x.x;
        ps[2 * j + 1] = (double)x.y;
      }
      for (int i0 = 1; i0 < a.T; i0 += 4) {  // four terms of loads in flight
        V q[4][E / 2];
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (i0 + u < a.T) {
#pragma unroll
            for (int j = 0; j < E / 2; ++j)
              q[u][j] = pair(a.terms + (size_t)(i0 + u) * N + rowoff, 2 * (t + P * j));
          }
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (i0 + u < a.T) {
            const double sc = s_sE[i0 + u];
#pragma unroll
            for (int j = 0; j < E / 2; ++j) {
              ps[2 * j] = fma((double)q[u][j].x, sc, ps[2 * j]);
              ps[2 * j + 1] = fma((double)q[u][j].y, sc, ps[2 * j + 1]);
            }
          }
      }
    }
#pragma unroll
    for (int j = 0; j < E / 2; ++j) {
      const int c0 = 2 * (t + P * j);
      R z0 = 0, z1 = 0;
      if (col_ok(c0)) {
        const bool ok1 = FULL || c0 + 1 < a.n1;
        double p0, p1;  // phi after this term
        R m0, m1;       // stored mantissas of this term
        if constexpr (MODE == ROW_PHI0) {
          // phi_0 = sum_k exp(-beta |m - y_k|)  (eq. phi_0Solution, C = 1),
          // or on the FFT route the inverse transform of its spectrum
          double s0 = 0.0, s1 = 0.0;
          if (a.phi0_fft) {
            s0 = (double)v[j].x;
            s1 = (double)v[j].y;
          } else if constexpr (sizeof(R) == 4) {
            const float nb = (float)(-beta * 1.4426950408889634);  // exp(x) = 2^(x log2 e)
            // the tilt's exponent a . x - A of the two columns (0 untilted)
            const float tl0 = tilted ? (float)((ta0 * r + ta1 * c0 - tA) * 1.4426950408889634) : 0.0f;
            const float tl1 = tilted ? tl0 + (float)(ta1 * 1.4426950408889634) : 0.0f;
            float f0 = 0.0f, f1 = 0.0f;
            auto add = [&](int y0, int y1, float lw) {
              const float d0 = (float)(r - y0);
              const float d1 = (float)(c0 - y1);
              const float q0 = d0 * d0;
              f0 += __builtin_amdgcn_exp2f(nb * __builtin_amdgcn_sqrtf(q0 + d1 * d1) + (lw + tl0));
              f1 += __builtin_amdgcn_exp2f(nb * __builtin_amdgcn_sqrtf(q0 + (d1 + 1.0f) * (d1 + 1.0f)) + (lw + tl1));
            };
            // the first kSrcLds sources from LDS, the rest from global memory
            // (two loops, so that no load picks its address space at run time)
            const int nl = min(a.n_src, kSrcLds);
            for (int k = 0; k < nl; ++k) add(s_src[2 * k], s_src[2 * k + 1], (float)s_lw[k]);
            for (int k = nl; k < a.n_src; ++k) add(a.src[2 * k], a.src[2 * k + 1], (float)logw(k));
            s0 = f0;
            s1 = f1;
          } else {
            const double tl0 = tilted ? ta0 * r + ta1 * c0 - tA : 0.0;
            const double tl1 = tilted ? tl0 + ta1 : 0.0;
            auto add = [&](int y0, int y1, double lw) {
              const double d0 = (double)(r - y0);
              const double d1 = (double)(c0 - y1);
              s0 += exp((lw + tl0) - beta * sqrt(d0 * d0 + d1 * d1));
              s1 += exp((lw + tl1) - beta * sqrt(d0 * d0 + (d1 + 1) * (d1 + 1)));
            };
            const int nl = min(a.n_src, kSrcLds);
            for (int k = 0; k < nl; ++k) add(s_src[2 * k], s_src[2 * k + 1], (double)s_lw[k]);
            for (int k = nl; k < a.n_src; ++k) add(a.src[2 * k], a.src[2 * k + 1], logw(k));
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
          if constexpr (MODE == ROW_LASTT) {
            const double ax = ta0 * r + ta1 * c0 - tA;
            nbad += write_S_tilt(a, rowoff + c0, p0, ax, lnB, bprev[2 * j]);
            if (ok1) nbad += write_S_tilt(a, rowoff + c0 + 1, p1, ax + ta1, lnB, bprev[2 * j + 1]);
          } else {
            nbad += write_S(a, rowoff + c0, p0);
            if (a.ck_phi) a.ck_phi[rowoff + c0] = p0;
            if (ok1) {
              nbad += write_S(a, rowoff + c0 + 1, p1);
              if (a.ck_phi) a.ck_phi[rowoff + c0 + 1] = p1;
            }
          }
        } else {
          (void)p0;
          (void)p1;
          if (even_n1)
            *reinterpret_cast<cplx<R> *>(tout + c0) = cmake<cplx<R>>(m0, m1);
          else {
            tout[c0] = m0;
            if (ok1) tout[c0 + 1] = m1;
          }
          // gamma = f^2/ftilde^2 - 1 (exactly 0 where f = ftilde); the
          // first pass forms it from f and keeps it for the later ones
          R g0, g1 = (R)0;
          if constexpr (MODE == ROW_PHI0) {
            const double fa = (double)opr(2 * j, c0, a.f);
            g0 = (R)((fa - ft) * (fa + ft) * inv_ft2);
            a.gam[rowoff + c0] = g0;
            if (ok1) {
              const double fb = (double)opr(2 * j + 1, c0 + 1, a.f);
              g1 = (R)((fb - ft) * (fb + ft) * inv_ft2);
              a.gam[rowoff + c0 + 1] = g1;
            }
          } else {
            g0 = opr(2 * j, c0, a.gam);
            if (ok1) g1 = opr(2 * j + 1, c0 + 1, a.gam);
          }
          z0 = g0 * m0;
          z1 = g1 * m1;
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
    if (tid == 0) a.mu[(size_t)slot * a.nbr + bid] = bm;
  }

  // full gradient: d phi_0 / d beta and d phi_0 / d hbar (through the
  // weights w_k = exp(-s_k / hbar)) at column cc of this row, in float64
  auto dphi0 = [&](int cc, double &dbeta, double &dhbar) {
    dbeta = 0.0;
    dhbar = 0.0;
    for (int k = 0; k < a.n_src; ++k) {
      const double d0 = (double)(r - a.src[2 * k]), d1 = (double)(cc - a.src[2 * k + 1]);
      const double dist = sqrt(d0 * d0 + d1 * d1);
      const double sk = a.src_s ? (double)a.src_s[k] : 0.0;
      const double e = exp(-sk / a.hbar - beta * dist);
      dbeta -= dist * e;
      dhbar += e * sk / (a.hbar * a.hbar);
    }
  };
  // per-work-group slot of the full gradient's partial sums
  auto gslot = [&](int slot) -> double & { return a.gpart[(size_t)slot * a.nbr + bid]; };

  if constexpr (ADJ0) {
    // lambda mantissa (scale 2^-e_lam); a_T = (-1)^T lambda
    const double lam_scale = ldexp(1.0, -elam);
    const double sgnT = (a.T & 1) ? -1.0 : 1.0;
    double ps[FULLG ? 3 : 1] = {};  // S/hbar, a_0 d phi_0/d beta, a_0 d phi_0/d hbar
#pragma unroll
    for (int j0 = 0; j0 < E / 2; j0 += kOpChunk) {
      // the chunk's reads first (see kOpChunk)
      R qf[kOpChunk][2], qs[kOpChunk][2];
      double qp[kOpChunk][2];
#pragma unroll
      for (int jj = 0; jj < kOpChunk; ++jj)
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int cc = 2 * (t + P * (j0 + jj)) + e;
          const bool ok = col_ok(cc);
          qf[jj][e] = ok ? a.f[rowoff + cc] : (R)1;
          qs[jj][e] = ok ? a.dLdS[rowoff + cc] : (R)0;
          qp[jj][e] = ok ? a.ck_phi[rowoff + cc] : 1.0;
        }
#pragma unroll
      for (int jj = 0; jj < kOpChunk; ++jj) {
        const int j = j0 + jj;
        R zz[2] = {(R)0, (R)0};
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int cc = 2 * (t + P * j) + e;
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
        v[j] = cmake<C>(zz[0], zz[1]);
      }
    }
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
    const double gscale = ldexp(1.0, Ei + elam);
    // full gradient: <c_i, gamma phi_{i-1}>, and at term 1 a_0 d phi_0 and
    // dL/dgamma f^2 (mantissa sums; scales applied per work-group)
    double ps[FULLG ? 4 : 1] = {};
    const double sgn_prev = ((term - 1) & 1) ? -1.0 : 1.0;  // (-1)^(i-1)
    const R *mprev = a.ck_terms + (size_t)(term - 1) * N;
    const R *p2 = term > 1 ? a.gam : a.f;  // gamma, or f at the last step
    const bool need3 = term > 1 || FULLG;   // lambda
#pragma unroll
    for (int j0 = 0; j0 < E / 2; j0 += kOpChunk) {
      // the chunk's reads first (see kOpChunk): phi_{i-1}, gamma or f,
      // lambda, the dL/dgamma accumulator
      R q1[kOpChunk][2], q2[kOpChunk][2], q3[kOpChunk][2];
      double qd[kOpChunk][2];
#pragma unroll
      for (int jj = 0; jj < kOpChunk; ++jj)
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int cc = 2 * (t + P * (j0 + jj)) + e;
          const bool ok = col_ok(cc);
          q1[jj][e] = ok ? op1(cc, mprev) : (R)0;
          q2[jj][e] = ok ? op2(cc, p2) : (R)0;
          q3[jj][e] = (ok && need3) ? op3(cc, a.lam) : (R)0;
          qd[jj][e] = (ok && term != a.T) ? opd(cc, a.acc) : 0.0;
        }
#pragma unroll
      for (int jj = 0; jj < kOpChunk; ++jj) {
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
            if constexpr (MODE == ROW_ADJ_B) {
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
    if constexpr (MODE == ROW_ADJ_B) {
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
  }

  // ---- 6. forward real FFT of the new forcing, store the tile --------------
  row_r2c_store<FULL, R, H, E>(v, t, tid, line, lines, twl, tws, tile);
  if constexpr (FULLG) {  // the same spectrum again, for the convolution with dkappa/dbeta
    Tile t2;
    t2.init(a.spec2, row0, a.nb * spec_rb<R>());
    tile_store<FULL>(t2, tid, lines);
  }
}

template <typename R, int MODE, int H, int E>
__device__ __forceinline__ void row_block(const Args2<R> &a, int term, unsigned char *smem_raw,
                                          int bid) {
  const int row0 = bid * row_rpw(H);
  if (row0 + row_rpw(H) <= a.n0 && a.n1 == H)
    row_pass<R, MODE, H, E, true>(a, term, smem_raw, bid);
  else
    row_pass<R, MODE, H, E, false>(a, term, smem_raw, bid);
}

// When a tile holds fewer rows than a spectrum block (RPW < RB), the tiles of
// one block share its 32-byte entries: work-groups are then mapped so that
// neighbouring tiles run on the same XCD, where the halves of an entry meet
// in one L2 instead of being fetched, and written back as partial lines, once
// per XCD (this doubled the row passes' traffic at 2048 columns).  Tiles of
// whole blocks keep the dispatch order, which measures faster for them.
template <typename R, int H> __device__ __forceinline__ int row_tile_id(int b, int nblocks) {
  return row_rpw(H) < spec_rb<R>() ? xcd_tile(b, nblocks) : b;
}

template <typename R, int MODE, int H, int E>
__global__ void __launch_bounds__(row_threads(H, E)) k_row2(Args2<R> a, int term) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  row_block<R, MODE, H, E>(a, term, smem_raw, row_tile_id<R, H>(blockIdx.x, gridDim.x));
}

// The kernel-table row pass (work-groups [0, nbr), into ag's spectrum) and
// the phi_0 row pass (work-groups [nbr, 2 nbr), into ap's) in one launch:
// they depend only on the reduction of f, and side by side their load and
// compute phases overlap on each CU.  ap.own_par is set.
template <typename R, int H, int E>
__global__ void __launch_bounds__(row_threads(H, E)) k_row2_init(Args2<R> ag, Args2<R> ap, int nbr) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int b = blockIdx.x;
  if (b < nbr)
    row_block<R, ROW_GHAT, H, E>(ag, 0, smem_raw, row_tile_id<R, H>(b, nbr));
  else
    row_block<R, ROW_PHI0, H, E>(ap, 0, smem_raw, row_tile_id<R, H>(b - nbr, nbr));
}

// Uneven batch: one launch over the row work-groups of every instance of a
// size class; items[i].begin is the first work-group of instance i.
template <typename R, int MODE, int H, int E>
__global__ void __launch_bounds__(row_threads(H, E)) k_row2_batch(const BatchItem<R> *__restrict__ items,
                                                         int nitems, int term) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int g = row_tile_id<R, H>(blockIdx.x, gridDim.x);
  const int i = find_item(items, nitems, g);
  const Args2<R> a = item_args(items[i]);
  row_block<R, MODE, H, E>(a, term, smem_raw, g - items[i].begin);
}

// Adjoint start: max |lambda| partials (with the twiddle table).
template <typename R>
__global__ void __launch_bounds__(256) k_adj_prep(const R *__restrict__ dLdS,
                                                  const double *__restrict__ phi, long long N,
                                                  double hbar, double *__restrict__ red,
                                                  cplx<R> *__restrict__ tw, int lmax) {
  double mx = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x) {
    const double p = phi[i];
    if (p > 0.0 && isfinite(p)) {
      const double l = fabs(hbar * (double)dLdS[i] / p);
      if (isfinite(l)) mx = l > mx ? l : mx;
    }
  }
  mx = block_max(mx);
  if (threadIdx.x == 0) red[blockIdx.x] = mx;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < lmax; j += gridDim.x * blockDim.x) {
    double s, cs;
    sincospi(2.0 * (double)j / (double)lmax, &s, &cs);
    cplx<R> w;
    w.x = (R)cs;
    w.y = (R)(-s);
    tw[j] = w;
  }
}

// Full gradient: the first grid point (C order) where f equals its minimum
// and its maximum (from the checkpointed scalars), per work-group.
template <typename R>
__global__ void __launch_bounds__(256) k_argext(const R *__restrict__ f, long long N,
                                                const Params *__restrict__ par,
                                                long long *__restrict__ ext) {
  const double lo = par->fmin, hi = par->fmax;
  long long imin = LLONG_MAX, imax = LLONG_MAX;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x) {
    const double v = (double)f[i];
    if (v == lo && i < imin) imin = i;
    if (v == hi && i < imax) imax = i;
  }
  __shared__ long long s[2][4];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const long long a = __shfl_xor(imin, o, 64), b = __shfl_xor(imax, o, 64);
    imin = a < imin ? a : imin;
    imax = b < imax ? b : imax;
  }
  if ((threadIdx.x & 63) == 0) {
    s[0][threadIdx.x >> 6] = imin;
    s[1][threadIdx.x >> 6] = imax;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 4; ++w) {
      imin = s[0][w] < imin ? s[0][w] : imin;
      imax = s[1][w] < imax ? s[1][w] : imax;
    }
    ext[blockIdx.x] = s[0][0] < imin ? s[0][0] : imin;
    ext[gridDim.x + blockIdx.x] = s[1][0] < imax ? s[1][0] : imax;
  }
}

// Full gradient, last step (one work-group): the scalar derivatives
//   dL/dbeta   = G_C + G_B0
//   dL/dhbar   = G_S - (beta / hbar) dL/dbeta + G_H0
//   dL/dftilde = (h / hbar) dL/dbeta - (2 / ftilde^3) G_GF
// and dL/dftilde times a subgradient of ftilde(f) added to dL/df at the
// first minimum and maximum of f (nu: fmin / 2 ftilde and fmax / 2 ftilde;
// sup f: 1 at the maximum; a given ftilde: nothing).  out[0..2] = dL/dhbar,
// dL/dftilde, dL/dbeta (nullable).
template <typename R>
__global__ void __launch_bounds__(256) k_adj_full_finish(const double *__restrict__ gpart, int nbr,
                                                         const long long *__restrict__ ext,
                                                         int next, const Params *__restrict__ par,
                                                         int ft_mode, double h, double hbar,
                                                         R *__restrict__ dLdf,
                                                         double *__restrict__ out) {
  double v[kGradSlots];
#pragma unroll
  for (int k = 0; k < kGradSlots; ++k) {
    double t = 0.0;
    for (int i = threadIdx.x; i < nbr; i += blockDim.x) t += gpart[(size_t)k * nbr + i];
    v[k] = t;
  }
  block_sums_d(v);
  long long imin = LLONG_MAX, imax = LLONG_MAX;
  for (int i = threadIdx.x; i < next; i += blockDim.x) {
    imin = ext[i] < imin ? ext[i] : imin;
    imax = ext[next + i] < imax ? ext[next + i] : imax;
  }
  __shared__ long long s[2][4];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const long long a = __shfl_xor(imin, o, 64), b = __shfl_xor(imax, o, 64);
    imin = a < imin ? a : imin;
    imax = b < imax ? b : imax;
  }
  if ((threadIdx.x & 63) == 0) {
    s[0][threadIdx.x >> 6] = imin;
    s[1][threadIdx.x >> 6] = imax;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int w = 0; w < 4; ++w) {
    imin = s[0][w] < imin ? s[0][w] : imin;
    imax = s[1][w] < imax ? s[1][w] : imax;
  }
  const double beta = par->beta, ft = par->ftilde;
  const double dbeta = v[G_C] + v[G_B0];
  const double dhbar = v[G_S] - beta / hbar * dbeta + v[G_H0];
  const double dft = h / hbar * dbeta - 2.0 / (ft * ft * ft) * v[G_GF];
  if (ft_mode == SWEIK_FT_NU) {
    if (imin != LLONG_MAX) dLdf[imin] = (R)((double)dLdf[imin] + dft * par->fmin / (2.0 * ft));
    if (imax != LLONG_MAX) dLdf[imax] = (R)((double)dLdf[imax] + dft * par->fmax / (2.0 * ft));
  } else if (ft_mode == SWEIK_FT_FMAX) {
    if (imax != LLONG_MAX) dLdf[imax] = (R)((double)dLdf[imax] + dft);
  }
  if (out) {
    out[0] = dhbar;
    out[1] = dft;
    out[2] = dbeta;
    out[3] = 0.0;
  }
}

template <typename R>
__global__ void __launch_bounds__(256) k_fill(R *__restrict__ out, long long N, R v) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x)
    out[i] = v;
}

}  // namespace sweik
