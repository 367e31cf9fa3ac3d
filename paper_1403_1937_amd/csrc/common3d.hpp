// common3d.hpp -- geometry and arguments of the 3D perturbation-series solve.
//
// Grid n0 x n1 x n2 (C order), zero-padded to M0 x M1 x M2 (M_d >= 2 n_d - 1,
// powers of two, Hd = Md / 2).  One correction term (Table 1, steps 9-13)
// is four passes over two spectra:
//   x pass   (axis 2, contiguous) per grid line (i0, i1): inverse real FFT
//            of the previous term, crop, rescale, store the term, form
//            gamma * phi_i, forward real FFT -> s1[i0][i1][k2] (n0 n1 H2
//            complex); the last one sums the stored terms in float64
//   y fwd    (axis 1) per (i0, k2): FFT of the n1 rows zero-padded to M1
//            -> s2[i0][k1][k2]                              (n0 M1 H2 complex;
//            planes i0 are ld2 = M1 H2 + pad apart, so that the axis-0 pass
//            does not step through memory by a large power of two)
//   z conv   (axis 0) per (k1, k2): FFT of the n0 rows zero-padded to M0,
//            product with the kernel spectrum, inverse FFT, first n0 rows
//            back into s2
//   y inv    (axis 1) per (i0, k2): inverse FFT of the M1 rows, first n1
//            rows -> s1
// The real transform along axis 2 samples the odd frequencies
// (k2 + 1/2) / M2: a real line then has exactly H2 independent bins, with no
// separate zero and Nyquist bins.  With at least 2 n2 - 1 padded samples the
// convolution it implies (nega-cyclic) equals the linear convolution, as
// the cyclic one does.  The kernel table is therefore extended nega-cyclically
// along axis 2 (kappa at -d sits at M2 - d with the opposite sign) and evenly
// along axes 0 and 1; its spectrum is real and even in k0 and k1, and is
// stored as the orthant g[k1'][k0'][k2], k0' <= H0, k1' <= H1, k2 < H2,
// pre-scaled by 1 / (4 M0 M1 M2) (the unnormalised transforms' round trips).
#pragma once

#include "common2d.hpp"

namespace sweik {

// X_LAST: the pass after the last convolution (float64 sum of the stored
// terms and the log), its own kernel so that X_TERM is not sized for it.
// X_ADJ0, X_ADJ: the adjoint sweep's start and steps (see x3d.hpp).
// X_DGHAT, X_ADJ0_B, X_ADJ_B: the same for the full gradient (the kernel's
// beta-derivative table, and the sweep with the scalar partial sums).
// X_ETAB, X_SEED, X_PHI0F: phi_0 by FFT (Table 1 steps 1-5): the table of
// exp(-beta |m|), the source grid's transform, and the phi_0 pass that takes
// phi_0 from the inverse transform of their product.
enum XMode {
  X_GHAT = 0, X_PHI0 = 1, X_TERM = 2, X_LAST = 3, X_ADJ0 = 4, X_ADJ = 5,
  X_DGHAT = 6, X_ADJ0_B = 7, X_ADJ_B = 8, X_PHI0F = 9, X_ETAB = 10, X_SEED = 11
};
enum C3Mode { C3_YF = 0, C3_Z = 1, C3_YI = 2, C3_GY = 3, C3_GZ = 4 };

// x pass: one team of P = H2/16 threads per line, 256 threads per group
constexpr int x_lpw(int H) { return kThreads / (H / 16); }
// Line length of an x pass: a 32-lane group holds 32/P lines (P = H/16
// threads per line); float2 lines are spread over the banks.  (The column
// passes, whose 32-lane groups interleave 16 columns two lanes each,
// measured twice the conflicts with spread lines and keep the padded length.)
template <typename R> constexpr int x_line_len(int H) {
  return sizeof(R) == 4 ? lds_line_len_spread(H, H / 16 < 32 ? 32 / (H / 16) : 1) : lds_line_len(H);
}
template <typename R> constexpr size_t x_lds_bytes(int H) {
  // twiddles exp(-2 pi i 2m / 4H), m < H (the odd-frequency transform's
  // even ones; it forms the odd ones from them), the FFT's stage tables and
  // one padded line per team
  return sizeof(R) * 2 *
         ((size_t)H + (size_t)stage_tw_len(H, 16) + (size_t)x_lpw(H) * x_line_len<R>(H));
}
// column passes: CPW neighbouring k2 columns per group, one team of M/16
// threads per column, threads ordered column-fastest so that a wave reads
// CPW contiguous spectrum entries per row.  A work-group's lines hold 8192
// float (4096 double) complex values: about 72 KB of LDS in either
// precision, two work-groups per CU (with 8192 double values one work-group
// filled a CU, and its load, FFT and store phases ran strictly one after
// the other: 256^3 FP64 16.1 -> 13.0 ms; float with 4096 values, four
// work-groups per CU, measured slower, 6.6 -> 7.0 ms)
template <typename R> constexpr int c3_cpw(int M) {
  return (sizeof(R) == 4 ? 8192 : 4096) / M < (sizeof(R) == 4 ? 32 : 16)
             ? (sizeof(R) == 4 ? 8192 : 4096) / M
             : (sizeof(R) == 4 ? 32 : 16);
}
template <typename R> constexpr int c3_threads(int M) { return c3_cpw<R>(M) * (M / 16); }
// static shared memory of an x pass (reductions, scalars, term scales; phi_0
// also holds up to 512 sources and their weights), at least what the compiled
// kernels declare (group segment of the code objects: 1184 bytes for the
// other modes, 512 more for the full gradient's partial sums; phi_0 16640
// in float, 20736 in double), and of a column pass
template <typename R> constexpr size_t x_lds_static(int mode) {
  return mode == X_PHI0 ? (sizeof(R) == 4 ? 17408 : 21504)
         : (mode == X_ADJ0_B || mode == X_ADJ_B) ? 2048 : 1536;
}
constexpr size_t kC3LdsStatic = 512;
template <typename R> constexpr size_t c3_lds_bytes(int M) {
  // the FFT's stage tables and one padded line per column
  return sizeof(R) * 2 * ((size_t)stage_tw_len(M, 16) + (size_t)c3_cpw<R>(M) * lds_line_len(M));
}

template <typename R> struct Args3 {
  int n0, n1, n2;
  int M0, M1, M2, H0, H1, H2;
  int nlines;    // n0 n1 grid lines along axis 2
  long long ld2; // plane stride of s2 (M1 H2 plus a pad that breaks the power-of-two stride)
  int nbx;       // x-pass work-groups
  int lmax_log;  // log2 of the twiddle table length
  int T, n_src, ft_mode;
  double ftilde_given, h, hbar;
  const R *f;
  const int *src;
  const R *src_s;  // nullable: S at the sources
  R *S;
  Params *par;
  double *red;     // kRedBlocks x 3
  double *mu;      // (T+1) x nbx partial max |m_i|
  double *mu_red;  // T+1 reduced maxima
  int *expo;       // T+1 exponents
  const cplx<R> *tw;
  cplx<R> *s1, *s2;
  cplx<R> *s1o;    // where the y inverse pass writes (s1, or the full gradient's s1b)
  cplx<R> *s1b;    // full gradient: dkappa/dbeta (*) a_i after the y inverse pass
  R *g;            // kernel spectrum orthant
  R *terms;        // T x N mantissas of phi_0..phi_{T-1} (the checkpoint's when kept)
  R *gam;          // N
  sweik_info *info;
  // checkpoint of a solve for its adjoint (null when none is kept)
  int *ck_expo;    // T+1 exponents of the stored terms
  double *ck_phi;  // N, phi in float64
  // adjoint
  const R *dLdS;
  R *dLdf;
  R *lam;          // N, lambda mantissas (scale 2^expo[0])
  double *acc;     // N, dL/dgamma in float64
  double *gpart;   // full gradient: kGradSlots x nbx per-work-group partial sums
};

}  // namespace sweik
