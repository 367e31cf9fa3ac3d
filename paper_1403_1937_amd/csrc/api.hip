// api.hip -- C ABI of the gfx950 eikonal solver: validation, plans, workspace
// layout and the launch sequence of a solve.  See include/sweik.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <tuple>
#include <vector>

#include "launch2d.hpp"
#include "launch3d.hpp"
#include "plan.hpp"

using namespace sweik;

namespace {

// HIP resources (streams, events, pinned host buffers, graph executables)
// created by the library so far: solves and batch solves create none.
std::atomic<long long> g_resources{0};
template <typename T> T counted(T err) {
  if (err == hipSuccess) g_resources.fetch_add(1, std::memory_order_relaxed);
  return err;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }


int64_t next_pow2(int64_t m) {
  int64_t p = 1;
  while (p < m) p <<= 1;
  return p;
}
int ilog2(int64_t x) {
  int l = 0;
  while ((int64_t(1) << l) < x) ++l;
  return l;
}

}  // namespace

namespace sweik {

thread_local char g_last_error[256] = "";

void note_launch_error(const char *family, int mode, int length, int E, hipError_t err) {
  std::snprintf(g_last_error, sizeof(g_last_error), "%s (mode %d, length %d, %d elements per thread): %s",
                family, mode, length, E, hipGetErrorName(err));
}

// Chebyshev coefficients of sqrt(x) e^x K0(x) and sqrt(x) e^x K1(x) on
// x >= 2 in t = 4/x - 1, from their values at the Chebyshev points
// (discrete cosine transform).
const ChebK0 &bessel_cheb_k0() {
  static const ChebK0 tab = [] {
    ChebK0 t;
    const int n = 40;
    const double pi = 3.14159265358979323846;
    double g0[n], g1[n];
    for (int j = 0; j < n; ++j) {
      const double tj = std::cos(pi * (j + 0.5) / n);
      const double x = 4.0 / (tj + 1.0);
      g0[j] = std::sqrt(x) * k_laplace_scaled(x, 0);
      g1[j] = std::sqrt(x) * k_laplace_scaled(x, 1);
    }
    for (int k = 0; k < kChebK0; ++k) {
      double s0 = 0.0, s1 = 0.0;
      for (int j = 0; j < n; ++j) {
        const double c = std::cos(pi * k * (j + 0.5) / n);
        s0 += g0[j] * c;
        s1 += g1[j] * c;
      }
      t.c[k] = (k == 0 ? 1.0 : 2.0) * s0 / n;
      t.c32[k] = (float)t.c[k];
      t.c1[k] = (k == 0 ? 1.0 : 2.0) * s1 / n;
    }
    return t;
  }();
  return tab;
}

sweik_status validate_problem(const sweik_problem *p) {
  if (!p) return SWEIK_EINVAL;
  if (p->ndim != 2 && p->ndim != 3) return SWEIK_EINVAL;
  for (int d = 0; d < p->ndim; ++d)
    if (p->dims[d] < 2) return SWEIK_EINVAL;
  if (!(p->h > 0) || !(p->hbar > 0) || !std::isfinite(p->h) || !std::isfinite(p->hbar))
    return SWEIK_EINVAL;
  if (p->T < 0 || p->T > SWEIK_MAX_TERMS) return SWEIK_EINVAL;
  if (p->n_src < 1) return SWEIK_EINVAL;
  if (p->prec != SWEIK_F32_SCALED && p->prec != SWEIK_F64) return SWEIK_EINVAL;
  if (p->ft_mode != SWEIK_FT_NU && p->ft_mode != SWEIK_FT_FMAX && p->ft_mode != SWEIK_FT_GIVEN)
    return SWEIK_EINVAL;
  if (p->ft_mode == SWEIK_FT_GIVEN && !(p->ftilde > 0 && std::isfinite(p->ftilde)))
    return SWEIK_EINVAL;
  return SWEIK_OK;
}

// Process-wide schedule table filled by the autotuner: (pass family,
// length, precision) -> elements per team thread.
enum { SCHED_ROW2 = 0, SCHED_COL2 = 1 };
std::mutex g_sched_mu;
std::map<std::tuple<int, int, int>, int> g_sched;

int sched_lookup(int fam, int len, int prec, int dflt) {
  std::lock_guard<std::mutex> lk(g_sched_mu);
  auto it = g_sched.find(std::make_tuple(fam, len, prec));
  return it == g_sched.end() ? dflt : it->second;
}
void sched_store(int fam, int len, int prec, int e) {
  std::lock_guard<std::mutex> lk(g_sched_mu);
  g_sched[std::make_tuple(fam, len, prec)] = e;
}

// Sources beyond which a 2D plan takes the FFT route of phi_0: at 1024^2 the
// direct sum costs about 1.4 us per source, the route about 80 us.
constexpr int kPhi0FftSources = 64;
// The same for a 3D plan, per precision: at 256^3 the direct sum costs about
// 3.4 us per source in float32 and 32 us in float64, the route about 0.43 ms
// and 0.97 ms.
constexpr int kPhi0FftSources3F32 = 128, kPhi0FftSources3F64 = 32;

// Schedule and workspace layout of a 2D problem.
sweik_status plan2d(sweik_plan_s *pl) {
  const sweik_problem &p = pl->p;
  const int esz = p.prec == SWEIK_F64 ? 8 : 4;
  const int csz = 2 * esz;
  Geo2 &g = pl->g2;
  g.n0 = (int)p.dims[0];
  g.n1 = (int)p.dims[1];
  const int64_t M0 = std::max<int64_t>(64, next_pow2(2 * p.dims[0] - 1));
  const int64_t M1 = std::max<int64_t>(64, next_pow2(2 * p.dims[1] - 1));
  if (M0 > 8192 || M1 > 16384) return SWEIK_EUNSUPPORTED;
  g.M0 = (int)M0;
  g.H0 = (int)(M0 / 2);
  g.ldg = g.H0 + 1;
  g.H1 = (int)(M1 / 2);
  g.ldk = g.H1;  // spectral columns; column 0 carries bins 0 and H1
  if (g.H1 > 8192 || g.H1 < 32) return SWEIK_EUNSUPPORTED;
  g.RB = p.prec == SWEIK_F64 ? spec_rb<double>() : spec_rb<float>();
  g.nb = (g.n0 + g.RB - 1) / g.RB;
  // every pass must fit the work-group LDS limit
  const bool f64 = p.prec == SWEIK_F64;
  for (int mode = ROW_GHAT; mode <= ROW_LASTT; ++mode) {
    if (!(f64 ? row_fits<double>(g.H1, mode) : row_fits<float>(g.H1, mode)))
      return SWEIK_EUNSUPPORTED;
  }
  if (!(f64 ? col_fits<double>(g.M0) : col_fits<float>(g.M0))) return SWEIK_EUNSUPPORTED;
  g.rpw = row_rpw(g.H1);
  g.cpw = col_cpw(g.M0);
  const int spec_rows = g.nb * g.RB;
  g.nbr = (spec_rows + g.rpw - 1) / g.rpw;
  g.ncw = (g.ldk + g.cpw - 1) / g.cpw;
  g.lmax = (int)std::max(M0, M1);
  g.lmax_log = ilog2(g.lmax);
  g.erow = sched_lookup(SCHED_ROW2, g.H1, p.prec, 16);
  if (g.H1 > 4096) g.erow = 16;  // 8192-point rows: radix 16 only
  g.ecol = sched_lookup(SCHED_COL2, g.M0, p.prec, 16);
  if (!(f64 ? col_ok<double>(g.M0, g.ecol) : col_ok<float>(g.M0, g.ecol))) g.ecol = 16;
  // phi_0 by FFT (Table 1 steps 1-5) when the direct sum over the sources
  // costs more than the extra kernel spectrum and convolution
  g.phi0_fft = p.n_src > kPhi0FftSources ? 1 : 0;
  pl->padded[0] = M0;
  pl->padded[1] = M1;
  pl->padded[2] = 1;

  // workspace
  const int64_t N = (int64_t)g.n0 * g.n1;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  Layout &L = pl->ws;
  L.par = take(sizeof(Params));
  L.red = take(sizeof(double) * 3 * kRedBlocks);
  L.expo = take(sizeof(int) * (SWEIK_MAX_TERMS + 1));
  L.mu = take(sizeof(double) * (size_t)(p.T + 1) * g.nbr);
  L.tw = take((size_t)csz * g.lmax);
  L.g = take((size_t)esz * (g.ldk + 1) * g.ldg);
  L.g0 = take((size_t)esz * (g.ldk + 1) * g.ldg);  // spectrum of exp(-beta |m|) (phi_0 by FFT)
  L.spec = take((size_t)csz * g.nb * g.ldk * g.RB);
  L.spec0 = take((size_t)csz * g.nb * g.ldk * g.RB);  // kernel-table rows of the paired pass
  L.acc = take(sizeof(double) * N);
  L.terms = take((size_t)esz * N * (size_t)p.T);
  L.lam = take((size_t)esz * N);
  L.gam = take((size_t)esz * N);
  L.total = off;
  L.fg_spec2 = take((size_t)csz * g.nb * g.ldk * g.RB);
  L.fg_part = take(sizeof(double) * kGradSlots * g.nbr);
  L.fg_ext = take(sizeof(long long) * 2 * kRedBlocks);
  L.fg_total = off;
  off = 0;
  L.ck_expo = take(sizeof(int) * (SWEIK_MAX_TERMS + 1));
  L.ck_par = take(sizeof(Params));
  L.ck_g = take((size_t)esz * (g.ldk + 1) * g.ldg);
  L.ck_phi = take(sizeof(double) * N);
  L.ck_terms = take((size_t)esz * N * (size_t)p.T);
  L.ck_total = off;
  return SWEIK_OK;
}

template <typename R>
Args2<R> make_args2(const sweik_plan_s *pl, const void *f, const int32_t *src, void *S,
                    void *ws, void *ckpt, sweik_info *info) {
  const Geo2 &g = pl->g2;
  const sweik_problem &p = pl->p;
  const Layout &L = pl->ws;
  char *w = (char *)ws;
  Args2<R> a;
  a.n0 = g.n0;
  a.n1 = g.n1;
  a.H1 = g.H1;
  a.ldk = g.ldk;
  a.M0 = g.M0;
  a.H0 = g.H0;
  a.ldg = g.ldg;
  a.nb = g.nb;
  a.nbr = g.nbr;
  a.ncw = g.ncw;
  a.lmax_log = g.lmax_log;
  a.T = p.T;
  a.n_src = p.n_src;
  a.ft_mode = p.ft_mode;
  a.table = 0;
  a.phi0_fft = 0;
  a.own_par = 0;
  a.ftilde_given = p.ftilde;
  a.h = p.h;
  a.hbar = p.hbar;
  a.f = (const R *)f;
  a.src = src;
  a.src_s = nullptr;
  a.S = (R *)S;
  a.par = (Params *)(w + L.par);
  a.red = (double *)(w + L.red);
  a.mu = (double *)(w + L.mu);
  a.expo = (int *)(w + L.expo);
  a.tw = (const cplx<R> *)(w + L.tw);
  a.spec = (cplx<R> *)(w + L.spec);
  a.g = (R *)(w + L.g);
  a.acc = (double *)(w + L.acc);
  a.lam = (R *)(w + L.lam);
  a.gam = (R *)(w + L.gam);
  a.k0tab = bessel_cheb_k0();
  a.dLdS = nullptr;
  a.dLdf = nullptr;
  a.spec2 = nullptr;
  a.gpart = nullptr;
  a.tilt0 = 0.0;
  a.tilt1 = 0.0;
  a.tsign = 1;
  a.tfirst = 0;
  a.tlast = 0;
  a.gc = nullptr;
  a.spec_neg = nullptr;
  a.best = nullptr;
  a.tmax = nullptr;
  a.info = info;
  char *c = (char *)ckpt;
  if (c) {  // the kernel spectrum and scalars live in the checkpoint
    a.par = (Params *)(c + L.ck_par);
    a.g = (R *)(c + L.ck_g);
  }
  a.ck_expo = c ? (int *)(c + L.ck_expo) : nullptr;
  a.ck_phi = c ? (double *)(c + L.ck_phi) : nullptr;
  a.ck_terms = c ? (R *)(c + L.ck_terms) : nullptr;
  // the forward stores its terms in the checkpoint when one is kept
  a.terms = c ? a.ck_terms : (R *)(w + L.terms);
  return a;
}

// Optional per-kernel timing: one event on the solve's stream before the
// first kernel and one after every kernel, so that each interval covers one
// kernel and the dispatch gap before it; durations are summed per class.
struct KernelTimer {
  static constexpr int kMax = 4 * (SWEIK_MAX_TERMS + 2) + 8;
  hipEvent_t ev[kMax + 1];
  int cls[kMax];
  int n = 0;
  bool ok = true;
  KernelTimer() {
    for (int i = 0; i <= kMax; ++i)
      if (counted(hipEventCreateWithFlags(&ev[i], hipEventDisableSystemFence)) != hipSuccess)
        ok = false;
  }
  ~KernelTimer() {
    for (int i = 0; i <= kMax; ++i) (void)hipEventDestroy(ev[i]);
  }
};

template <typename R>
sweik_status enqueue2d(const sweik_plan_s *pl, const void *f, const int32_t *src, void *S,
                       void *ws, void *ckpt, hipStream_t st, sweik_info *info,
                       KernelTimer *tm = nullptr, const void *src_s = nullptr) {
  const Geo2 &g = pl->g2;
  Args2<R> a = make_args2<R>(pl, f, src, S, ws, ckpt, info);
  a.src_s = (const R *)src_s;
  const long long N = (long long)g.n0 * g.n1;
  hipError_t err = hipSuccess;
  auto launch = [&](int cls, auto &&fn) {
    if (err != hipSuccess) return;
    if (tm && tm->n < KernelTimer::kMax) {
      if (tm->n == 0) (void)hipEventRecord(tm->ev[0], st);
      err = fn();
      (void)hipEventRecord(tm->ev[tm->n + 1], st);
      tm->cls[tm->n++] = cls;
    } else {
      err = fn();
    }
  };
  const dim3 grow(g.nbr), gcol(g.ncw);
  launch(SWEIK_KC_PREP, [&] { return launch_prep<R>((const R *)f, N, a.red, (cplx<R> *)a.tw, g.lmax, st); });
  // the kernel-table and phi_0 row passes in one launch where two of its
  // work-groups fit a CU (the timed variant keeps them apart, one class each)
  const bool paired = tm == nullptr && !g.phi0_fft && pl->p.T > 0 && row_init_pairs<R>(g.H1);
  if (paired) {
    Args2<R> ag = a, ap = a;
    ag.spec = (cplx<R> *)((char *)ws + pl->ws.spec0);
    ap.own_par = 1;
    launch(SWEIK_KC_GHAT_ROW, [&] { return launch_row2_init<R>(g.H1, g.erow, g.nbr, st, ag, ap); });
    launch(SWEIK_KC_GHAT_COL, [&] { return launch_col2<R>(COL_GHAT, g.M0, g.ecol, gcol, st, ag); });
  } else {
    launch(SWEIK_KC_GHAT_ROW, [&] { return launch_row2<R>(ROW_GHAT, g.H1, g.erow, grow, st, a, 0); });
    launch(SWEIK_KC_GHAT_COL, [&] { return launch_col2<R>(COL_GHAT, g.M0, g.ecol, gcol, st, a); });
  }
  if (g.phi0_fft) {
    // Table 1 steps 1-5: spectrum of exp(-beta |m|), transform of the source
    // grid (weights exp(-s_k/hbar)), product, inverse in the phi_0 pass
    Args2<R> a0 = a;
    a0.table = 1;
    a0.g = (R *)((char *)ws + pl->ws.g0);
    const long long N2 = (long long)g.n0 * g.n1;
    launch(SWEIK_KC_PHI0_FFT, [&] { return launch_row2<R>(ROW_GHAT, g.H1, g.erow, grow, st, a0, 0); });
    launch(SWEIK_KC_PHI0_FFT, [&] { return launch_col2<R>(COL_GHAT, g.M0, g.ecol, gcol, st, a0); });
    launch(SWEIK_KC_PHI0_FFT, [&] { return launch_fill<R>(a.gam, N2, (R)0, st); });
    launch(SWEIK_KC_PHI0_FFT, [&] {
      return launch_seed_scatter<R>(a.gam, src, (const R *)src_s, pl->p.n_src, pl->p.hbar, g.n0,
                                    g.n1, 0, st);
    });
    launch(SWEIK_KC_PHI0_FFT, [&] { return launch_row2<R>(ROW_SEED, g.H1, g.erow, grow, st, a0, 0); });
    launch(SWEIK_KC_PHI0_FFT, [&] { return launch_col2<R>(COL_CONV, g.M0, g.ecol, gcol, st, a0); });
    a.phi0_fft = 1;
  }
  if (!paired)
    launch(SWEIK_KC_PHI0_ROW, [&] { return launch_row2<R>(ROW_PHI0, g.H1, g.erow, grow, st, a, 0); });
  for (int i = 1; i <= pl->p.T; ++i) {
    launch(SWEIK_KC_CONV_COL, [&] { return launch_col2<R>(COL_CONV, g.M0, g.ecol, gcol, st, a); });
    const bool lastp = i == pl->p.T;
    launch(lastp ? SWEIK_KC_LAST_ROW : SWEIK_KC_TERM_ROW, [&] {
      return launch_row2<R>(lastp ? ROW_LAST : ROW_TERM, g.H1, g.erow, grow, st, a, i);
    });
  }
  return err == hipSuccess ? SWEIK_OK : SWEIK_EDEVICE;
}

// Workspace of a tilted solve with n_tilt tilts: the plan's solve workspace
// (shared by the tilts: reductions of f, twiddles, gamma, and the float64
// accumulator of the per-source split), then one slice per tilt, then the
// tilts' three work lists.
struct TiltWs {
  TiltSlice sl;
  size_t slices, items, total;
};
TiltWs tilt_ws(const sweik_plan_s *pl, int n_tilt) {
  const Geo2 &g = pl->g2;
  const sweik_problem &p = pl->p;
  const size_t esz = p.prec == SWEIK_F64 ? 8 : 4, csz = 2 * esz;
  const size_t N = (size_t)g.n0 * g.n1;
  TiltWs t;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  t.sl.spec = take(csz * g.nb * g.ldk * g.RB);
  t.sl.spec_neg = take(csz * g.nb * g.ldk * g.RB);
  t.sl.gc = take(csz * (g.ldk + 1) * g.M0);
  t.sl.terms = take(esz * N * (size_t)p.T);
  t.sl.mu = take(sizeof(double) * (size_t)(p.T + 1) * g.nbr);
  t.sl.expo = take(sizeof(int) * (SWEIK_MAX_TERMS + 1));
  t.sl.tmax = take(sizeof(double) * (size_t)(p.T + 2));
  t.sl.S = take(esz * N);
  t.sl.best = take(sizeof(float) * N);
  t.sl.bytes = off;
  t.slices = align256(pl->ws.total);
  t.items = align256(t.slices + (size_t)n_tilt * t.sl.bytes);
  const size_t item = p.prec == SWEIK_F64 ? sizeof(BatchItem<double>) : sizeof(BatchItem<float>);
  t.total = align256(t.items + 3 * (size_t)n_tilt * item);
  return t;
}

// Far-field stabilised solve (2D): the series of Table 1 once per tilt a =
// beta (tilts[2d], tilts[2d+1]), each on phi_i exp(a . x) with the kernel
// kappa(m) exp(a . m) (the same convolution, exactly, in tilted variables).
// The tilts run side by side: every pass is one launch over the work-groups
// of all tilts (an uneven batch whose work lists k_tilt_items forms on the
// device), each tilt in its own workspace slice; per point k_tilt_select
// then keeps the tilt whose rounding noise is smallest relative to its
// value.  The tilted passes run with radix-16 teams; the term passes use the
// plan's row schedule.  With per_source the solve is split over the sources
// (one tilted solve per source, its own tilt offsets), summed as phi = sum_k
// exp(-S_k / hbar) in float64 (acc, the adjoint's accumulator, is free in a
// forward solve); the count of points without a positive phi then comes
// from the sum.
template <typename R>
sweik_status enqueue2d_tilted(const sweik_plan_s *pl, const void *f, const int32_t *src,
                              const void *src_s, void *S, const double *tilts, int n_tilt,
                              bool per_source, void *ws, hipStream_t st, sweik_info *info) {
  const Geo2 &g = pl->g2;
  const TiltWs tw = tilt_ws(pl, n_tilt);
  unsigned char *w = (unsigned char *)ws;
  Args2<R> a = make_args2<R>(pl, f, src, S, ws, nullptr, info);
  a.src_s = (const R *)src_s;
  TiltTable tt;
  for (int d = 0; d < SWEIK_MAX_TILTS; ++d) {
    tt.t[2 * d] = d < n_tilt ? tilts[2 * d] : 0.0;
    tt.t[2 * d + 1] = d < n_tilt ? tilts[2 * d + 1] : 0.0;
  }
  unsigned char *slices = w + tw.slices;
  BatchItem<R> *rows = reinterpret_cast<BatchItem<R> *>(w + tw.items);
  BatchItem<R> *negs = rows + n_tilt, *cols = negs + n_tilt;
  const long long N = (long long)g.n0 * g.n1;
  const int nrow = n_tilt * g.nbr, ncol = n_tilt * g.ncw;
  hipError_t err = launch_prep<R>((const R *)f, N, a.red, (cplx<R> *)a.tw, g.lmax, st);
  const int nsrc = pl->p.n_src;
  const int parts = per_source && nsrc > 1 ? nsrc : 1;
  if (parts > 1) a.n_src = 1;
  for (int k = 0; k < parts && err == hipSuccess; ++k) {
    if (parts > 1) {
      a.src = src + 2 * k;
      a.src_s = src_s ? (const R *)src_s + k : nullptr;
    }
    err = launch_tilt_items<R>(a, tt, n_tilt, slices, tw.sl, rows, negs, cols, st);
    // the tilted kernels' spectra: table rows m0 >= 0 into spec, m0 <= 0
    // into spec_neg, then the complex column transforms into gc
    if (err == hipSuccess) err = launch_row2_batch<R>(ROW_GHATT, g.H1, 16, nrow, st, rows, n_tilt, 0);
    if (err == hipSuccess) err = launch_row2_batch<R>(ROW_GHATT, g.H1, 16, nrow, st, negs, n_tilt, 0);
    if (err == hipSuccess) err = launch_col2_batch<R>(COL_GHATC, g.M0, 16, ncol, st, cols, n_tilt);
    if (err == hipSuccess)
      err = launch_row2_batch<R>(ROW_PHI0, g.H1, g.erow, nrow, st, rows, n_tilt, 0);
    for (int i = 1; i <= pl->p.T && err == hipSuccess; ++i) {
      err = launch_col2_batch<R>(COL_CONVC, g.M0, 16, ncol, st, cols, n_tilt);
      const bool lastp = i == pl->p.T;
      if (err == hipSuccess)
        err = launch_row2_batch<R>(lastp ? ROW_LASTT : ROW_TERM, g.H1, lastp ? 16 : g.erow, nrow,
                                   st, rows, n_tilt, i);
    }
    if (err == hipSuccess)
      err = launch_tilt_select<R>((R *)S, slices, tw.sl, n_tilt, N, parts == 1, info, st);
    if (parts > 1 && err == hipSuccess)
      err = launch_source_lse<R>((R *)S, a.acc, N, pl->p.hbar, k == 0, k == parts - 1, info, st);
  }
  if (err != hipSuccess) return SWEIK_EDEVICE;
  return SWEIK_OK;
}

template <typename R>
sweik_status enqueue2d_adjoint(const sweik_plan_s *pl, const void *f, const int32_t *src,
                               const void *ckpt, const void *dLdS, void *dLdf, void *ws,
                               hipStream_t st) {
  const Geo2 &g = pl->g2;
  Args2<R> a = make_args2<R>(pl, f, src, nullptr, ws, const_cast<void *>(ckpt), nullptr);
  a.dLdS = (const R *)dLdS;
  a.dLdf = (R *)dLdf;
  const long long N = (long long)g.n0 * g.n1;
  if (pl->p.T == 0)  // ftilde fixed: no term depends on f
    return launch_fill<R>((R *)dLdf, N, (R)0, st) == hipSuccess ? SWEIK_OK : SWEIK_EDEVICE;
  const dim3 grow(g.nbr), gcol(g.ncw);
  hipError_t err = launch_adj_prep<R>((const R *)dLdS, (const double *)a.ck_phi, N,
                                      pl->p.hbar, a.red, (cplx<R> *)a.tw, g.lmax, st);
  if (err == hipSuccess) err = launch_row2<R>(ROW_ADJ0, g.H1, g.erow, grow, st, a, pl->p.T);
  for (int i = pl->p.T; i >= 1 && err == hipSuccess; --i) {
    err = launch_col2<R>(COL_CONV, g.M0, g.ecol, gcol, st, a);
    if (err == hipSuccess) err = launch_row2<R>(ROW_ADJ, g.H1, g.erow, grow, st, a, i);
  }
  return err == hipSuccess ? SWEIK_OK : SWEIK_EDEVICE;
}


// Full gradient (2D): the adjoint sweep of enqueue2d_adjoint, with every
// convolution of a_i done twice (with the kernel and with its
// beta-derivative), the scalar partial sums in the row passes, then the
// argmin / argmax of f and the scalar derivatives.
template <typename R>
sweik_status enqueue2d_adjoint_full(const sweik_plan_s *pl, const void *f, const int32_t *src,
                                    const void *src_s, const void *ckpt, const void *dLdS,
                                    void *dLdf, double *grads, void *ws, hipStream_t st) {
  const Geo2 &g = pl->g2;
  const Layout &L = pl->ws;
  char *w = (char *)ws;
  Args2<R> a = make_args2<R>(pl, f, src, nullptr, ws, const_cast<void *>(ckpt), nullptr);
  a.src_s = (const R *)src_s;
  a.dLdS = (const R *)dLdS;
  a.dLdf = (R *)dLdf;
  a.spec2 = (cplx<R> *)(w + L.fg_spec2);
  a.gpart = (double *)(w + L.fg_part);
  const long long N = (long long)g.n0 * g.n1;
  const dim3 grow(g.nbr), gcol(g.ncw);
  // the same arguments with the beta-derivative convolution's spectra
  Args2<R> ab = a;
  ab.spec = a.spec2;
  ab.g = (R *)(w + L.g0);
  hipError_t err = launch_adj_prep<R>((const R *)dLdS, (const double *)a.ck_phi, N,
                                      pl->p.hbar, a.red, (cplx<R> *)a.tw, g.lmax, st);
  if (pl->p.T == 0) {
    if (err == hipSuccess) err = launch_fill<R>((R *)dLdf, N, (R)0, st);
    if (err == hipSuccess) err = launch_row2<R>(ROW_ADJ0_B, g.H1, g.erow, grow, st, a, 0);
  } else {
    // spectrum of dkappa/dbeta (rows into spec2, columns into g0)
    if (err == hipSuccess) err = launch_row2<R>(ROW_DGHAT, g.H1, g.erow, grow, st, ab, 0);
    if (err == hipSuccess) err = launch_col2<R>(COL_GHAT, g.M0, g.ecol, gcol, st, ab);
    if (err == hipSuccess) err = launch_row2<R>(ROW_ADJ0_B, g.H1, g.erow, grow, st, a, pl->p.T);
    for (int i = pl->p.T; i >= 1 && err == hipSuccess; --i) {
      err = launch_col2<R>(COL_CONV, g.M0, g.ecol, gcol, st, a);
      if (err == hipSuccess) err = launch_col2<R>(COL_CONV, g.M0, g.ecol, gcol, st, ab);
      if (err == hipSuccess) err = launch_row2<R>(ROW_ADJ_B, g.H1, g.erow, grow, st, a, i);
    }
  }
  if (err == hipSuccess)
    err = launch_adj_full_finish<R>((const R *)f, N, a.par, a.gpart, g.nbr,
                                    (long long *)(w + L.fg_ext), pl->p.ft_mode, pl->p.h,
                                    pl->p.hbar, (R *)dLdf, grads, st);
  return err == hipSuccess ? SWEIK_OK : SWEIK_EDEVICE;
}

// Extra complex elements between the planes of the 3D spectrum s2.
constexpr long long kS2PlanePad = 16;

// Schedule and workspace layout of a 3D problem.
sweik_status plan3d(sweik_plan_s *pl) {
  const sweik_problem &p = pl->p;
  const bool f64 = p.prec == SWEIK_F64;
  const int esz = f64 ? 8 : 4;
  const int csz = 2 * esz;
  Geo3 &g = pl->g3;
  int64_t M[3];
  for (int d = 0; d < 3; ++d) {
    M[d] = std::max<int64_t>(64, next_pow2(2 * p.dims[d] - 1));
    if (M[d] > 2048) return SWEIK_EUNSUPPORTED;
  }
  g.n0 = (int)p.dims[0];
  g.n1 = (int)p.dims[1];
  g.n2 = (int)p.dims[2];
  g.M0 = (int)M[0];
  g.M1 = (int)M[1];
  g.M2 = (int)M[2];
  g.H0 = g.M0 / 2;
  g.H1 = g.M1 / 2;
  g.H2 = g.M2 / 2;
  const size_t xl = f64 ? x_lds_bytes<double>(g.H2) : x_lds_bytes<float>(g.H2);
  const size_t c0 = f64 ? c3_lds_bytes<double>(g.M0) : c3_lds_bytes<float>(g.M0);
  const size_t c1 = f64 ? c3_lds_bytes<double>(g.M1) : c3_lds_bytes<float>(g.M1);
  const size_t xs = f64 ? x_lds_static<double>(X_PHI0) : x_lds_static<float>(X_PHI0);
  if (xl + xs > kLdsDevice || c0 + kC3LdsStatic > kLdsDevice ||
      c1 + kC3LdsStatic > kLdsDevice)
    return SWEIK_EUNSUPPORTED;
  g.nlines = g.n0 * g.n1;
  g.nbx = (g.nlines + x_lpw(g.H2) - 1) / x_lpw(g.H2);
  g.ncb0 = g.H2 / (f64 ? c3_cpw<double>(g.M0) : c3_cpw<float>(g.M0));
  g.ncb1 = g.H2 / (f64 ? c3_cpw<double>(g.M1) : c3_cpw<float>(g.M1));
  pl->g2.erow = pl->g2.ecol = 16;  // the 3D passes have one radix schedule
  pl->g2.phi0_fft = p.n_src > (f64 ? kPhi0FftSources3F64 : kPhi0FftSources3F32) ? 1 : 0;
  g.lmax = std::max(2 * g.M2, std::max(g.M0, g.M1));
  g.lmax_log = ilog2(g.lmax);
  for (int d = 0; d < 3; ++d) pl->padded[d] = M[d];

  const int64_t N = (int64_t)g.n0 * g.n1 * g.n2;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  Layout &L = pl->ws;
  L.par = take(sizeof(Params));
  L.red = take(sizeof(double) * 3 * kRedBlocks);
  L.expo = take(sizeof(int) * (SWEIK_MAX_TERMS + 1));
  L.mu = take(sizeof(double) * (size_t)(p.T + 1) * g.nbx);
  L.mu_red = take(sizeof(double) * (size_t)(p.T + 1));
  L.tw = take((size_t)csz * g.lmax);
  L.g = take((size_t)esz * (g.H1 + 1) * (g.H0 + 1) * g.H2);
  // spectrum of exp(-beta |m|) (phi_0 by FFT), or of dkappa/dbeta (full gradient)
  L.g0 = take((size_t)esz * (g.H1 + 1) * (g.H0 + 1) * g.H2);
  L.spec = take((size_t)csz * g.nlines * g.H2);
  g.ld2 = (long long)g.M1 * g.H2 + kS2PlanePad;
  L.s2 = take((size_t)csz * g.n0 * (size_t)g.ld2);
  L.acc = take(sizeof(double) * N);  // the adjoint's dL/dgamma
  L.terms = take((size_t)esz * N * (size_t)p.T);
  L.gam = take((size_t)esz * N);
  L.lam = take((size_t)esz * N);
  L.total = off;
  // full gradient: the second x-pass spectrum, the per-work-group partial
  // sums and the argmin / argmax partials
  L.fg_spec2 = take((size_t)csz * g.nlines * g.H2);
  L.fg_part = take(sizeof(double) * kGradSlots * g.nbx);
  L.fg_ext = take(sizeof(long long) * 2 * kRedBlocks);
  L.fg_total = off;
  // checkpoint of a solve for its adjoint: scalars, kernel spectrum, term
  // exponents, phi in float64 and the stored terms
  off = 0;
  L.ck_expo = take(sizeof(int) * (SWEIK_MAX_TERMS + 1));
  L.ck_par = take(sizeof(Params));
  L.ck_g = take((size_t)esz * (g.H1 + 1) * (g.H0 + 1) * g.H2);
  L.ck_phi = take(sizeof(double) * N);
  L.ck_terms = take((size_t)esz * N * (size_t)p.T);
  L.ck_total = off;
  return SWEIK_OK;
}

template <typename R>
Args3<R> make_args3(const sweik_plan_s *pl, const void *f, const int32_t *src, void *S,
                    void *ws, sweik_info *info, void *ckpt = nullptr) {
  const Geo3 &g = pl->g3;
  const sweik_problem &p = pl->p;
  const Layout &L = pl->ws;
  char *w = (char *)ws;
  Args3<R> a;
  a.n0 = g.n0;
  a.n1 = g.n1;
  a.n2 = g.n2;
  a.M0 = g.M0;
  a.M1 = g.M1;
  a.M2 = g.M2;
  a.H0 = g.H0;
  a.H1 = g.H1;
  a.H2 = g.H2;
  a.nlines = g.nlines;
  a.ld2 = g.ld2;
  a.nbx = g.nbx;
  a.lmax_log = g.lmax_log;
  a.T = p.T;
  a.n_src = p.n_src;
  a.ft_mode = p.ft_mode;
  a.ftilde_given = p.ftilde;
  a.h = p.h;
  a.hbar = p.hbar;
  a.f = (const R *)f;
  a.src = src;
  a.src_s = nullptr;
  a.S = (R *)S;
  a.par = (Params *)(w + L.par);
  a.red = (double *)(w + L.red);
  a.mu = (double *)(w + L.mu);
  a.mu_red = (double *)(w + L.mu_red);
  a.expo = (int *)(w + L.expo);
  a.tw = (const cplx<R> *)(w + L.tw);
  a.s1 = (cplx<R> *)(w + L.spec);
  a.s2 = (cplx<R> *)(w + L.s2);
  a.s1o = a.s1;
  a.s1b = nullptr;
  a.gpart = nullptr;
  a.g = (R *)(w + L.g);
  a.terms = (R *)(w + L.terms);
  a.gam = (R *)(w + L.gam);
  a.info = info;
  a.dLdS = nullptr;
  a.dLdf = nullptr;
  a.lam = (R *)(w + L.lam);
  a.acc = (double *)(w + L.acc);
  char *c = (char *)ckpt;
  if (c) {  // the scalars, kernel spectrum and terms live in the checkpoint
    a.par = (Params *)(c + L.ck_par);
    a.g = (R *)(c + L.ck_g);
    a.terms = (R *)(c + L.ck_terms);
  }
  a.ck_expo = c ? (int *)(c + L.ck_expo) : nullptr;
  a.ck_phi = c ? (double *)(c + L.ck_phi) : nullptr;
  return a;
}

// One 3D solve: reduction of f, kernel spectrum (x, y, z passes), phi_0,
// then per term y forward, z convolution, y inverse and the x pass.
template <typename R>
sweik_status enqueue3d(const sweik_plan_s *pl, const void *f, const int32_t *src, void *S,
                       void *ws, hipStream_t st, sweik_info *info, KernelTimer *tm = nullptr,
                       const void *src_s = nullptr, void *ckpt = nullptr) {
  const Geo3 &g = pl->g3;
  Args3<R> a = make_args3<R>(pl, f, src, S, ws, info, ckpt);
  a.src_s = (const R *)src_s;
  const long long N = (long long)g.n0 * g.n1 * g.n2;
  hipError_t err = hipSuccess;
  auto launch = [&](int cls, auto &&fn) {
    if (err != hipSuccess) return;
    if (tm && tm->n < KernelTimer::kMax) {
      if (tm->n == 0) (void)hipEventRecord(tm->ev[0], st);
      err = fn();
      (void)hipEventRecord(tm->ev[tm->n + 1], st);
      tm->cls[tm->n++] = cls;
    } else {
      err = fn();
    }
  };
  const int ny = g.n0 * g.ncb1;  // y passes: planes i0
  const int T = pl->p.T;
  launch(SWEIK_KC_PREP, [&] { return launch_prep<R>((const R *)f, N, a.red, (cplx<R> *)a.tw, g.lmax, st); });
  launch(SWEIK_KC_GHAT_ROW, [&] { return launch_x3<R>(X_GHAT, g.H2, g.nbx, st, a, 0); });
  if (T > 0) {
    launch(SWEIK_KC_GHAT_COL, [&] { return launch_c3<R>(C3_GY, g.M1, ny, st, a, -1); });
    launch(SWEIK_KC_GHAT_Z, [&] { return launch_c3<R>(C3_GZ, g.M0, (g.H1 + 1) * g.ncb0, st, a, -1); });
  }
  if (pl->g2.phi0_fft) {
    // Table 1 steps 1-5: spectrum of exp(-beta |m|) into g0, transform of the
    // source grid (weights exp(-s_k/hbar), held in gamma), product, inverse
    // in the phi_0 pass
    Args3<R> a0 = a;
    a0.g = (R *)((char *)ws + pl->ws.g0);
    launch(SWEIK_KC_PHI0_FFT, [&] { return launch_x3<R>(X_ETAB, g.H2, g.nbx, st, a0, 0); });
    launch(SWEIK_KC_PHI0_FFT, [&] { return launch_c3<R>(C3_GY, g.M1, ny, st, a0, -1); });
    launch(SWEIK_KC_PHI0_FFT, [&] { return launch_c3<R>(C3_GZ, g.M0, (g.H1 + 1) * g.ncb0, st, a0, -1); });
    launch(SWEIK_KC_PHI0_FFT, [&] { return launch_fill<R>(a.gam, N, (R)0, st); });
    launch(SWEIK_KC_PHI0_FFT, [&] {
      return launch_seed_scatter<R>(a.gam, src, (const R *)src_s, pl->p.n_src, pl->p.hbar, g.n0,
                                    g.n1, g.n2, st);
    });
    launch(SWEIK_KC_PHI0_FFT, [&] { return launch_x3<R>(X_SEED, g.H2, g.nbx, st, a0, 0); });
    launch(SWEIK_KC_PHI0_FFT, [&] { return launch_c3<R>(C3_YF, g.M1, ny, st, a0, -1); });
    launch(SWEIK_KC_PHI0_FFT, [&] { return launch_c3<R>(C3_Z, g.M0, g.M1 * g.ncb0, st, a0, -1); });
    launch(SWEIK_KC_PHI0_FFT, [&] { return launch_c3<R>(C3_YI, g.M1, ny, st, a0, -1); });
    launch(SWEIK_KC_PHI0_ROW, [&] { return launch_x3<R>(X_PHI0F, g.H2, g.nbx, st, a, 0); });
  } else {
    launch(SWEIK_KC_PHI0_ROW, [&] { return launch_x3<R>(X_PHI0, g.H2, g.nbx, st, a, 0); });
  }
  for (int i = 1; i <= T; ++i) {
    launch(SWEIK_KC_Y_FWD, [&] { return launch_c3<R>(C3_YF, g.M1, ny, st, a, i - 1); });
    launch(SWEIK_KC_CONV_COL, [&] { return launch_c3<R>(C3_Z, g.M0, g.M1 * g.ncb0, st, a, -1); });
    launch(SWEIK_KC_Y_INV, [&] { return launch_c3<R>(C3_YI, g.M1, ny, st, a, -1); });
    launch(i == T ? SWEIK_KC_LAST_ROW : SWEIK_KC_TERM_ROW,
           [&] { return launch_x3<R>(i == T ? X_LAST : X_TERM, g.H2, g.nbx, st, a, i); });
  }
  return err == hipSuccess ? SWEIK_OK : SWEIK_EDEVICE;
}

// Adjoint of a 3D solve (f~ held fixed) from its checkpoint: lambda =
// -hbar dL/dS / phi, a_T = (-1)^T lambda; for i = T..1 b_i = kappa (*) a_i
// through the same y, z and y passes as the forward (kappa is even),
// dL/dgamma += phi_{i-1} b_i and a_{i-1} = (-1)^(i-1) lambda + gamma b_i in
// the x passes; dL/df = dL/dgamma 2 f / f~^2.
template <typename R>
sweik_status enqueue3d_adjoint(const sweik_plan_s *pl, const void *f, const int32_t *src,
                               const void *ckpt, const void *dLdS, void *dLdf, void *ws,
                               hipStream_t st) {
  const Geo3 &g = pl->g3;
  Args3<R> a = make_args3<R>(pl, f, src, nullptr, ws, nullptr, const_cast<void *>(ckpt));
  a.dLdS = (const R *)dLdS;
  a.dLdf = (R *)dLdf;
  const long long N = (long long)g.n0 * g.n1 * g.n2;
  const int T = pl->p.T;
  if (T == 0)  // f~ fixed: no term depends on f
    return launch_fill<R>((R *)dLdf, N, (R)0, st) == hipSuccess ? SWEIK_OK : SWEIK_EDEVICE;
  const int ny = g.n0 * g.ncb1;
  hipError_t err = launch_adj_prep<R>((const R *)dLdS, (const double *)a.ck_phi, N, pl->p.hbar,
                                      a.red, (cplx<R> *)a.tw, g.lmax, st);
  if (err == hipSuccess) err = launch_x3<R>(X_ADJ0, g.H2, g.nbx, st, a, T);
  for (int i = T; i >= 1 && err == hipSuccess; --i) {
    err = launch_c3<R>(C3_YF, g.M1, ny, st, a, -1);
    if (err == hipSuccess) err = launch_c3<R>(C3_Z, g.M0, g.M1 * g.ncb0, st, a, -1);
    if (err == hipSuccess) err = launch_c3<R>(C3_YI, g.M1, ny, st, a, -1);
    if (err == hipSuccess) err = launch_x3<R>(X_ADJ, g.H2, g.nbx, st, a, i);
  }
  return err == hipSuccess ? SWEIK_OK : SWEIK_EDEVICE;
}

// Full gradient (3D): the adjoint sweep of enqueue3d_adjoint with every
// convolution of a_i done twice, first with the kernel's beta-derivative
// (its y inverse pass writes the second spectrum s1b), then with the kernel;
// the x passes form the scalar partial sums; then the argmin / argmax of f
// and the scalar derivatives.
template <typename R>
sweik_status enqueue3d_adjoint_full(const sweik_plan_s *pl, const void *f, const int32_t *src,
                                    const void *src_s, const void *ckpt, const void *dLdS,
                                    void *dLdf, double *grads, void *ws, hipStream_t st) {
  const Geo3 &g = pl->g3;
  const Layout &L = pl->ws;
  char *w = (char *)ws;
  Args3<R> a = make_args3<R>(pl, f, src, nullptr, ws, nullptr, const_cast<void *>(ckpt));
  a.src_s = (const R *)src_s;
  a.dLdS = (const R *)dLdS;
  a.dLdf = (R *)dLdf;
  a.s1b = (cplx<R> *)(w + L.fg_spec2);
  a.gpart = (double *)(w + L.fg_part);
  // the same arguments with the beta-derivative's kernel spectrum and output
  Args3<R> ab = a;
  ab.g = (R *)(w + L.g0);
  ab.s1o = a.s1b;
  const long long N = (long long)g.n0 * g.n1 * g.n2;
  const int T = pl->p.T;
  const int ny = g.n0 * g.ncb1;
  hipError_t err = launch_adj_prep<R>((const R *)dLdS, (const double *)a.ck_phi, N, pl->p.hbar,
                                      a.red, (cplx<R> *)a.tw, g.lmax, st);
  if (T == 0) {
    if (err == hipSuccess) err = launch_fill<R>((R *)dLdf, N, (R)0, st);
    if (err == hipSuccess) err = launch_x3<R>(X_ADJ0_B, g.H2, g.nbx, st, a, 0);
  } else {
    // spectrum of dkappa/dbeta (x pass into s1, y and z passes into g0)
    if (err == hipSuccess) err = launch_x3<R>(X_DGHAT, g.H2, g.nbx, st, ab, 0);
    if (err == hipSuccess) err = launch_c3<R>(C3_GY, g.M1, ny, st, ab, -1);
    if (err == hipSuccess) err = launch_c3<R>(C3_GZ, g.M0, (g.H1 + 1) * g.ncb0, st, ab, -1);
    if (err == hipSuccess) err = launch_x3<R>(X_ADJ0_B, g.H2, g.nbx, st, a, T);
    for (int i = T; i >= 1 && err == hipSuccess; --i) {
      for (const Args3<R> *q : {&ab, &a}) {
        if (err == hipSuccess) err = launch_c3<R>(C3_YF, g.M1, ny, st, *q, -1);
        if (err == hipSuccess) err = launch_c3<R>(C3_Z, g.M0, g.M1 * g.ncb0, st, *q, -1);
        if (err == hipSuccess) err = launch_c3<R>(C3_YI, g.M1, ny, st, *q, -1);
      }
      if (err == hipSuccess) err = launch_x3<R>(X_ADJ_B, g.H2, g.nbx, st, a, i);
    }
  }
  if (err == hipSuccess)
    err = launch_adj_full_finish<R>((const R *)f, N, a.par, a.gpart, g.nbx,
                                    (long long *)(w + L.fg_ext), pl->p.ft_mode, pl->p.h,
                                    pl->p.hbar, (R *)dLdf, grads, st);
  return err == hipSuccess ? SWEIK_OK : SWEIK_EDEVICE;
}

// ---- uneven batches ---------------------------------------------------------
// Instances are grouped into size classes of equal (H1, M0): one launch per
// pass and class covers every instance of the class.  The per-instance
// arguments (BatchItem) live at the head of the workspace; they are written
// from a pinned host staging buffer by an asynchronous copy at the start of
// every solve.  Class chains run on forked streams joined back into the
// caller's stream.
struct BatchClass {
  int H1, M0, erow, ecol;
  std::vector<int> members;
  size_t row_items, col_items;  // workspace offsets of the two item lists
  int row_blocks, col_blocks;
  double work;
};

struct BatchKey {
  std::vector<const void *> ptrs;
  void *ws = nullptr;
  void *infos = nullptr;
  bool operator==(const BatchKey &o) const {
    return ptrs == o.ptrs && ws == o.ws && infos == o.infos;
  }
};

}  // namespace sweik

struct sweik_batch_s {
  int count = 0, prec = 0, T = 0;
  std::vector<sweik_plan_s> plans;
  std::vector<size_t> inst_off;
  std::vector<sweik::BatchClass> classes;
  size_t items_bytes = 0, total = 0;
  // created by sweik_batch_prepare (on its current device)
  bool rt = false;
  int device = -1;
  std::vector<hipStream_t> side;
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
  static constexpr int kRing = 4;
  void *stage[kRing] = {};
  hipEvent_t stage_ev[kRing] = {};
  bool stage_used[kRing] = {};
  int ring = 0;
  void *gstage = nullptr;
  hipStream_t cap = nullptr;
  hipGraphExec_t exec = nullptr;
  sweik::BatchKey key;

  ~sweik_batch_s() {
    if (exec) (void)hipGraphExecDestroy(exec);
    for (int i = 0; i < kRing; ++i) {
      if (stage_ev[i]) {
        (void)hipEventSynchronize(stage_ev[i]);
        (void)hipEventDestroy(stage_ev[i]);
      }
      if (stage[i]) (void)hipHostFree(stage[i]);
    }
    if (gstage) (void)hipHostFree(gstage);
    for (hipStream_t s : side) (void)hipStreamDestroy(s);
    if (cap) (void)hipStreamDestroy(cap);
    if (fork) (void)hipEventDestroy(fork);
    for (hipEvent_t e : join) (void)hipEventDestroy(e);
  }
};

namespace sweik {

size_t batch_item_bytes(int prec) {
  return prec == SWEIK_F64 ? sizeof(BatchItem<double>) : sizeof(BatchItem<float>);
}

// Streams, events and pinned staging of a batch, on the current device
// (sweik_batch_prepare): solves only use them.
sweik_status batch_runtime(sweik_batch_s *b) {
  if (b->rt) return SWEIK_OK;
  const int nside = (int)b->classes.size() - 1;
  for (int c = 0; c < nside; ++c) {
    hipStream_t s;
    if (counted(hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess)
      return SWEIK_EDEVICE;
    b->side.push_back(s);
    hipEvent_t e;
    if (counted(hipEventCreateWithFlags(&e, hipEventDisableTiming)) != hipSuccess)
      return SWEIK_EDEVICE;
    b->join.push_back(e);
  }
  if (counted(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming)) != hipSuccess)
    return SWEIK_EDEVICE;
  if (counted(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking)) != hipSuccess)
    return SWEIK_EDEVICE;
  for (int i = 0; i < sweik_batch_s::kRing; ++i) {
    if (counted(hipHostMalloc(&b->stage[i], b->items_bytes, hipHostMallocDefault)) != hipSuccess)
      return SWEIK_EDEVICE;
    if (counted(hipEventCreateWithFlags(&b->stage_ev[i], hipEventDisableTiming)) != hipSuccess)
      return SWEIK_EDEVICE;
  }
  if (counted(hipHostMalloc(&b->gstage, b->items_bytes, hipHostMallocDefault)) != hipSuccess)
    return SWEIK_EDEVICE;
  if (hipGetDevice(&b->device) != hipSuccess) return SWEIK_EDEVICE;
  b->rt = true;
  return SWEIK_OK;
}

template <typename R>
void batch_fill_items(const sweik_batch_s *b, const void *const *f, const int32_t *const *src,
                      void *const *S, void *ws, sweik_info *infos, void *host) {
  char *h = (char *)host;
  char *w = (char *)ws;
  for (const BatchClass &c : b->classes) {
    BatchItem<R> *ri = (BatchItem<R> *)(h + c.row_items);
    BatchItem<R> *ci = (BatchItem<R> *)(h + c.col_items);
    int rbeg = 0, cbeg = 0;
    for (size_t j = 0; j < c.members.size(); ++j) {
      const int i = c.members[j];
      const sweik_plan_s &pl = b->plans[i];
      Args2<R> a = make_args2<R>(&pl, f[i], src[i], S[i], w + b->inst_off[i], nullptr,
                                 infos ? infos + i : nullptr);
      ri[j].a = a;
      ri[j].begin = rbeg;
      ri[j].pad_ = 0;
      ci[j].a = a;
      ci[j].begin = cbeg;
      ci[j].pad_ = 0;
      rbeg += pl.g2.nbr;
      cbeg += pl.g2.ncw;
    }
  }
}

template <typename R>
hipError_t batch_class_chain(const sweik_batch_s *b, const BatchClass &c, char *ws,
                             hipStream_t st) {
  const BatchItem<R> *ri = (const BatchItem<R> *)(ws + c.row_items);
  const BatchItem<R> *ci = (const BatchItem<R> *)(ws + c.col_items);
  const int n = (int)c.members.size();
  hipError_t err = launch_prep_batch<R>(n, st, ri);
  if (err == hipSuccess) err = launch_row2_batch<R>(ROW_GHAT, c.H1, c.erow, c.row_blocks, st, ri, n, 0);
  if (err == hipSuccess) err = launch_col2_batch<R>(COL_GHAT, c.M0, c.ecol, c.col_blocks, st, ci, n);
  if (err == hipSuccess) err = launch_row2_batch<R>(ROW_PHI0, c.H1, c.erow, c.row_blocks, st, ri, n, 0);
  for (int i = 1; i <= b->T && err == hipSuccess; ++i) {
    err = launch_col2_batch<R>(COL_CONV, c.M0, c.ecol, c.col_blocks, st, ci, n);
    if (err == hipSuccess)
      err = launch_row2_batch<R>(i == b->T ? ROW_LAST : ROW_TERM, c.H1, c.erow, c.row_blocks, st,
                                 ri, n, i);
  }
  return err;
}

// Upload the item lists from `host` and enqueue every class chain, forked
// from and joined back into `st`.
template <typename R>
sweik_status batch_enqueue(sweik_batch_s *b, void *host, char *ws, hipStream_t st,
                           hipEvent_t upload_done) {
  if (hipMemcpyAsync(ws, host, b->items_bytes, hipMemcpyHostToDevice, st) != hipSuccess)
    return SWEIK_EDEVICE;
  if (upload_done && hipEventRecord(upload_done, st) != hipSuccess) return SWEIK_EDEVICE;
  const int nc = (int)b->classes.size();
  if (nc > 1 && hipEventRecord(b->fork, st) != hipSuccess) return SWEIK_EDEVICE;
  for (int c = 1; c < nc; ++c)
    if (hipStreamWaitEvent(b->side[c - 1], b->fork, 0) != hipSuccess) return SWEIK_EDEVICE;
  for (int c = 0; c < nc; ++c) {
    hipStream_t s = c == 0 ? st : b->side[c - 1];
    if (batch_class_chain<R>(b, b->classes[c], ws, s) != hipSuccess) return SWEIK_EDEVICE;
  }
  for (int c = 1; c < nc; ++c) {
    if (hipEventRecord(b->join[c - 1], b->side[c - 1]) != hipSuccess) return SWEIK_EDEVICE;
    if (hipStreamWaitEvent(st, b->join[c - 1], 0) != hipSuccess) return SWEIK_EDEVICE;
  }
  return SWEIK_OK;
}

sweik_status batch_args_ok(const sweik_batch_s *b, const void *const *f,
                           const int32_t *const *src, void *const *S, void *ws,
                           size_t ws_bytes) {
  if (!b || !f || !src || !S || !ws || !b->rt) return SWEIK_EINVAL;
  if (ws_bytes < b->total) return SWEIK_EWORKSPACE;
  for (int i = 0; i < b->count; ++i)
    if (!f[i] || !src[i] || !S[i]) return SWEIK_EINVAL;
  return SWEIK_OK;
}

}  // namespace sweik

namespace {

// Average milliseconds of `reps` launches of fn on st (events around all).
template <typename F> float time_launches(hipStream_t st, int reps, F &&fn, bool *ok) {
  hipEvent_t e0, e1;
  if (counted(hipEventCreate(&e0)) != hipSuccess) return *ok = false, 0.0f;
  if (counted(hipEventCreate(&e1)) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return *ok = false, 0.0f;
  }
  bool good = fn() == hipSuccess;  // warm-up (also sets the LDS attribute)
  good = good && hipEventRecord(e0, st) == hipSuccess;
  for (int r = 0; r < reps && good; ++r) good = fn() == hipSuccess;
  good = good && hipEventRecord(e1, st) == hipSuccess;
  good = good && hipEventSynchronize(e1) == hipSuccess;
  float ms = 0.0f;
  good = good && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (!good) *ok = false;
  return ms / reps;
}

template <typename R> int32_t autotune2d(sweik_plan_s *pl, void *ws, hipStream_t st) {
  Geo2 &g = pl->g2;
  Args2<R> a = make_args2<R>(pl, nullptr, nullptr, nullptr, ws, nullptr, nullptr);
  const dim3 grow(g.nbr), gcol(g.ncw);
  // a term is a column convolution followed by a row pass; time the pair as
  // it runs in a solve (row pass of term 1, which is not the last term and so
  // writes no output; without two terms only the column pass is timed)
  const bool rows = pl->p.T >= 2;
  const int cand[3] = {16, 8, 4};
  const int ncand = pl->p.prec == SWEIK_F64 ? 2 : 3;  // radix 4: float32 only
  int pc[9], pr[9], npair = 0;
  for (int ic = 0; ic < ncand; ++ic)
    for (int ir = 0; ir < ncand; ++ir) {
      if (!col_ok<R>(g.M0, cand[ic])) continue;
      if (!rows && ir != 0) continue;
      if (rows && !row_ok<R>(g.H1, cand[ir], ROW_TERM)) continue;
      pc[npair] = cand[ic];
      pr[npair] = cand[ir];
      ++npair;
    }
  // the pairs take turns within every repetition, so that a drift of the
  // clocks during tuning does not favour the pairs timed first; the median
  // of the repetitions decides
  constexpr int kReps = 5;
  float t[9][kReps];
  for (int rep = 0; rep < kReps; ++rep)
    for (int k = 0; k < npair; ++k) {
      bool ok = true;
      t[k][rep] = time_launches(st, 4, [&] {
        hipError_t e = launch_col2<R>(COL_CONV, g.M0, pc[k], gcol, st, a);
        if (e == hipSuccess && rows) e = launch_row2<R>(ROW_TERM, g.H1, pr[k], grow, st, a, 1);
        return e;
      }, &ok);
      if (!ok) return -1;
    }
  int timed = 0, bc = g.ecol, br = g.erow;
  float best = 0.0f;
  for (int k = 0; k < npair; ++k) {
    std::sort(t[k], t[k] + kReps);
    const float med = t[k][kReps / 2];
    if (timed == 0 || med < best) {
      best = med;
      bc = pc[k];
      br = rows ? pr[k] : g.erow;
    }
    ++timed;
  }
  g.ecol = bc;
  sched_store(SCHED_COL2, g.M0, pl->p.prec, bc);
  if (rows) {
    g.erow = br;
    sched_store(SCHED_ROW2, g.H1, pl->p.prec, br);
  }
  return timed;
}

}  // namespace

// Workspace of sweik_solve_noalloc: a static device array, one copy per GPU
// the library runs on (held until the process ends).  Its host-side name
// only stands for the symbol; the device address comes from
// hipGetSymbolAddress, once per device with that device current, and only
// that address is ever passed to kernels.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kScratchDevices] = {};

sweik_status scratch_address(void **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return SWEIK_EDEVICE;
  if (dev < 0 || dev >= kScratchDevices) return SWEIK_EUNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
      return SWEIK_EDEVICE;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return SWEIK_OK;
}
}  // namespace

extern "C" {

sweik_status sweik_plan_create(const sweik_problem *problem, sweik_plan *out) {
  if (!out) return SWEIK_EINVAL;
  *out = nullptr;
  sweik_status st = validate_problem(problem);
  if (st != SWEIK_OK) return st;
  sweik_plan_s *pl = new (std::nothrow) sweik_plan_s();
  if (!pl) return SWEIK_ENOMEM;
  pl->p = *problem;
  pl->lds_max = kLdsDevice;
  st = problem->ndim == 2 ? plan2d(pl) : plan3d(pl);
  if (st != SWEIK_OK) {
    delete pl;
    return st;
  }
  *out = pl;
  return SWEIK_OK;
}

void sweik_plan_destroy(sweik_plan plan) { delete plan; }

size_t sweik_workspace_bytes(sweik_plan plan) { return plan ? plan->ws.total : 0; }
size_t sweik_checkpoint_bytes(sweik_plan plan) { return plan ? plan->ws.ck_total : 0; }

int32_t sweik_plan_padded_dims(sweik_plan plan, int64_t *out) {
  if (!plan) return 0;
  if (out)
    for (int d = 0; d < 3; ++d) out[d] = plan->padded[d];
  return plan->p.ndim;
}

sweik_status sweik_check_sources(sweik_plan plan, const int32_t *src) {
  if (!plan || !src) return SWEIK_EINVAL;
  const sweik_problem &p = plan->p;
  std::set<std::tuple<int, int, int>> seen;
  for (int k = 0; k < p.n_src; ++k) {
    int c[3] = {0, 0, 0};
    for (int d = 0; d < p.ndim; ++d) {
      c[d] = src[k * p.ndim + d];
      if (c[d] < 0 || c[d] >= p.dims[d]) return SWEIK_EINVAL;
    }
    if (!seen.insert(std::make_tuple(c[0], c[1], c[2])).second) return SWEIK_EINVAL;
  }
  return SWEIK_OK;
}

sweik_status sweik_solve_seeded(sweik_plan plan, const void *f, const int32_t *src,
                                const void *src_s, void *S, void *ws, size_t ws_bytes,
                                void *ckpt, void *stream, sweik_info *info) {
  if (!plan || !f || !src || !S || !ws) return SWEIK_EINVAL;
  if (ws_bytes < plan->ws.total) return SWEIK_EWORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  const bool f64 = plan->p.prec == SWEIK_F64;
  if (plan->p.ndim == 2) {
    return f64 ? enqueue2d<double>(plan, f, src, S, ws, ckpt, st, info, nullptr, src_s)
               : enqueue2d<float>(plan, f, src, S, ws, ckpt, st, info, nullptr, src_s);
  }
  return f64 ? enqueue3d<double>(plan, f, src, S, ws, st, info, nullptr, src_s, ckpt)
             : enqueue3d<float>(plan, f, src, S, ws, st, info, nullptr, src_s, ckpt);
}

sweik_status sweik_solve(sweik_plan plan, const void *f, const int32_t *src, void *S, void *ws,
                         size_t ws_bytes, void *ckpt, void *stream, sweik_info *info) {
  return sweik_solve_seeded(plan, f, src, nullptr, S, ws, ws_bytes, ckpt, stream, info);
}

size_t sweik_tilted_workspace_bytes(sweik_plan plan, int32_t n_tilt) {
  if (!plan || plan->p.ndim != 2 || n_tilt < 1 || n_tilt > SWEIK_MAX_TILTS) return 0;
  return tilt_ws(plan, n_tilt).total;
}

sweik_status sweik_solve_tilted(sweik_plan plan, const void *f, const int32_t *src,
                                const void *src_s, void *S, const double *tilts, int32_t n_tilt,
                                int32_t per_source, void *ws, size_t ws_bytes, void *stream,
                                sweik_info *info) {
  if (!plan || !f || !src || !S || !ws || !tilts) return SWEIK_EINVAL;
  if (plan->p.ndim != 2) return SWEIK_EUNSUPPORTED;
  if (n_tilt < 1 || n_tilt > SWEIK_MAX_TILTS) return SWEIK_EINVAL;
  for (int d = 0; d < n_tilt; ++d) {
    const double t0 = tilts[2 * d], t1 = tilts[2 * d + 1];
    if (!std::isfinite(t0) || !std::isfinite(t1) || !(t0 * t0 + t1 * t1 < 1.0)) return SWEIK_EINVAL;
  }
  if (ws_bytes < tilt_ws(plan, n_tilt).total) return SWEIK_EWORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  const bool f64 = plan->p.prec == SWEIK_F64;
  if (plan->p.T == 0)  // phi = phi_0 in closed form: nothing for a tilt to stabilise
    return f64 ? enqueue2d<double>(plan, f, src, S, ws, nullptr, st, info, nullptr, src_s)
               : enqueue2d<float>(plan, f, src, S, ws, nullptr, st, info, nullptr, src_s);
  return f64 ? enqueue2d_tilted<double>(plan, f, src, src_s, S, tilts, n_tilt, per_source != 0, ws,
                                        st, info)
             : enqueue2d_tilted<float>(plan, f, src, src_s, S, tilts, n_tilt, per_source != 0, ws,
                                       st, info);
}

size_t sweik_noalloc_scratch_bytes(void) { return kScratchBytes; }

sweik_status sweik_solve_noalloc(sweik_plan plan, const void *f, const int32_t *src, void *S,
                                 void *stream, sweik_info *info) {
  if (!plan || !f || !src || !S) return SWEIK_EINVAL;
  if (plan->ws.total > kScratchBytes) return SWEIK_EWORKSPACE;
  void *ws = nullptr;
  const sweik_status rc = scratch_address(&ws);
  if (rc != SWEIK_OK) return rc;
  // every workspace buffer of a solve is written before it is read, so the
  // previous call's contents need no clearing
  return sweik_solve_seeded(plan, f, src, nullptr, S, ws, kScratchBytes, nullptr, stream, info);
}

sweik_status sweik_solve_timed(sweik_plan plan, const void *f, const int32_t *src, void *S,
                               void *ws, size_t ws_bytes, void *stream, float *ms,
                               int32_t *count) {
  if (!plan || !f || !src || !S || !ws || !ms || !count) return SWEIK_EINVAL;
  if (ws_bytes < plan->ws.total) return SWEIK_EWORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  KernelTimer tm;
  if (!tm.ok) return SWEIK_EDEVICE;
  const bool f64 = plan->p.prec == SWEIK_F64;
  sweik_status rc =
      plan->p.ndim == 2
          ? (f64 ? enqueue2d<double>(plan, f, src, S, ws, nullptr, st, nullptr, &tm)
                 : enqueue2d<float>(plan, f, src, S, ws, nullptr, st, nullptr, &tm))
          : (f64 ? enqueue3d<double>(plan, f, src, S, ws, st, nullptr, &tm)
                 : enqueue3d<float>(plan, f, src, S, ws, st, nullptr, &tm));
  if (rc != SWEIK_OK) return rc;
  if (hipStreamSynchronize(st) != hipSuccess) return SWEIK_EDEVICE;
  for (int c = 0; c < SWEIK_KC_COUNT; ++c) {
    ms[c] = 0.0f;
    count[c] = 0;
  }
  for (int i = 0; i < tm.n; ++i) {
    float t = 0.0f;
    if (hipEventElapsedTime(&t, tm.ev[i], tm.ev[i + 1]) != hipSuccess)
      return SWEIK_EDEVICE;
    ms[tm.cls[i]] += t;
    count[tm.cls[i]] += 1;
  }
  return SWEIK_OK;
}

sweik_status sweik_solve_adjoint(sweik_plan plan, const void *f, const int32_t *src,
                                 const void *ckpt, const void *dLdS, void *dLdf, void *ws,
                                 size_t ws_bytes, void *stream) {
  if (!plan || !f || !src || !ckpt || !dLdS || !dLdf || !ws) return SWEIK_EINVAL;
  if (ws_bytes < plan->ws.total) return SWEIK_EWORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  if (plan->p.ndim == 2) {
    return plan->p.prec == SWEIK_F64
               ? enqueue2d_adjoint<double>(plan, f, src, ckpt, dLdS, dLdf, ws, st)
               : enqueue2d_adjoint<float>(plan, f, src, ckpt, dLdS, dLdf, ws, st);
  }
  return plan->p.prec == SWEIK_F64
             ? enqueue3d_adjoint<double>(plan, f, src, ckpt, dLdS, dLdf, ws, st)
             : enqueue3d_adjoint<float>(plan, f, src, ckpt, dLdS, dLdf, ws, st);
}

size_t sweik_adjoint_full_workspace_bytes(sweik_plan plan) {
  if (!plan) return 0;
  return plan->ws.fg_total;
}

sweik_status sweik_solve_adjoint_full(sweik_plan plan, const void *f, const int32_t *src,
                                      const void *src_s, const void *ckpt, const void *dLdS,
                                      void *dLdf, double *grads, void *ws, size_t ws_bytes,
                                      void *stream) {
  if (!plan || !f || !src || !ckpt || !dLdS || !dLdf || !ws) return SWEIK_EINVAL;
  if (ws_bytes < plan->ws.fg_total) return SWEIK_EWORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  if (plan->p.ndim == 3)
    return plan->p.prec == SWEIK_F64
               ? enqueue3d_adjoint_full<double>(plan, f, src, src_s, ckpt, dLdS, dLdf, grads, ws, st)
               : enqueue3d_adjoint_full<float>(plan, f, src, src_s, ckpt, dLdS, dLdf, grads, ws, st);
  return plan->p.prec == SWEIK_F64
             ? enqueue2d_adjoint_full<double>(plan, f, src, src_s, ckpt, dLdS, dLdf, grads, ws, st)
             : enqueue2d_adjoint_full<float>(plan, f, src, src_s, ckpt, dLdS, dLdf, grads, ws, st);
}

sweik_status sweik_batch_create(const sweik_problem *problems, int32_t count, sweik_batch *out) {
  if (!out) return SWEIK_EINVAL;
  *out = nullptr;
  if (!problems || count < 1) return SWEIK_EINVAL;
  for (int i = 0; i < count; ++i) {
    sweik_status st = validate_problem(&problems[i]);
    if (st != SWEIK_OK) return st;
    if (problems[i].ndim != 2) return SWEIK_EUNSUPPORTED;
    if (problems[i].prec != problems[0].prec || problems[i].T != problems[0].T)
      return SWEIK_EINVAL;
  }
  sweik_batch_s *b = new (std::nothrow) sweik_batch_s();
  if (!b) return SWEIK_ENOMEM;
  b->count = count;
  b->prec = problems[0].prec;
  b->T = problems[0].T;
  b->plans.resize(count);
  for (int i = 0; i < count; ++i) {
    sweik_plan_s &pl = b->plans[i];
    pl.p = problems[i];
    pl.lds_max = kLdsDevice;
    sweik_status st = plan2d(&pl);
    if (st != SWEIK_OK) {
      delete b;
      return st;
    }
    pl.g2.phi0_fft = 0;  // batched phi_0 passes sum over the sources directly
  }
  // size classes, largest total work first (it runs on the caller's stream)
  for (int i = 0; i < count; ++i) {
    const Geo2 &g = b->plans[i].g2;
    auto it = std::find_if(b->classes.begin(), b->classes.end(), [&](const BatchClass &c) {
      return c.H1 == g.H1 && c.M0 == g.M0 && c.erow == g.erow && c.ecol == g.ecol;
    });
    if (it == b->classes.end()) {
      b->classes.push_back(BatchClass{g.H1, g.M0, g.erow, g.ecol, {}, 0, 0, 0, 0, 0.0});
      it = b->classes.end() - 1;
    }
    it->members.push_back(i);
    it->row_blocks += g.nbr;
    it->col_blocks += g.ncw;
    it->work += (double)g.M0 * g.H1;
  }
  std::stable_sort(b->classes.begin(), b->classes.end(),
                   [](const BatchClass &x, const BatchClass &y) { return x.work > y.work; });
  const size_t isz = batch_item_bytes(b->prec);
  size_t off = 0;
  for (BatchClass &c : b->classes) {
    c.row_items = off;
    off = align256(off + isz * c.members.size());
    c.col_items = off;
    off = align256(off + isz * c.members.size());
  }
  b->items_bytes = off;
  b->inst_off.resize(count);
  for (int i = 0; i < count; ++i) {
    b->inst_off[i] = off;
    off = align256(off + b->plans[i].ws.total);
  }
  b->total = off;
  *out = b;
  return SWEIK_OK;
}

sweik_status sweik_batch_prepare(sweik_batch b) {
  if (!b) return SWEIK_EINVAL;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return SWEIK_EDEVICE;
  if (b->rt) return dev == b->device ? SWEIK_OK : SWEIK_EINVAL;
  return batch_runtime(b);
}

int64_t sweik_resource_count(void) { return g_resources.load(std::memory_order_relaxed); }

void sweik_batch_destroy(sweik_batch batch) { delete batch; }

size_t sweik_batch_workspace_bytes(sweik_batch batch) { return batch ? batch->total : 0; }

sweik_status sweik_batch_solve(sweik_batch b, const void *const *f, const int32_t *const *src,
                               void *const *S, void *ws, size_t ws_bytes, void *stream,
                               sweik_info *infos) {
  sweik_status rc = batch_args_ok(b, f, src, S, ws, ws_bytes);
  if (rc != SWEIK_OK) return rc;
  // staging slot: wait (host side) only for the copy issued kRing calls ago
  const int slot = b->ring;
  b->ring = (b->ring + 1) % sweik_batch_s::kRing;
  if (b->stage_used[slot] && hipEventSynchronize(b->stage_ev[slot]) != hipSuccess)
    return SWEIK_EDEVICE;
  b->stage_used[slot] = true;
  void *host = b->stage[slot];
  hipStream_t st = (hipStream_t)stream;
  if (b->prec == SWEIK_F64) {
    batch_fill_items<double>(b, f, src, S, ws, infos, host);
    return batch_enqueue<double>(b, host, (char *)ws, st, b->stage_ev[slot]);
  }
  batch_fill_items<float>(b, f, src, S, ws, infos, host);
  return batch_enqueue<float>(b, host, (char *)ws, st, b->stage_ev[slot]);
}

sweik_status sweik_batch_solve_graph(sweik_batch b, const void *const *f,
                                     const int32_t *const *src, void *const *S, void *ws,
                                     size_t ws_bytes, void *stream, sweik_info *infos) {
  sweik_status rc = batch_args_ok(b, f, src, S, ws, ws_bytes);
  if (rc != SWEIK_OK) return rc;
  BatchKey key;
  for (int i = 0; i < b->count; ++i) {
    key.ptrs.push_back(f[i]);
    key.ptrs.push_back(src[i]);
    key.ptrs.push_back(S[i]);
  }
  key.ws = ws;
  key.infos = infos;
  if (!b->exec || !(key == b->key)) {
    if (b->exec) {
      // the staging buffer is read by earlier replays: let them finish
      if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return SWEIK_EDEVICE;
      (void)hipGraphExecDestroy(b->exec);
      b->exec = nullptr;
    }
    if (b->prec == SWEIK_F64)
      batch_fill_items<double>(b, f, src, S, ws, infos, b->gstage);
    else
      batch_fill_items<float>(b, f, src, S, ws, infos, b->gstage);
    if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return SWEIK_EDEVICE;
    rc = b->prec == SWEIK_F64 ? batch_enqueue<double>(b, b->gstage, (char *)ws, b->cap, nullptr)
                              : batch_enqueue<float>(b, b->gstage, (char *)ws, b->cap, nullptr);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(b->cap, &graph);
    if (rc != SWEIK_OK || ec != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return SWEIK_EDEVICE;
    }
    const hipError_t ei = counted(hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0));
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) {
      b->exec = nullptr;
      return SWEIK_EDEVICE;
    }
    b->key = key;
  }
  return hipGraphLaunch(b->exec, (hipStream_t)stream) == hipSuccess ? SWEIK_OK : SWEIK_EDEVICE;
}

sweik_status sweik_plan_get_schedule(sweik_plan plan, sweik_schedule *out) {
  if (!plan || !out) return SWEIK_EINVAL;
  std::memset(out, 0, sizeof(*out));
  out->row_e = plan->g2.erow;
  out->col_e = plan->g2.ecol;
  out->phi0_fft = plan->g2.phi0_fft;
  return SWEIK_OK;
}

sweik_status sweik_plan_set_schedule(sweik_plan plan, const sweik_schedule *sc) {
  if (!plan || !sc) return SWEIK_EINVAL;
  auto ok = [](int e) { return e == 16 || e == 8 || e == 4; };
  if (!ok(sc->row_e) || !ok(sc->col_e)) return SWEIK_EINVAL;
  if (plan->p.prec == SWEIK_F64 && (sc->row_e == 4 || sc->col_e == 4)) return SWEIK_EUNSUPPORTED;
  if (sc->phi0_fft != 0 && sc->phi0_fft != 1) return SWEIK_EINVAL;
  if (plan->p.ndim == 3 && (sc->row_e != 16 || sc->col_e != 16)) return SWEIK_EUNSUPPORTED;
  if (plan->p.ndim == 2) {
    const int H = plan->g2.H1;
    if (H < sc->row_e || (H > 4096 && sc->row_e != 16)) return SWEIK_EUNSUPPORTED;
    const int M0 = plan->g2.M0;
    if (!(plan->p.prec == SWEIK_F64 ? col_ok<double>(M0, sc->col_e) : col_ok<float>(M0, sc->col_e)))
      return SWEIK_EUNSUPPORTED;
  }
  plan->g2.erow = sc->row_e;
  plan->g2.ecol = sc->col_e;
  plan->g2.phi0_fft = sc->phi0_fft;
  return SWEIK_OK;
}

int32_t sweik_autotune(sweik_plan plan, void *ws, size_t ws_bytes, void *stream) {
  if (!plan || !ws || ws_bytes < plan->ws.total) return -1;
  if (plan->p.ndim != 2) return 0;
  hipStream_t st = (hipStream_t)stream;
  return plan->p.prec == SWEIK_F64 ? autotune2d<double>(plan, ws, st)
                                   : autotune2d<float>(plan, ws, st);
}

const char *sweik_status_string(sweik_status s) {
  switch (s) {
    case SWEIK_OK: return "ok";
    case SWEIK_EINVAL: return "invalid argument";
    case SWEIK_EUNSUPPORTED: return "unsupported problem";
    case SWEIK_EWORKSPACE: return "workspace too small";
    case SWEIK_EDEVICE: return "HIP error";
    case SWEIK_ENOMEM: return "out of host memory";
  }
  return "unknown status";
}

int32_t sweik_abi_version(void) { return SWEIK_ABI_VERSION; }

const char *sweik_last_error(void) { return g_last_error; }

}  // extern "C"
