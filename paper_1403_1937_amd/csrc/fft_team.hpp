// fft_team.hpp -- register/LDS Stockham FFT for gfx950 (wave64).
//
// A "team" of P = L/E threads transforms one complex line of length L
// (compile-time power of two, E <= L <= 8192; E = 16 or 8 elements per
// thread).  Thread t of the team always holds the E elements with indices
// t + P*j, j < E, in registers: on entry the input samples, on exit the
// transform values at the same indices.  Stages are Stockham autosort steps
// of radix E with spans p = 1, E, E^2, ... (the last one of radix L/p); data
// moves through LDS only between stages, so a line costs ceil(log_E L) - 1
// LDS round trips.  E = 8 uses twice the threads per line (more waves per
// SIMD to hide latency) for one more LDS round trip.  Because the first stage
// reads and the last stage writes the same index pattern, a forward
// transform, a pointwise spectral product and an inverse transform chain
// without any extra exchange.
//
// Twiddles come from per-stage tables in LDS (see stage_tw_len), which the
// kernel copies once from the solve's global table.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sweik {

template <typename R> struct cplx_t;
template <> struct cplx_t<float> { using type = float2; };
// float64 complex values are a native two-lane vector: register arrays of
// them stay in registers, where arrays of HIP's double2 (or of a plain
// struct of two doubles) were placed in scratch memory by the compiler
typedef double double2v __attribute__((ext_vector_type(2)));
template <> struct cplx_t<double> { using type = double2v; };
template <typename R> using cplx = typename cplx_t<R>::type;
template <typename C> struct real_of;
template <> struct real_of<float2> { using type = float; };
template <> struct real_of<double2v> { using type = double; };
template <typename C> using real_t = typename real_of<C>::type;

template <typename C> __device__ __forceinline__ C cmake(real_t<C> a, real_t<C> b) {
  C c;
  c.x = a;
  c.y = b;
  return c;
}
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return cmake<C>(a.x + b.x, a.y + b.y); }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return cmake<C>(a.x - b.x, a.y - b.y); }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  return cmake<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename C> __device__ __forceinline__ C cmulc(C a, C b) {
  return cmake<C>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename C> __device__ __forceinline__ C cconj(C a) { return cmake<C>(a.x, -a.y); }
template <typename C> __device__ __forceinline__ C cscale(C a, real_t<C> s) { return cmake<C>(a.x * s, a.y * s); }
// multiply by -i (forward) or +i (inverse)
template <bool INV, typename C> __device__ __forceinline__ C cmul_mi(C a) {
  return INV ? cmake<C>(-a.y, a.x) : cmake<C>(a.y, -a.x);
}

// cos and sin of 2 pi m / 16, m = 0..15
__device__ constexpr double kCos16[16] = {
    1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
    0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
    -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173,
    0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613};
__device__ constexpr double kSin16[16] = {
    0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613,
    1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
    0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
    -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173};

// v *= exp(-+ 2 pi i m / R) with compile-time R, m  (sign: - forward, + inverse)
template <int R, int M, bool INV, typename C> __device__ __forceinline__ C twc(C v) {
  using T = real_t<C>;
  constexpr int m16 = (M * (16 / R)) & 15;
  if constexpr (m16 == 0) {
    return v;
  } else if constexpr (m16 == 4) {
    return cmul_mi<INV>(v);
  } else if constexpr (m16 == 8) {
    return cmake<C>(-v.x, -v.y);
  } else if constexpr (m16 == 12) {
    return cmul_mi<!INV>(v);
  } else {
    const T c = (T)kCos16[m16];
    const T s = INV ? (T)kSin16[m16] : -(T)kSin16[m16];
    return cmake<C>(v.x * c - v.y * s, v.x * s + v.y * c);
  }
}

// In-register DFT of length R in natural order: u[q] <- sum_r u[r] w^{rq}.
template <int R, bool INV, typename C> struct Dft;

template <bool INV, typename C> struct Dft<1, INV, C> {
  __device__ __forceinline__ static void run(C *) {}
};
template <bool INV, typename C> struct Dft<2, INV, C> {
  __device__ __forceinline__ static void run(C *u) {
    C a = u[0], b = u[1];
    u[0] = cadd(a, b);
    u[1] = csub(a, b);
  }
};
template <bool INV, typename C> struct Dft<4, INV, C> {
  __device__ __forceinline__ static void run(C *u) {
    C s02 = cadd(u[0], u[2]), d02 = csub(u[0], u[2]);
    C s13 = cadd(u[1], u[3]), d13 = cmul_mi<INV>(csub(u[1], u[3]));
    u[0] = cadd(s02, s13);
    u[2] = csub(s02, s13);
    u[1] = cadd(d02, d13);
    u[3] = csub(d02, d13);
  }
};

// R = 4 B: index n = B n1 + n2, frequency k = k1 + 4 k2.
template <int R, bool INV, typename C> struct Dft {
  static constexpr int B = R / 4;
  template <int N2, int K1> __device__ __forceinline__ static void tw(C (&y)[R]) {
    y[N2 * 4 + K1] = twc<R, N2 * K1, INV>(y[N2 * 4 + K1]);
    if constexpr (K1 + 1 < 4) tw<N2, K1 + 1>(y);
    else if constexpr (N2 + 1 < B) tw<N2 + 1, 0>(y);
  }
  __device__ __forceinline__ static void run(C *u) {
    C y[R];
#pragma unroll
    for (int n2 = 0; n2 < B; ++n2) {
      C t[4] = {u[n2], u[B + n2], u[2 * B + n2], u[3 * B + n2]};
      Dft<4, INV, C>::run(t);
#pragma unroll
      for (int k1 = 0; k1 < 4; ++k1) y[n2 * 4 + k1] = t[k1];
    }
    tw<0, 0>(y);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      C s[B];
#pragma unroll
      for (int n2 = 0; n2 < B; ++n2) s[n2] = y[n2 * 4 + k1];
      Dft<B, INV, C>::run(s);
#pragma unroll
      for (int k2 = 0; k2 < B; ++k2) u[k1 + 4 * k2] = s[k2];
    }
  }
};

__host__ __device__ constexpr int ilog2c(int x) { return x <= 1 ? 0 : 1 + ilog2c(x >> 1); }

// LDS layouts of a line.
//   padded   one pad slot every 16 elements (breaks the stride-16 pattern of
//            the first Stockham stage); lpad, lds_line_len
//   packed   float2 lines only: unpadded, the exchanges inside the FFT
//            XOR-swizzled per stage (stage_slot); lslot.  The LDS serves a
//            wave's 8-byte accesses 32 lanes at a time over 64 four-byte
//            banks, so 32 consecutive float2 elements fill the banks exactly
//            once, and a pad slot inside such a run costs a second cycle.
//            Used by the 2D row passes (one team per wave at the benchmark
//            sizes).  The column passes (the 2048-point ones interleave two
//            teams in a wave) and the 3D passes measured slower with it and
//            keep the padded layout, as does every double2 line.
__host__ __device__ constexpr int lpad(int i) { return i + (i >> 4); }
__host__ __device__ constexpr int lds_line_len(int L) { return L + (L >> 4) + 1; }
template <typename C> __host__ __device__ constexpr int lslot(int i) {
  return sizeof(C) == 8 ? i : lpad(i);
}
// Padded line length of a pass whose 32-lane groups hold G lines (teams):
// the shortest length that holds lpad(L - 1) and starts the lines 32/G
// float2 elements apart modulo 32 (64/G banks), so that the G lines of a
// group fall on disjoint banks.
__host__ __device__ constexpr int lds_line_len_spread(int L, int G) {
  return G <= 1 ? lds_line_len(L)
                : (L + L / 16 - 1) + ((32 / G - (L + L / 16 - 1) % 32) % 32 + 32) % 32;
}

// Slot of element x of the exchange after a Stockham stage of span p and
// radix R (float2 lines).  The stage's writes are runs of p lanes at stride
// p R elements (p = 1: single lanes at stride R); the swizzle moves run m of
// a 32-lane group to its own bank range by XOR-ing the bits of x below 32
// that vary inside a run with m.  The gather that follows reads 32 aligned
// consecutive elements, which the swizzle only permutes.  Only the five
// lowest bits of x change, so a slot stays inside its aligned run of 32.
template <int p, int R, bool PACKED, typename C> __device__ __forceinline__ int stage_slot(int x) {
  if constexpr (!PACKED || sizeof(C) != 8) {
    return lpad(x);
  } else if constexpr (p == 1) {
    return x ^ ((x >> 5) & (R - 1));
  } else if constexpr (p < 32 && p * R >= 64) {
    return x ^ (((x >> ilog2c(p * R)) & (32 / p - 1)) << ilog2c(p));
  } else {
    return x;
  }
}

// Stage twiddle tables: for every stage of span p > 1 (p = E, E^2, ... < L)
// the p entries exp(-2 pi i k / (p R)), k < p, stored contiguously in LDS one
// stage after the other, so that the butterflies of consecutive k read
// consecutive entries (no bank conflicts from strided table reads).  A span
// beyond 2048 (the last stage of an 8192-point line) keeps two shorter
// tables instead, the entries k = 64 j (j < p/64) and k < 64, whose product
// is entry k: 128 entries instead of 4096, so that an 8192-point line fits
// the LDS with room for a second work-group (float) or at all (double).
constexpr bool stage_tw_split(int p) { return p > 2048; }
constexpr int kStageFineBits = 6;
constexpr int stage_tw_entries(int p) {
  return stage_tw_split(p) ? (p >> kStageFineBits) + (1 << kStageFineBits) : p;
}
constexpr int stage_tw_len(int L, int E) {
  int n = 0;
  for (int p = E; p < L; p *= E) n += stage_tw_entries(p);
  return n;
}
constexpr int stage_tw_off(int p, int E) {
  int n = 0;
  for (int q = E; q < p; q *= E) n += stage_tw_entries(q);
  return n;
}
// index into a global table of 2^lmax_log entries exp(-2 pi i j / 2^lmax_log)
// of entry e of the concatenated stage tables of a length-L line
template <int L, int E> __device__ __forceinline__ int stage_tw_index(int e, int lmax_log) {
  int off = 0;
#pragma unroll
  for (int p = E; p < L; p *= E) {
    const int R = L / p < E ? L / p : E;
    if (e < off + stage_tw_entries(p)) {
      int k = e - off;  // entry k of the stage's table, or of its two tables
      if (stage_tw_split(p))
        k = k < (p >> kStageFineBits) ? k << kStageFineBits : k - (p >> kStageFineBits);
      return k << (lmax_log - ilog2c(p * R));
    }
    off += stage_tw_entries(p);
  }
  return 0;
}

// One Stockham stage of radix R and span p on a team line (compile-time L,
// E elements per thread).  Twiddles exp(-2 pi i q k / (p R)) are powers of
// the stage table's entry k; LAST: results stay in registers (index t + P j),
// else they go to LDS at the autosort position.
template <int L, int R, int p, bool INV, bool LAST, bool PACKED, int E, typename C>
__device__ __forceinline__ void stage(C (&v)[E], int t, C *lds, const C *tws) {
  constexpr int P = L / E;
  constexpr int NB = E / R;  // butterflies per thread
  static_assert(R >= 2 && R <= E && E % R == 0, "stage radix");
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int i = t + P * b;
    const int k = i & (p - 1);
    C u[R];
#pragma unroll
    for (int q = 0; q < R; ++q) u[q] = v[b + q * NB];
    if constexpr (p > 1) {
      // one table read per butterfly; the other twiddles are its powers
      C w[R];
      if constexpr (stage_tw_split(p)) {
        constexpr int o = stage_tw_off(p, E);
        w[1] = cmul(tws[o + (k >> kStageFineBits)],
                    tws[o + (p >> kStageFineBits) + (k & ((1 << kStageFineBits) - 1))]);
      } else {
        w[1] = tws[stage_tw_off(p, E) + k];
      }
      if (INV) w[1] = cconj(w[1]);
#pragma unroll
      for (int q = 2; q < R; ++q) w[q] = cmul(w[q / 2], w[q - q / 2]);
#pragma unroll
      for (int q = 1; q < R; ++q) u[q] = cmul(u[q], w[q]);
    }
    Dft<R, INV, C>::run(u);
    if constexpr (LAST) {
#pragma unroll
      for (int q = 0; q < R; ++q) v[b + q * NB] = u[q];
    } else {
      const int base = (i - k) * R + k;
#pragma unroll
      for (int q = 0; q < R; ++q) lds[stage_slot<p, R, PACKED, C>(base + q * p)] = u[q];
    }
  }
}

// the gather after the stage of span p (radix E)
template <int L, int E, int p, bool PACKED, typename C>
__device__ __forceinline__ void lds_gather(C (&v)[E], int t, const C *lds) {
  constexpr int P = L / E;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < E; ++j) v[j] = lds[stage_slot<p, E, PACKED, C>(t + P * j)];
  __syncthreads();
}

// Stages of span p, p E, p E^2, ... (radix E), the last of radix L / p.
template <int L, bool INV, bool PACKED, int E, int p, typename C>
__device__ __forceinline__ void team_stages(C (&v)[E], int t, C *lds, const C *tws) {
  if constexpr (p * E >= L) {
    stage<L, L / p, p, INV, true, PACKED, E>(v, t, lds, tws);
  } else {
    stage<L, E, p, INV, false, PACKED, E>(v, t, lds, tws);
    lds_gather<L, E, p, PACKED>(v, t, lds);
    team_stages<L, INV, PACKED, E, p * E>(v, t, lds, tws);
  }
}

// Complex FFT of length L held by a team of L/E threads (E = 16: radix-16
// stages; E = 8: radix-8 stages); tws: the LDS stage twiddle tables of a
// length-L line (stage_tw_len(L, E) entries).  Barriers are block-wide:
// every thread of the block calls this.  With lead_sync a barrier first
// protects LDS data still being read from earlier work.  PACKED selects the
// packed line layout (float2 only; see lslot).
template <int L, bool INV, bool PACKED = false, int E, typename C>
__device__ __forceinline__ void team_fft(C (&v)[E], int t, C *lds, const C *tws,
                                         bool lead_sync = true) {
  static_assert(L >= E && L <= 8192 && (L & (L - 1)) == 0, "line length");
  static_assert(E == 4 || E == 8 || E == 16, "elements per thread");
  if (lead_sync) __syncthreads();
  team_stages<L, INV, PACKED, E, 1>(v, t, lds, tws);
}

// The stage tables of a length-L line: issue the global reads into
// registers (tr, NR = ceil(stage_tw_len / nthreads) per thread) ...
template <int L, int E, int NR, typename C>
__device__ __forceinline__ void stage_tw_issue(C (&tr)[NR], const C *tw, int lmax_log, int tid,
                                               int nthreads) {
  constexpr int NC = stage_tw_len(L, E);
  if constexpr (NC > 0) {
    // every register is loaded (threads past the end re-read the last entry
    // and do not store it): a conditionally written register array would be
    // kept in scratch memory
#pragma unroll
    for (int u = 0; u < NR; ++u) {
      const int e = min(tid + u * nthreads, NC - 1);
      tr[u] = tw[stage_tw_index<L, E>(e, lmax_log)];
    }
  }
}
// ... and store them to LDS (before the barrier that precedes the FFT)
template <int L, int E, int NR, typename C>
__device__ __forceinline__ void stage_tw_store(const C (&tr)[NR], C *tws, int tid, int nthreads) {
  constexpr int NC = stage_tw_len(L, E);
#pragma unroll
  for (int u = 0; u < NR; ++u) {
    const int e = tid + u * nthreads;
    if (e < NC) tws[e] = tr[u];
  }
}

// ---- block reductions ----------------------------------------------------

template <typename T> __device__ __forceinline__ T wave_max(T x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    T y = __shfl_xor(x, o, 64);
    x = y > x ? y : x;
  }
  return x;
}
template <typename T> __device__ __forceinline__ T wave_min(T x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    T y = __shfl_xor(x, o, 64);
    x = y < x ? y : x;
  }
  return x;
}
template <typename T> __device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}
__device__ __forceinline__ int wave_or(int x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x |= __shfl_xor(x, o, 64);
  return x;
}

}  // namespace sweik
