// geom2d.hpp -- compile-time geometry of the 2D passes, shared by the host
// planner and the kernels.
//
//   row pass     one team of P = H1/E threads per grid row (E = 16 or 8
//                elements per thread); 4096/E threads per work-group, i.e.
//                rpw = 4096 / H1 rows (at least 1) for either E
//   column pass  one team of P = M0/E threads per spectral column; cpw =
//                4096 / M0 columns per work-group (one 8192-point column,
//                8192/E threads, in float32 with E = 16)
//   spectrum     half spectrum of the rows, blocked transposed:
//                spec[b][k1][rr], RB = 4 (float) or 2 (double) rows per block,
//                so that one block entry is 32 bytes
#pragma once

#include <cstddef>

#include "fft_team.hpp"

namespace sweik {

// ROW_LAST is the pass after the last convolution (no forcing, no forward
// transform: the float64 sum of the stored terms and the log); it is its own
// kernel so that the term passes are not sized for its registers.
// ROW_DGHAT, ROW_ADJ0_B and ROW_ADJ_B serve the full gradient: the kernel
// table's beta-derivative, and the adjoint passes that also carry the
// convolutions with it and the scalar partial sums.  ROW_GHATT and ROW_LASTT
// serve the far-field stabilised (tilted) solve: the rows of the tilted
// kernel table, and the last pass that undoes the tilt and keeps, per
// point, the best-conditioned of the tilts solved so far; COL_GHATC and
// COL_CONVC are the column passes with the tilted kernel's complex spectrum.
enum RowMode {
  ROW_GHAT = 0, ROW_PHI0 = 1, ROW_TERM = 2, ROW_ADJ0 = 3, ROW_ADJ = 4, ROW_SEED = 5, ROW_LAST = 6,
  ROW_DGHAT = 7, ROW_ADJ0_B = 8, ROW_ADJ_B = 9, ROW_GHATT = 10, ROW_LASTT = 11
};
enum ColMode { COL_GHAT = 0, COL_CONV = 1, COL_GHATC = 2, COL_CONVC = 3 };

template <typename R> constexpr int spec_rb() { return sizeof(R) == 4 ? 4 : 2; }
constexpr int kThreads = 256;
// threads of a 2D pass work-group with E elements per team thread
constexpr int team_threads(int E) { return kThreads * 16 / E; }
// Row passes: rows per work-group (kRowThreads / (H/16) rows at radix 16;
// one row when a row needs more threads) and threads per work-group.
constexpr int kRowThreads = 256;
constexpr int row_rpw(int H) { return H / 16 >= kRowThreads ? 1 : kRowThreads / (H / 16); }
constexpr int row_threads(int H, int E) { return row_rpw(H) * (H / E); }
constexpr int col_cpw(int M0) { return M0 / 16 >= kThreads ? 1 : kThreads / (M0 / 16); }
// threads of a column-pass work-group: 4096/E up to M0 = 4096, M0/E beyond
constexpr int col_threads(int M0, int E) { return col_cpw(M0) * (M0 / E); }
constexpr size_t kLdsDevice = 163840;  // gfx950 limit per work-group

// Split-step twiddles exp(-2 pi i k / 2H), k < H: one table of H entries up to
// H = 4096; beyond, a coarse table (k a multiple of 64) and a fine one
// (k < 64) whose product is the twiddle, so that an 8192-point row (float32)
// fits the LDS.
constexpr int kSplitFineBits = 6;
constexpr bool row_split2(int H) { return H > 4096; }
constexpr int row_twl_len(int H) {
  return row_split2(H) ? (H >> kSplitFineBits) + (1 << kSplitFineBits) : H;
}
// Row pass LDS: twiddle table(s) of the split steps (row_twl_len), the stage
// tables of the length-H FFT (room for either schedule), one padded line per
// row, and (when it fits) staging rows for the pointwise operands so that
// their loads are issued with the spectrum's.
template <typename R> constexpr int row_stage_tw(int H) {
  int n = stage_tw_len(H, 16);
  if (H > 4096) return n;  // rows beyond 4096 points run at radix 16 only
  n = stage_tw_len(H, 8) > n ? stage_tw_len(H, 8) : n;
  if (sizeof(R) == 4) n = stage_tw_len(H, 4) > n ? stage_tw_len(H, 4) : n;  // radix 4: float only
  return n;
}
// Line length of a row pass.  The tile transposes put Q = min(RPW, RB) rows
// in a 32-lane group (row fastest): float2 lines start 32/Q elements apart
// modulo 32, so the Q rows of a group fall on disjoint banks.
template <typename R> constexpr int row_tile_q(int H) {
  return row_rpw(H) < spec_rb<R>() ? row_rpw(H) : spec_rb<R>();
}
// double2 lines keep the padded layout; with the two rows of a block in a
// tile (16-byte accesses) they start 8 elements apart modulo 16, which the
// bank probe measured conflict-free for that interleave.
template <typename R> constexpr int row_line_len(int H) {
  return sizeof(R) != 4
             ? (row_tile_q<R>(H) > 1 ? (H + H / 16 - 1) + ((8 - (H + H / 16 - 1) % 16) % 16 + 16) % 16
                                     : lds_line_len(H))
             : H + (row_tile_q<R>(H) > 1 ? 32 / row_tile_q<R>(H) : 0);
}
template <typename R> constexpr size_t row_lds_core(int H) {
  return sizeof(R) * 2 *
         ((size_t)row_twl_len(H) + (size_t)row_stage_tw<R>(H) +
          (size_t)row_rpw(H) * row_line_len<R>(H));
}
// sources of the phi_0 row pass held in LDS (the rest are read from memory):
// 512, or 128 for rows beyond 4096 points, so that a double 8192-point row
// fits
constexpr int row_src_lds(int H) { return H > 4096 ? 128 : 512; }
// static shared memory of a row pass (block reductions, scalars, the term
// scales; phi_0 also holds up to row_src_lds sources and their weights), at
// least what the compiled kernels declare (group segment of the code
// objects: 1312 bytes for the other modes; phi_0 with 512 sources 12912 in
// float, 16960 in double, each source 8 + sizeof(R) bytes of it)
template <typename R> constexpr size_t row_lds_static(int mode, int H) {
  return mode == ROW_PHI0 ? (sizeof(R) == 4 ? 13312 : 17408) -
                                (size_t)(512 - row_src_lds(H)) * (8 + sizeof(R))
                          : 1536;
}
template <typename R> constexpr size_t row_stage_bytes(int H, int mode) {
  // per staged row: f for phi_0 (the source grid for its transform);
  // previous term, gamma or f, lambda (R) + gradient (double) for the
  // adjoint.  The forward terms hold gamma in registers.
  return (size_t)row_rpw(H) * H *
         (mode == ROW_PHI0 || mode == ROW_SEED
              ? sizeof(R)
              : (mode == ROW_ADJ || mode == ROW_ADJ_B) ? 3 * sizeof(R) + 8 : 0);
}
// Staging is used when it fits, unless it would cost the second work-group
// per CU that the pass has room for without it (the adjoint's 20 bytes per
// point at 2048 columns): then the operands are read from memory where they
// are used.  The full gradient's adjoint pass keeps its staging: its
// registers allow one work-group per CU anyway.
template <typename R> constexpr bool row_staged(int H, int mode) {
  const size_t plain = row_lds_core<R>(H) + row_lds_static<R>(mode, H);
  const size_t staged = plain + row_stage_bytes<R>(H, mode);
  return row_stage_bytes<R>(H, mode) > 0 && staged <= kLdsDevice &&
         (staged <= kLdsDevice / 2 || plain > kLdsDevice / 2 || mode == ROW_ADJ_B);
}
template <typename R> constexpr size_t row_lds_bytes(int H, int mode) {
  return row_lds_core<R>(H) + (row_staged<R>(H, mode) ? row_stage_bytes<R>(H, mode) : 0);
}
// dynamic + static shared memory of a row pass fits a work-group
template <typename R> constexpr bool row_fits(int H, int mode) {
  return row_lds_bytes<R>(H, mode) + row_lds_static<R>(mode, H) <= kLdsDevice;
}
// a row pass of length H with radix-E teams is built and planned: it fits the
// LDS, E <= H, and rows beyond 4096 complex points (one per work-group) take
// E = 16 only (512 threads)
template <typename R> constexpr bool row_ok(int H, int E, int mode) {
  return row_fits<R>(H, mode) && E <= H && (H <= 4096 || E == 16);
}
// the paired kernel-table + phi_0 pass (both passes' static shared memory,
// the larger dynamic size) is used where two of its work-groups fit a CU
template <typename R> constexpr size_t row_init_lds_bytes(int H) {
  return row_lds_bytes<R>(H, ROW_GHAT) > row_lds_bytes<R>(H, ROW_PHI0) ? row_lds_bytes<R>(H, ROW_GHAT)
                                                                       : row_lds_bytes<R>(H, ROW_PHI0);
}
template <typename R> constexpr bool row_init_pairs(int H) {
  return row_init_lds_bytes<R>(H) + row_lds_static<R>(ROW_GHAT, H) + row_lds_static<R>(ROW_PHI0, H) <=
         kLdsDevice / 2;
}
// Column pass LDS: the stage twiddle tables of the length-M0 FFT (room for
// any schedule) and one padded line per column.
template <typename R> constexpr int col_stage_tw(int M0) {
  int n = stage_tw_len(M0, 16);
  if (M0 > 4096) return n;  // columns beyond 4096 points run at radix 16 only
  n = stage_tw_len(M0, 8) > n ? stage_tw_len(M0, 8) : n;
  if (sizeof(R) == 4) n = stage_tw_len(M0, 4) > n ? stage_tw_len(M0, 4) : n;  // radix 4: float only
  return n;
}
// Line length of a column pass: the CPW columns of a work-group interleave
// their teams in a 32-lane group, so float2 lines are spread over the banks;
// double2 lines of two columns start 8 elements apart modulo 16.
template <typename R> constexpr int col_line_len(int M0) {
  return sizeof(R) == 4 ? lds_line_len_spread(M0, col_cpw(M0) < 32 ? col_cpw(M0) : 32)
         : col_cpw(M0) == 2 ? (M0 + M0 / 16 - 1) + ((8 - (M0 + M0 / 16 - 1) % 16) % 16 + 16) % 16
                            : lds_line_len(M0);
}
template <typename R> constexpr size_t col_lds_bytes(int M0) {
  return sizeof(R) * 2 * ((size_t)col_stage_tw<R>(M0) + (size_t)col_cpw(M0) * col_line_len<R>(M0));
}
constexpr size_t kColLdsStatic = 512;  // static shared memory of a column pass
template <typename R> constexpr bool col_fits(int M0) {
  return col_lds_bytes<R>(M0) + kColLdsStatic <= kLdsDevice;
}
// a column pass of length M0 with radix-E teams is built and planned: it fits
// the LDS, and columns beyond 4096 points (one per work-group) take E = 16
// only (512 threads; E = 8 would need 1024 threads at 128 registers each)
template <typename R> constexpr bool col_ok(int M0, int E) {
  return col_fits<R>(M0) && (M0 <= 4096 || E == 16);
}

}  // namespace sweik
