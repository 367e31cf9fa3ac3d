// plan.hpp -- host-side plan of a solve: the problem, its padded geometry,
// the kernel schedule and the workspace / checkpoint layout.
#pragma once

#include <cmath>
#include <cstddef>
#include <cstdint>

#include "sweik.h"

namespace sweik {

struct Geo2 {
  int n0, n1;
  int M0, H0, ldg;   // column FFT length, half, kernel-spectrum leading dim
  int H1, ldk;       // row half length, spectral columns
  int RB, nb;        // rows per spectral block, blocks
  int rpw, cpw;      // rows per row WG, columns per column WG
  int nbr, ncw;      // row WGs, column WGs
  int lmax, lmax_log;
  int erow, ecol;    // schedule: elements per team thread of the row / column passes
  int phi0_fft;      // phi_0 by FFT of the source grid (Table 1 steps 1-5)
};

struct Geo3 {
  int n0, n1, n2;
  int M0, M1, M2, H0, H1, H2;
  int nlines, nbx;     // x-pass lines and work-groups
  int ncb0, ncb1;      // column blocks per plane of the z and y passes
  long long ld2;       // plane stride of s2 (complex elements)
  int lmax, lmax_log;
};

struct Layout {      // byte offsets into the workspace / checkpoint
  size_t par, red, expo, mu, mu_red, tw, g, g0, spec, spec0, s2, acc, terms, lam, gam, total;
  size_t ck_expo, ck_par, ck_g, ck_phi, ck_terms, ck_total;
  // full gradient: after `total`, a second spectrum, the per-work-group
  // partial sums and the argmin / argmax partials (the kernel table's
  // beta-derivative spectrum: g0, in 2D part of the solve's workspace, in 3D
  // also after `total`)
  size_t fg_spec2, fg_part, fg_ext, fg_total;
};

}  // namespace sweik

struct sweik_plan_s {
  sweik_problem p;
  int64_t padded[3];
  size_t lds_max;
  sweik::Geo2 g2;
  sweik::Geo3 g3;
  sweik::Layout ws;
};
