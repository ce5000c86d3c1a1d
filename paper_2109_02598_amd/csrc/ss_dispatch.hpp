// Launch planning and run-time dispatch of the templated kernels.
//
// Every kernel takes its tiling (rows or lines per workgroup) at run time
// and sizes its LDS dynamically, so one compiled kernel serves every tile
// choice and the autotuner can time the alternatives.  The launch
// functions are instantiated once per element type in ss_kernels_f32.hip /
// ss_kernels_f64.hip.
#pragma once

#include <hip/hip_ext.h>

#include "ss_adjoint.hpp"
#include "ss_batch.hpp"
#include "ss_fd.hpp"
#include "ss_kernels.hpp"
#include "ss_small.hpp"

namespace ss {

// Optional start/stop events recorded around a launch (kernel time only).
struct LaunchEvents {
  hipEvent_t start = nullptr, stop = nullptr;
};

// Threads per block limits (register budgets of the kernels).
constexpr int k_max_threads() { return 512; }
constexpr int y_max_threads() { return 1024; }

// ---- tile validity and defaults (host side, no templates) -----------------
inline bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

// x pass: `rows` rows (even) per block, as R/2 row pairs
inline bool x_tile_ok(int esz, int nx, int nf, int64_t nrows, int rows) {
  return is_pow2(rows) && rows >= 2 && rows <= 64 && rows <= nrows && nrows % rows == 0 &&
         x_lds(esz, nx, nf, rows) <= LDS_BUDGET;
}
inline int x_threads(int esz, int nx, int nf, int rows, bool sp = false) {
  const int S = nx / x_pts_for(esz, nx, nf, sp);
  int G = x_block_threads(esz, nx, nf, sp) / S;
  if (G > rows / 2) G = rows / 2;
  if (G < 1) G = 1;
  return G * S;
}
// persistent x pass: needs every pair of the tile in flight at once; only
// built with 8 points per thread (with 16, or with two FP64 fields, the
// prefetched values do not fit in the registers beside the transform)
inline bool x_pp_ok(int esz, int nx, int nf, int64_t nrows, int rows) {
  const int S = nx / x_pts(esz, nx, nf);
  return x_tile_ok(esz, nx, nf, nrows, rows) && (rows / 2) * S <= 512 && (rows / 2) * S >= 64 &&
         !(esz == 16 && nf == 2) && x_pts(esz, nx, nf) == 8 && !x_small(esz, nx, nf, nrows);
}
inline int x_tile_default(int esz, int nx, int nf, int64_t nrows) {
  // at most 128 contiguous bytes per staged chunk, at most half the LDS
  // (two blocks per CU), and enough blocks to cover the CUs twice
  int best = 2;
  for (int r = 2; r <= 64; r *= 2) {
    if (!x_tile_ok(esz, nx, nf, nrows, r)) break;
    if (r * esz > 128 || x_lds(esz, nx, nf, r) > LDS_BUDGET / 2) break;
    if (r > 2 && nrows / r < 256) break;
    best = r;
  }
  return best;
}

// y pass: `lines` lines (consecutive z) per block
inline bool y_tile_ok(int esz, int ny, int64_t nz, int lines) {
  return is_pow2(lines) && lines <= 64 && lines <= nz && nz % lines == 0 &&
         y_lds(esz, ny, lines) <= LDS_BUDGET;
}
inline int y_threads(int ny, int lines) {
  const int S = ny / 8;
  int G = y_max_threads() / S;
  if (G > lines) G = lines;
  if (G < 1) G = 1;
  return G * S;
}
inline int y_tile_default(int esz, int ny, int64_t nz) {
  int best = 1;
  for (int r = 1; r <= 64; r *= 2) {
    if (!y_tile_ok(esz, ny, nz, r)) break;
    if (r * esz > 128 || y_lds(esz, ny, r) > LDS_BUDGET / 2) break;
    best = r;
  }
  return best;
}

// k-space pass: `lines` lines per block (even in 3D: mirror pairs)
inline bool k_tile_ok(int esz, int nl, int64_t nlines, bool three_d, int lines) {
  const int S = nl / k_pts(esz, nl);   // the stepping form's threads per line (>= nl / 8)
  return is_pow2(lines) && lines <= nlines && nlines % lines == 0 && lines * S <= k_max_threads() &&
         (!three_d || lines >= 2) && k_lds(esz, nl, lines) <= LDS_BUDGET;
}
inline int k_tile_default(int esz, int nl, int64_t nlines, bool three_d) {
  const int S = nl / k_pts(esz, nl);
  int l = 256 / S > 1 ? 256 / S : 1;
  if (three_d && l < 2) l = 2;
  while (l > 1 && !k_tile_ok(esz, nl, nlines, three_d, l)) l /= 2;
  return l;
}

// structure-factor pass: the k-space line tiling plus the LDS histogram
inline bool sf_tile_ok(int esz, int nl, int64_t nlines, bool three_d, int lines, int nbins) {
  const int S = nl / 8;
  return is_pow2(lines) && lines <= nlines && nlines % lines == 0 && lines * S <= k_max_threads() &&
         (!three_d || lines >= 2) && sf_lds(esz, nl, lines, nbins) <= LDS_BUDGET;
}

// batched (grouped) launches: `threads` per block, `blocks` blocks
template <typename T>
hipError_t run_batch_x(BatchArgs b, int threads, int blocks, uint32_t lds, hipStream_t s, LaunchEvents ev);
template <typename T>
hipError_t run_batch_k(BatchArgs b, int threads, int blocks, uint32_t lds, hipStream_t s, LaunchEvents ev);
// single-launch form: the counter reset, then one launch of y.nsteps
// steps, one workgroup per work item
template <typename T>
hipError_t run_batch_single(BatchArgs b, BatchSync y, int threads, uint32_t lds, hipStream_t s, LaunchEvents ev);
// every step in one cooperative launch of `blocks` resident workgroups
// (blocks = 0: ask how many fit, into *fit)
template <typename T>
hipError_t run_batch_coop(BatchArgs b, BatchSync y, int threads, uint32_t lds, int blocks, int* fit, hipStream_t s,
                          LaunchEvents ev);

// adjoint (Gray-Scott, 2D): sizes 8 .. 1024
inline int xadj_tile(int esz, int nx, int64_t rows) {
  int best = 0;
  for (int r = 2; r <= 64; r *= 2) {
    if (r > rows || rows % r) break;
    if (xadj_lds(esz, nx, r) > (int64_t)LDS_BUDGET * 7 / 10) break;
    if ((r / 2) * (nx / adj_pts(nx)) > 512) break;
    best = r;
  }
  if (!best && xadj_lds(esz, nx, 2) <= LDS_BUDGET) best = 2;
  return best;
}
inline int kadj_tile(int nl, int64_t nlines) {
  const int S = nl / adj_pts(nl);
  int l = 256 / S > 1 ? 256 / S : 1;
  while (l > nlines) l /= 2;
  return l;
}
template <typename T>
hipError_t run_kadj(int nl, KAdjArgs a, hipStream_t s);
template <typename T>
hipError_t run_xadj(int nx, XAdjArgs a, hipStream_t s);

template <typename T>
hipError_t run_xpass(int nx, int nf, int mode, int nlm, XArgs a, hipStream_t s, LaunchEvents ev);
template <typename T>
hipError_t run_ypass(int ny, int dir, YArgs a, int64_t nkx, hipStream_t s, LaunchEvents ev);
template <typename T>
hipError_t run_kpass(int nl, KArgs a, int mode, hipStream_t s, LaunchEvents ev);
template <typename T>
hipError_t run_sfpass(int nl, SFArgs a, hipStream_t s);
template <typename T>
hipError_t run_sfreduce(SFArgs a, hipStream_t s);
template <typename T>
hipError_t run_fd(int dim, int stencil, FDArgs a, hipStream_t s);
template <typename T>
hipError_t run_finite(FiniteArgs a, hipStream_t s);
// one-workgroup run of a.nsteps steps of a square N x N one-field grid
// (N = 16 .. 128): the factor table, then the steps
inline bool small_size_ok(int n) { return n == 16 || n == 32 || n == 64 || n == 128; }
template <typename T>
hipError_t run_small(int n, SmallArgs a, hipStream_t s);
template <typename T>
hipError_t run_fd_eq(int dim, int stencil, int depth, FDArgs a, const FDEq& q, hipStream_t s);

#ifdef SS_DISPATCH_IMPL

template <typename K, typename... A>
hipError_t launch_with(K kernel, dim3 grid, dim3 block, uint32_t lds, hipStream_t s, LaunchEvents ev,
                       const A&... a) {
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  if (ev.start || ev.stop)
    hipExtLaunchKernelGGL(kernel, grid, block, lds, s, ev.start, ev.stop, 0, a...);
  else
    hipLaunchKernelGGL(kernel, grid, block, lds, s, a...);
  return hipGetLastError();
}

template <typename T, int NX, int NF, int MODE, int NLM>
hipError_t launch_x(XArgs a, hipStream_t s, LaunchEvents ev) {
  constexpr int ESZ = (int)sizeof(C<T>);
  const int R = a.rows_per_block;
  if (!x_tile_ok(ESZ, NX, NF, a.rows, R)) return hipErrorInvalidConfiguration;
  const int ntiles = (int)(a.rows / R);
  const bool sp = x_small(ESZ, NX, NF, a.rows);
  const int threads = x_threads(ESZ, NX, NF, R, sp);
  const uint32_t lds = (uint32_t)x_lds(ESZ, NX, NF, R);
  if constexpr (NX >= 8 && NX <= 512) {
    if (sp) return launch_with(xpass_kernel<T, NX, NF, MODE, NLM, true>, dim3(ntiles), dim3(threads), lds, s, ev, a);
  }
  if constexpr (MODE == XMODE_STEP && !(sizeof(T) == 8 && NF == 2) && XCfg<T, NX, NF>::P == 8) {
    if (a.tiles_per_block > 1 && x_pp_ok(ESZ, NX, NF, a.rows, R)) {
      const int grid = (ntiles + a.tiles_per_block - 1) / a.tiles_per_block;
      return launch_with(xpass_pp_kernel<T, NX, NF, NLM>, dim3(grid), dim3(threads), lds, s, ev, a, ntiles);
    }
  }
  return launch_with(xpass_kernel<T, NX, NF, MODE, NLM>, dim3(ntiles), dim3(threads), lds, s, ev, a);
}

#define SS_POW2_CASES(M) M(8) M(16) M(32) M(64) M(128) M(256) M(512) M(1024) M(2048) M(4096)

template <typename T, int NF, int MODE, int NLM>
hipError_t xdisp(int nx, const XArgs& a, hipStream_t s, LaunchEvents ev) {
  switch (nx) {
#define SS_CASE(n) \
  case n:          \
    return launch_x<T, n, NF, MODE, NLM>(a, s, ev);
    SS_POW2_CASES(SS_CASE)
#undef SS_CASE
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t run_xpass(int nx, int nf, int mode, int nlm, XArgs a, hipStream_t s, LaunchEvents ev) {
  if (mode == XMODE_FWD) return xdisp<T, 1, XMODE_FWD, NLIN_POLY>(nx, a, s, ev);
  if (mode == XMODE_INV) return xdisp<T, 1, XMODE_INV, NLIN_POLY>(nx, a, s, ev);
  if (nf == 1 && nlm == NLIN_THRESH) return xdisp<T, 1, XMODE_STEP, NLIN_THRESH>(nx, a, s, ev);
  if (nlm == NLIN_TABLE)
    return nf == 1 ? xdisp<T, 1, XMODE_STEP, NLIN_TABLE>(nx, a, s, ev) : xdisp<T, 2, XMODE_STEP, NLIN_TABLE>(nx, a, s, ev);
  if (nf == 1) return xdisp<T, 1, XMODE_STEP, NLIN_POLY>(nx, a, s, ev);
  if (nlm == NLIN_GS) return xdisp<T, 2, XMODE_STEP, NLIN_GS>(nx, a, s, ev);
  return xdisp<T, 2, XMODE_STEP, NLIN_MODELC>(nx, a, s, ev);
}

template <typename T, int NY, int DIR>
hipError_t launch_y(YArgs a, int64_t nkx, hipStream_t s, LaunchEvents ev) {
  constexpr int ESZ = (int)sizeof(C<T>);
  const int R = a.lines_per_block;
  if (!y_tile_ok(ESZ, NY, a.nz, R)) return hipErrorInvalidConfiguration;
  dim3 grid((unsigned)(nkx * (a.nz / R))), block((unsigned)y_threads(NY, R));
  return launch_with(ypass_kernel<T, NY, DIR>, grid, block, (uint32_t)y_lds(ESZ, NY, R), s, ev, a);
}

template <typename T>
hipError_t run_ypass(int ny, int dir, YArgs a, int64_t nkx, hipStream_t s, LaunchEvents ev) {
  switch (ny) {
#define SS_CASE(n)                                                       \
  case n:                                                                \
    return dir < 0 ? launch_y<T, n, -1>(a, nkx, s, ev) : launch_y<T, n, +1>(a, nkx, s, ev);
    SS_POW2_CASES(SS_CASE)
#undef SS_CASE
  }
  return hipErrorInvalidValue;
}

// mode: 0 = three transforms (T in, T out), 1 = stepping form (S^ and G in,
// S^ and T out), 2 = refresh S^ = FFT(T)/N_last only
template <typename T, int NL>
hipError_t launch_k(KArgs a, int mode, hipStream_t s, LaunchEvents ev) {
  constexpr int ESZ = (int)sizeof(C<T>);
  const int L = a.lines_per_block;
  if (!k_tile_ok(ESZ, NL, a.nlines, a.three_d != 0, L)) return hipErrorInvalidConfiguration;
  // threads per line: NL/8, or NL/k_pts for the stepping form
  dim3 grid((unsigned)(a.nlines / L), (unsigned)a.nf), block((unsigned)(L * (NL / 8)));
  dim3 block_hat((unsigned)(L * (NL / k_pts(ESZ, NL))));
  if (mode == 2) return launch_with(kfwd_kernel<T, NL>, grid, block, (uint32_t)k_lds(ESZ, NL, L), s, ev, a);
  const bool ch2 = a.fld[0].nonlin2 != nullptr;
  if (mode == 1 && ch2) {
    if (a.nf == 2 && !a.fld[1].nonlin2) return hipErrorInvalidValue;
    return a.scheme == 1
               ? launch_with(kpass_kernel<T, NL, true, 1, true>, grid, block_hat, (uint32_t)k_lds(ESZ, NL, L), s, ev, a)
               : launch_with(kpass_kernel<T, NL, true, 0, true>, grid, block_hat, (uint32_t)k_lds(ESZ, NL, L), s, ev, a);
  }
  if (mode == 1 && a.scheme == 1)
    return launch_with(kpass_kernel<T, NL, true, 1>, grid, block_hat, (uint32_t)k_lds(ESZ, NL, L), s, ev, a);
  if (mode == 1) return launch_with(kpass_kernel<T, NL, true>, grid, block_hat, (uint32_t)k_lds(ESZ, NL, L), s, ev, a);
  if (a.scheme != 0) return hipErrorInvalidValue;   // the three-transform form is ETD1 only
  return launch_with(kpass_kernel<T, NL, false>, grid, block, (uint32_t)k_lds(ESZ, NL, L), s, ev, a);
}

template <typename T>
hipError_t run_kpass(int nl, KArgs a, int mode, hipStream_t s, LaunchEvents ev) {
  switch (nl) {
#define SS_CASE(n) \
  case n:          \
    return launch_k<T, n>(a, mode, s, ev);
    SS_POW2_CASES(SS_CASE)
#undef SS_CASE
  }
  return hipErrorInvalidValue;
}

template <typename T, int NL>
hipError_t launch_sf(SFArgs a, hipStream_t s) {
  constexpr int ESZ = (int)sizeof(C<T>);
  const int L = a.lines_per_block;
  if (!sf_tile_ok(ESZ, NL, a.nlines, a.three_d != 0, L, a.nbins) || a.nblocks < 1)
    return hipErrorInvalidConfiguration;
  return launch_with(sfpass_kernel<T, NL>, dim3((unsigned)a.nblocks), dim3((unsigned)(L * (NL / 8))),
                     (uint32_t)sf_lds(ESZ, NL, L, a.nbins), s, LaunchEvents(), a);
}

template <typename T>
hipError_t run_sfpass(int nl, SFArgs a, hipStream_t s) {
  switch (nl) {
#define SS_CASE(n) \
  case n:          \
    return launch_sf<T, n>(a, s);
    SS_POW2_CASES(SS_CASE)
#undef SS_CASE
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t run_sfreduce(SFArgs a, hipStream_t s) {
  return launch_with(sf_reduce_kernel<T>, dim3((unsigned)((a.nbins + 31) / 32)), dim3(1024), 0, s,
                     LaunchEvents(), a);
}

// Cells along y per thread, chosen per stencil by measurement (CH, FP64,
// 2048^2 and 256^3; 1, 2 and 4 tried): two for the stencils whose loads
// along y overlap most per register spent (2D 9-point and fourth order,
// 3D axis-wise and fourth order), one otherwise.
constexpr int fd_rows(int dim, int st) {
  return dim == 2 ? (st == 0 ? 1 : 2) : (st == 0 || st == 4) ? 2 : 1;
}

// The z-marching kernel for the 3D wide stencils' one-Laplacian operations
// where the grid tiles into its blocks; false: use fd_kernel.
template <typename T, int ST>
bool launch_fd3_march(FDArgs a, hipStream_t s, hipError_t* e) {
  constexpr int HALO = fd_halo(3, ST);
  constexpr int TY = FD3_BY * fd3_rows(ST);
  if (a.nx % FD3_BX || a.ny % TY || a.nz % FD3_ZC) return false;
  const dim3 grid((unsigned)((a.nx / FD3_BX) * (a.ny / TY) * (a.nz / FD3_ZC))), block(256);
  switch (a.op) {
    case FD_AC: *e = launch_with(fd3_march_kernel<T, ST, FD_AC, HALO>, grid, block, 0, s, LaunchEvents(), a); return true;
    case FD_MU_CH: *e = launch_with(fd3_march_kernel<T, ST, FD_MU_CH, HALO>, grid, block, 0, s, LaunchEvents(), a); return true;
    case FD_UPD: *e = launch_with(fd3_march_kernel<T, ST, FD_UPD, HALO>, grid, block, 0, s, LaunchEvents(), a); return true;
    case FD_LAP: *e = launch_with(fd3_march_kernel<T, ST, FD_LAP, HALO>, grid, block, 0, s, LaunchEvents(), a); return true;
    case FD_MU_PFC: *e = launch_with(fd3_march_kernel<T, ST, FD_MU_PFC, HALO>, grid, block, 0, s, LaunchEvents(), a); return true;
    case FD_GS: *e = launch_with(fd3_march_kernel<T, ST, FD_GS, HALO>, grid, block, 0, s, LaunchEvents(), a); return true;
    case FD_MC: *e = launch_with(fd3_march_kernel<T, ST, FD_MC, HALO>, grid, block, 0, s, LaunchEvents(), a); return true;
    default: return false;
  }
}

template <typename T, int ST>
bool launch_fd2_march(FDArgs a, hipStream_t s, hipError_t* e) {
  constexpr int HALO = fd_halo(2, ST);
  if (a.nx % FD2_BX || a.ny % FD2_YC) return false;
  const dim3 grid((unsigned)((a.nx / FD2_BX) * (a.ny / FD2_YC))), block(256);
  switch (a.op) {
    case FD_AC: *e = launch_with(fd2_march_kernel<T, ST, FD_AC, HALO>, grid, block, 0, s, LaunchEvents(), a); return true;
    case FD_MU_CH: *e = launch_with(fd2_march_kernel<T, ST, FD_MU_CH, HALO>, grid, block, 0, s, LaunchEvents(), a); return true;
    case FD_UPD: *e = launch_with(fd2_march_kernel<T, ST, FD_UPD, HALO>, grid, block, 0, s, LaunchEvents(), a); return true;
    case FD_LAP: *e = launch_with(fd2_march_kernel<T, ST, FD_LAP, HALO>, grid, block, 0, s, LaunchEvents(), a); return true;
    case FD_MU_PFC: *e = launch_with(fd2_march_kernel<T, ST, FD_MU_PFC, HALO>, grid, block, 0, s, LaunchEvents(), a); return true;
    case FD_GS: *e = launch_with(fd2_march_kernel<T, ST, FD_GS, HALO>, grid, block, 0, s, LaunchEvents(), a); return true;
    case FD_MC: *e = launch_with(fd2_march_kernel<T, ST, FD_MC, HALO>, grid, block, 0, s, LaunchEvents(), a); return true;
    default: return false;
  }
}

template <typename T, int DIM, int ST>
hipError_t launch_fd(FDArgs a, hipStream_t s) {
  if constexpr (DIM == 2) {
    hipError_t e;
    if (launch_fd2_march<T, ST>(a, s, &e)) return e;
  }
  if constexpr (DIM == 3) {
    hipError_t e;
    if (launch_fd3_march<T, ST>(a, s, &e)) return e;
  }
  constexpr int R = fd_rows(DIM, ST);
  const int64_t n = a.nx * a.ny * a.nz / R;
  if (a.ny % R) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((n + 255) / 256)), block(256);
#define SS_FDOP(OP) \
  case OP: return launch_with(fd_kernel<T, DIM, ST, R, OP>, grid, block, 0, s, LaunchEvents(), a);
  switch (a.op) {
    SS_FDOP(FD_AC) SS_FDOP(FD_GS) SS_FDOP(FD_MU_CH) SS_FDOP(FD_UPD) SS_FDOP(FD_LAP) SS_FDOP(FD_MU_PFC)
    SS_FDOP(FD_MC)
    case FD_CH:   // the fused Cahn-Hilliard step: 2D axis-wise only
      if constexpr (DIM == 2 && ST == 0)
        return launch_with(fd_kernel<T, DIM, ST, R, FD_CH>, grid, block, 0, s, LaunchEvents(), a);
      return hipErrorInvalidValue;
  }
#undef SS_FDOP
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t run_fd(int dim, int stencil, FDArgs a, hipStream_t s) {
  if (dim == 2 && stencil == 0) return launch_fd<T, 2, 0>(a, s);
  if (dim == 2 && stencil == 9) return launch_fd<T, 2, 9>(a, s);
  if (dim == 2 && stencil == 4) return launch_fd<T, 2, 4>(a, s);
  if (dim == 2 && stencil == 17) return launch_fd<T, 2, 17>(a, s);
  if (dim == 2 && stencil == 21) return launch_fd<T, 2, 21>(a, s);
  if (dim == 3 && stencil == 0) return launch_fd<T, 3, 0>(a, s);
  if (dim == 3 && stencil == 15) return launch_fd<T, 3, 15>(a, s);
  if (dim == 3 && stencil == 21) return launch_fd<T, 3, 21>(a, s);
  if (dim == 3 && stencil == 19) return launch_fd<T, 3, 19>(a, s);
  if (dim == 3 && stencil == 27) return launch_fd<T, 3, 27>(a, s);
  if (dim == 3 && stencil == 4) return launch_fd<T, 3, 4>(a, s);
  return hipErrorInvalidValue;
}

// depth 0: no Laplacian (the stencil is unused); depth 1: one; the deeper
// level from an array (q.w) or from the fields; one or two fields
template <typename T, int NF>
hipError_t run_fd_eq_nf(int dim, int stencil, int depth, FDArgs a, const FDEq& q, hipStream_t s) {
  const bool lw = q.w[0] != nullptr;
  const dim3 block(256);
  auto grid = [&](int R) { return dim3((unsigned)((a.nx * a.ny * a.nz / R + 255) / 256)); };
#define SS_FDEQ(D, S, P)                                                                                        \
  if (dim == D && stencil == S && depth == P) {                                                                \
    constexpr int R = fd_rows(D, S);                                                                           \
    if (a.ny % R) return hipErrorInvalidValue;                                                                 \
    return lw ? launch_with(fd_eq_kernel<T, D, S, P, true, NF, R>, grid(R), block, 0, s, LaunchEvents(), a, q)  \
              : launch_with(fd_eq_kernel<T, D, S, P, false, NF, R>, grid(R), block, 0, s, LaunchEvents(), a, q); \
  }
  if (depth == 0) {
    if (dim == 2) return launch_with(fd_eq_kernel<T, 2, 0, 0, false, NF, 1>, grid(1), block, 0, s, LaunchEvents(), a, q);
    return launch_with(fd_eq_kernel<T, 3, 0, 0, false, NF, 1>, grid(1), block, 0, s, LaunchEvents(), a, q);
  }
  // one slot, one Laplacian, a grid the marching scheme tiles
  const int ty3 = FD3_BY * fd3_rows(stencil);
  const bool march = depth == 1 && q.nj == 1 &&
                     (dim == 2 ? (a.nx % FD2_BX == 0 && a.ny % FD2_YC == 0)
                               : (a.nx % FD3_BX == 0 && a.ny % ty3 == 0 && a.nz % FD3_ZC == 0));
#define SS_FDEQM(D, S)                                                                                        \
  if (march && dim == D && stencil == S) {                                                                    \
    constexpr int HALO = fd_halo(D, S);                                                                       \
    const dim3 g((unsigned)(D == 2 ? (a.nx / FD2_BX) * (a.ny / FD2_YC)                                       \
                                   : (a.nx / FD3_BX) * (a.ny / ty3) * (a.nz / FD3_ZC)));                      \
    return lw ? launch_with(fd_eq_march_kernel<T, D, S, true, NF, HALO>, g, block, 0, s, LaunchEvents(), a, q)  \
              : launch_with(fd_eq_march_kernel<T, D, S, false, NF, HALO>, g, block, 0, s, LaunchEvents(), a, q); \
  }
  SS_FDEQM(2, 0) SS_FDEQM(2, 9) SS_FDEQM(2, 4) SS_FDEQM(2, 17) SS_FDEQM(2, 21)
  SS_FDEQM(3, 0) SS_FDEQM(3, 15) SS_FDEQM(3, 19) SS_FDEQM(3, 21) SS_FDEQM(3, 27) SS_FDEQM(3, 4)
#undef SS_FDEQM
  SS_FDEQ(2, 0, 1) SS_FDEQ(2, 9, 1) SS_FDEQ(2, 4, 1) SS_FDEQ(2, 17, 1) SS_FDEQ(2, 21, 1)
  SS_FDEQ(3, 0, 1) SS_FDEQ(3, 15, 1) SS_FDEQ(3, 19, 1) SS_FDEQ(3, 21, 1) SS_FDEQ(3, 27, 1) SS_FDEQ(3, 4, 1)
#undef SS_FDEQ
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t run_fd_eq(int dim, int stencil, int depth, FDArgs a, const FDEq& q, hipStream_t s) {
  return a.in[1] ? run_fd_eq_nf<T, 2>(dim, stencil, depth, a, q, s) : run_fd_eq_nf<T, 1>(dim, stencil, depth, a, q, s);
}

template <typename T>
hipError_t run_batch_x(BatchArgs b, int threads, int blocks, uint32_t lds, hipStream_t s, LaunchEvents ev) {
  return launch_with(xpass_grouped<T>, dim3(blocks), dim3(threads), lds, s, ev, b);
}
template <typename T>
hipError_t run_batch_k(BatchArgs b, int threads, int blocks, uint32_t lds, hipStream_t s, LaunchEvents ev) {
  return launch_with(kpass_grouped<T>, dim3(blocks), dim3(threads), lds, s, ev, b);
}
template <typename T>
hipError_t run_batch_single(BatchArgs b, BatchSync y, int threads, uint32_t lds, hipStream_t s, LaunchEvents ev) {
  if (threads < 64 || threads > 512 || y.nsteps < 1) return hipErrorInvalidConfiguration;
  const uint64_t items = (uint64_t)(b.x_total + b.k_total) * (uint64_t)y.nsteps;
  if (items * (uint64_t)threads > 0xffffffffull) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(batch_sync_reset<T>, dim3(1), dim3(256), 0, s, b, y);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_with(batch_single<T>, dim3((unsigned)items), dim3(threads), lds, s, ev, b, y);
}

template <typename T>
hipError_t run_batch_coop(BatchArgs b, BatchSync y, int threads, uint32_t lds, int blocks, int* fit, hipStream_t s,
                          LaunchEvents ev) {
  if (threads < 64 || threads > 512) return hipErrorInvalidConfiguration;
  const void* k = (const void*)batch_coop<T>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  if (blocks == 0) {
    int dev = 0, ncu = 0, per = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, threads, lds);
    if (e != hipSuccess) return e;
    *fit = per * ncu;
    return hipSuccess;
  }
  if (y.nsteps < 1) return hipErrorInvalidConfiguration;
  hipError_t e = hipSuccess;
  if (ev.start) {
    e = hipEventRecord(ev.start, s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(batch_sync_reset<T>, dim3(1), dim3(256), 0, s, b, y);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  void* args[2] = {(void*)&b, (void*)&y};
  e = hipLaunchCooperativeKernel(k, dim3((unsigned)blocks), dim3((unsigned)threads), args, lds, s);
  if (e != hipSuccess) return e;
  if (ev.stop) e = hipEventRecord(ev.stop, s);
  return e;
}

#define SS_ADJ_CASES(M) M(8) M(16) M(32) M(64) M(128) M(256) M(512) M(1024)

template <typename T>
hipError_t run_kadj(int nl, KAdjArgs a, hipStream_t s) {
  constexpr int ESZ = (int)sizeof(C<T>);
  const int L = a.lines_per_block;
  const int threads = L * (nl / adj_pts(nl));
  if (L < 1 || a.nlines % L || threads > 512) return hipErrorInvalidConfiguration;
  const int64_t lds = kadj_lds(ESZ, nl, L, threads);
  if (lds > LDS_BUDGET) return hipErrorInvalidConfiguration;
  dim3 grid((unsigned)(a.nlines / L), 2), block((unsigned)threads);
  switch (nl) {
#define SS_CASE(n) \
  case n:          \
    return launch_with(kadj_kernel<T, n>, grid, block, (uint32_t)lds, s, LaunchEvents(), a);
    SS_ADJ_CASES(SS_CASE)
#undef SS_CASE
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t run_xadj(int nx, XAdjArgs a, hipStream_t s) {
  constexpr int ESZ = (int)sizeof(C<T>);
  const int R = a.rows_per_block;
  if (R < 2 || !is_pow2(R) || a.rows % R) return hipErrorInvalidConfiguration;
  const int64_t lds = xadj_lds(ESZ, nx, R);
  if (lds > LDS_BUDGET) return hipErrorInvalidConfiguration;
  const int S = nx / adj_pts(nx);
  int G = 512 / S;
  if (G > R / 2) G = R / 2;
  if (G < 1) G = 1;
  dim3 grid((unsigned)(a.rows / R)), block((unsigned)(G * S));
  switch (nx) {
#define SS_CASE(n) \
  case n:          \
    return launch_with(xadj_kernel<T, n>, grid, block, (uint32_t)lds, s, LaunchEvents(), a);
    SS_ADJ_CASES(SS_CASE)
#undef SS_CASE
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t run_finite(FiniteArgs a, hipStream_t s) {
  if (a.narr < 1 || a.narr > 2 || a.n < 1 || !a.flag) return hipErrorInvalidValue;
  hipLaunchKernelGGL(finite_clear_kernel<T>, dim3(1), dim3(64), 0, s, a);
  int64_t blocks = (a.n + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL(finite_kernel<T>, dim3((unsigned)blocks, (unsigned)a.narr), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <typename T, int N>
hipError_t launch_small(SmallArgs a, hipStream_t s) {
  constexpr int W = SmallCfg<T, N>::W;
  constexpr uint32_t lds = (uint32_t)small_lds((int)sizeof(C<T>), N);
  static_assert(small_lds((int)sizeof(C<T>), N) <= LDS_BUDGET, "LDS");
  hipLaunchKernelGGL((small_coef_kernel<T, N>), dim3(1), dim3(W), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_with(small_step_kernel<T, N>, dim3(1), dim3(W), lds, s, LaunchEvents(), a);
}

template <typename T>
hipError_t run_small(int n, SmallArgs a, hipStream_t s) {
  if (a.nsteps < 0) return hipErrorInvalidValue;
  switch (n) {
    case 16: return launch_small<T, 16>(a, s);
    case 32: return launch_small<T, 32>(a, s);
    case 64: return launch_small<T, 64>(a, s);
    case 128: return launch_small<T, 128>(a, s);
  }
  return hipErrorInvalidValue;
}

#define SS_INSTANTIATE(T)                                                                  \
  template hipError_t run_small<T>(int, SmallArgs, hipStream_t);                          \
  template hipError_t run_finite<T>(FiniteArgs, hipStream_t);                             \
  template hipError_t run_kadj<T>(int, KAdjArgs, hipStream_t);                          \
  template hipError_t run_xadj<T>(int, XAdjArgs, hipStream_t);                          \
  template hipError_t run_batch_x<T>(BatchArgs, int, int, uint32_t, hipStream_t, LaunchEvents); \
  template hipError_t run_batch_k<T>(BatchArgs, int, int, uint32_t, hipStream_t, LaunchEvents); \
  template hipError_t run_batch_single<T>(BatchArgs, BatchSync, int, uint32_t, hipStream_t, LaunchEvents); \
  template hipError_t run_batch_coop<T>(BatchArgs, BatchSync, int, uint32_t, int, int*, hipStream_t, LaunchEvents); \
  template hipError_t run_xpass<T>(int, int, int, int, XArgs, hipStream_t, LaunchEvents); \
  template hipError_t run_ypass<T>(int, int, YArgs, int64_t, hipStream_t, LaunchEvents);  \
  template hipError_t run_kpass<T>(int, KArgs, int, hipStream_t, LaunchEvents);           \
  template hipError_t run_sfpass<T>(int, SFArgs, hipStream_t);                            \
  template hipError_t run_sfreduce<T>(SFArgs, hipStream_t);                                \
  template hipError_t run_fd<T>(int, int, FDArgs, hipStream_t);                           \
  template hipError_t run_fd_eq<T>(int, int, int, FDArgs, const FDEq&, hipStream_t);

#endif  // SS_DISPATCH_IMPL

}  // namespace ss
