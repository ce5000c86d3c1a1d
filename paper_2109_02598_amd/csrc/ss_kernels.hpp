// Kernels of one semi-implicit Fourier spectral step (gfx950).
//
// Spectral state layout (both 2D and 3D): the field is kept transformed
// along x (and along y in 3D) and scaled, in a transposed complex array
//     T[kx][s],  kx = 0 .. Nx/2-1,  s = y*Nz + z  (Nz = 1 in 2D)
// so that lines along the last axis (y in 2D, z in 3D) are contiguous.
// Because the field is real, its kx = 0 and kx = Nx/2 planes are real in
// the remaining coordinates; they are stored together as one complex plane
// kx = 0 holding  S(0, .) + i S(Nx/2, .).  Every array is therefore exactly
// Nx*Ny*Nz reals.
//
// Scaling: 2D state T = FFT_x(psi)/Nx;  3D state = FFT_xy(psi)/(Nx Ny).
// The x pass inverts with an unnormalised transform, so psi comes out
// directly; the k-space pass folds 1/N_last into A and 1/N into B N.
//
// Kernels
//   xpass  rows along x, two real rows per complex FFT; modes
//          FWD  (real rows -> spectral, set-up),
//          INV  (spectral -> real rows, read-out),
//          STEP (spectral -> psi -> nonlinear f -> spectral of f).
//   ypass  3D only: complex FFT along y on chunks of consecutive z.
//   kpass  lines along the last axis: forward FFT of the state and of the
//          nonlinear term, ETD1 update  U = a T^ + b G^  (Sec. 2.4.2,
//          Eqs. 3-4 and 8), inverse FFT, in place; the packed kx = 0
//          lines are split into their two Hermitian parts with the mirror
//          mode (-k) before the update.
#pragma once

#include <type_traits>

#include "ss_fft.hpp"

namespace ss {

enum { XMODE_FWD = 0, XMODE_INV = 1, XMODE_STEP = 2 };
// NLIN_THRESH is no equation of motion: it maps psi to the occupancy
// [psi > 0] of the structure factor (Sec. 3).
enum { NLIN_POLY = 0, NLIN_GS = 1, NLIN_MODELC = 2, NLIN_THRESH = 3, NLIN_TABLE = 4 };

constexpr int LDS_BUDGET = 160 * 1024;

// Index of spectral element (kx, s) (kx < H, s = row).  Rows are grouped in
// blocks of B = 2^lb consecutive rows; inside a block the layout is
// [kx][s mod B] and blocks follow each other, so
//   index = ((s >> lb) * H + kx) * B + (s mod B).
// The x pass then reads a block of rows as one contiguous region, while
// the k-space pass reads a line as chunks of B consecutive elements.  With
// B = rows this is the plain transposed layout [kx][s].
__device__ __forceinline__ int64_t sidx(int64_t kx, int64_t s, int64_t H, int lb) {
  return (((s >> lb) * H + kx) << lb) + (s & ((int64_t(1) << lb) - 1));
}

// Compile-time loop: f(std::integral_constant<int, I>) for I in [B, E), so
// register arrays are only ever indexed by constants.
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>());
    static_for<B + 1, E>(f);
  }
}

#ifndef SS_KWAVES
#define SS_KWAVES 2
#endif
// FP32 factors: 1 takes A = 2^(z log2 e) from the hardware exponential
// (relative error about |z| 6e-8: where that exceeds FP32 rounding, A is
// below e^-1 and the mode decays) instead of the library's expf; 2% of an
// FP32 step at 2048^2
#ifndef SS_FAST_EXPF
#define SS_FAST_EXPF 1
#endif

// LDS geometry shared by the kernels and the host-side launch planning
// (esz = bytes of one complex element: 8 for FP32, 16 for FP64).
constexpr int padded_len_e(int esz, int n) { return esz == 16 ? n + (n >> 3) + 1 : n + (n >> 4) + 1; }
// x pass region stride: NF*REG = 2 (mod 8 or 16) keeps the staged rows of a
// block on distinct banks
constexpr int x_reg(int esz, int nx, int nf) {
  int r = padded_len_e(esz, nx);
  const int mod = esz == 16 ? 8 : 16;
  while (((nf * r) % mod) != 2 % mod) ++r;
  return r;
}
constexpr int64_t x_lds(int esz, int nx, int nf, int rows) { return (int64_t)(rows / 2) * nf * x_reg(esz, nx, nf) * esz; }
// y pass region stride = 1 (mod 8 or 16)
constexpr int y_reg(int esz, int ny) {
  int r = padded_len_e(esz, ny);
  const int mod = esz == 16 ? 8 : 16;
  while ((r % mod) != 1) ++r;
  return r;
}
constexpr int64_t y_lds(int esz, int ny, int lines) { return (int64_t)lines * y_reg(esz, ny) * esz; }
constexpr int k_reg(int esz, int nl) { return padded_len_e(esz, nl); }
// twiddle bases per thread of an nl-point transform with p points per
// thread (Twiddles<T, nl, p>::NW)
constexpr int k_nw(int nl, int p = 8) {
  return ((ilog2c(nl) + ilog2c(p) - 1) / ilog2c(p)) > 1 ? ((ilog2c(nl) + ilog2c(p) - 1) / ilog2c(p)) - 1 : 1;
}
// points per thread of the stepping-form k-space pass.  Eight: with 16 the
// FP64 pass spills even at 256 VGPRs, and the FP32 pass drops to two waves
// per SIMD and ran 6% slower at 2048 points.  Four on lines of up to 512
// points, where a step has too few lines to fill the GPU and a line's
// serial chain of loads and transform stages sets the time (Allen-Cahn
// 128^2 FP64 16.2 -> 13.7 us per step, 256^2 16.8 -> 13.3, 512^2 18.4 ->
// 16.5; PFC 256^3, whose lines are 256 points long but many, unchanged).
constexpr int k_pts(int, int nl) { return nl <= 512 ? 4 : 8; }
// FP64 k-space blocks keep the twiddle bases of the stepping-form pass in
// LDS after the line regions
// (sized for 8 points per thread, the three-transform form's, or the
// stepping form's count, whichever needs more)
constexpr int64_t k_twl(int esz, int nl) {
  return esz != 16 ? 0
                   : ((nl / 8) * k_nw(nl, 8) > (nl / k_pts(esz, nl)) * k_nw(nl, k_pts(esz, nl))
                          ? (nl / 8) * k_nw(nl, 8)
                          : (nl / k_pts(esz, nl)) * k_nw(nl, k_pts(esz, nl)));
}
constexpr int64_t k_lds(int esz, int nl, int lines) { return (int64_t)lines * (k_reg(esz, nl) + k_twl(esz, nl)) * esz; }

#ifndef SS_XPTS16
#define SS_XPTS16 1
#endif
// Points per thread of the x pass's transforms (the FFT's P): 16 (one LDS
// exchange fewer per 2048-point transform than 8) except on 8-point rows
// and in the two-field FP64 pass, which needs the registers for its second
// field.  The other passes use 8.
constexpr int x_pts(int esz, int nx, int nf) {
  return (SS_XPTS16 && nx >= 16 && !(esz == 16 && nf == 2)) ? 16 : 8;
}
// A small grid's x pass takes 4 points per thread: rows of 8 to 512 points
// when a launch at the count above would hold fewer than 64K threads (too
// few waves to hide each one's chain of loads and transform stages).
// Chosen at run time from the grid (both kernels are built for such rows).
constexpr bool x_small(int esz, int nx, int nf, int64_t nrows) {
  return nx >= 8 && nx <= 512 && (nrows / 2) * (nx / x_pts(esz, nx, nf)) < 65536;
}
constexpr int x_pts_for(int esz, int nx, int nf, bool sp) { return sp ? 4 : x_pts(esz, nx, nf); }
// threads per x-pass block: 512, or 1024 for FP32 with 8 points per thread
constexpr int x_block_threads(int esz, int nx, int nf, bool sp = false) {
  return (esz == 8 && x_pts_for(esz, nx, nf, sp) == 8) ? 1024 : 512;
}

// ---------------------------------------------------------------------------
// x pass
// ---------------------------------------------------------------------------
// Explicit terms of an equation read at run time (NLIN_TABLE), as dense
// polynomials: field j's pointwise function is
//   E_j(u, v) = sum_{k <= dv[j]} v^k H_jk(u),  H_jk(u) = sum_{i <= du[j][k]} a[j][k][i] u^i
// with u, v the fields 0 and 1 (exponents at most 7); af is a in FP32.
struct NTab {
  int dv[2];
  int du[2][8];
  double a[2][8][8];
  float af[2][8][8];
};

struct XArgs {
  const void* spec_in[2];   // per field, T[kx][s] (INV, STEP)
  void* spec_out[2];        // per field, (FWD, STEP); may alias spec_in
  const void* real_in;      // FWD: real field (z, y, x)
  void* real_out;           // INV: real field (z, y, x)
  int64_t rows;             // Ny*Nz = leading dimension of T
  int nz, ny;               // s = y*nz + z ; real row offset (z*ny + y)*Nx
  int rows_per_block;       // R at run time (even, divides rows)
  int tiles_per_block;      // STEP: > 1 selects the persistent, prefetching kernel
  int lb;                   // log2 of the row block of the spectral layout
  int xcd_remap;            // 1: spread consecutive chunks over one XCD
  double scale;             // multiplies the forward output (1/Nx for FWD)
  double p[5];              // nonlinear coefficients
  NTab tab;                 // NLIN_TABLE: the explicit terms as monomials
};

template <typename T, int NX, int NF, bool SP = false>
struct XCfg {
  static constexpr int P = x_pts_for((int)sizeof(C<T>), NX, NF, SP);   // points per thread
  static constexpr int S = NX / P;                  // threads per line
  static constexpr int H = NX / 2;                  // stored kx count
  static constexpr int ESZ = (int)sizeof(C<T>);
  // HB = H + 1 is the offset of the second row of a pair in its region
  static constexpr int HB = H + 1;
  static constexpr int reg_for(int nf) { return x_reg(ESZ, NX, nf); }
};

__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb, int remap) {
  // workgroups are dealt round-robin to the 8 XCDs; give each XCD a
  // contiguous range of chunks so neighbours share its L2
  if (!remap || (nb & 7)) return b;
  return (b & 7) * (nb >> 3) + (b >> 3);
}

// ---- staged copies between the spectral layout and x-pass LDS regions ----
// A tile is the R rows s0 .. s0+R-1 (R a power of two) of NS arrays.  Row r
// of array f sits in LDS at region((r/2)*NR + F0 + f) + (r&1)*HB + kx
// (region stride REG, NR regions per row pair).  Per array the tile's
// elements are ordered (kx, r) with r fastest and thread tid moves the
// elements tid + q*nthr, so a wave reads R consecutive rows of consecutive
// kx.  When nthr >= R the thread's row r = tid mod R is fixed: its global
// index is one row offset plus kx*B (B = 2^lb row block) and kx advances by
// nthr/R per element.  Eight loads (four when a thread's share is not a
// multiple of eight) are issued before their LDS writes; the arrays are
// walked one after the other so that each pointer is chosen at compile
// time.  Elements per thread and array: H*R/nthr = R*P/(2*G), a multiple
// of 4 for the x-pass launch shapes (nthr = G*NX/P with G dividing R/2, P
// at least 4).
template <int H>
__device__ __forceinline__ int64_t xstage_row(int64_t s, int lb) {
  return (((s >> lb) * H) << lb) + (s & ((int64_t(1) << lb) - 1));
}

// QB loads in flight before their LDS writes; per (a thread's elements of
// the tile) is a multiple of QB.
template <typename T, int QB>
__device__ __forceinline__ void xstage_in_run(C<T>* lrow, const C<T>* g, int per, int k0, int kstep, int lb) {
  for (int c = 0; c < per; c += QB, k0 += QB * kstep) {
    T vr[QB], vi[QB];   // scalar arrays: promoted to registers
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      const C<T> v = g[(int64_t)(k0 + q * kstep) << lb];
      vr[q] = v.x;
      vi[q] = v.y;
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) lrow[k0 + q * kstep] = mk<T>(vr[q], vi[q]);
  }
}
template <typename T, int QB>
__device__ __forceinline__ void xstage_out_run(C<T>* g, const C<T>* lrow, int per, int k0, int kstep, int lb) {
  for (int c = 0; c < per; c += QB, k0 += QB * kstep) {
    T vr[QB], vi[QB];
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      const C<T> v = lrow[k0 + q * kstep];
      vr[q] = v.x;
      vi[q] = v.y;
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) g[(int64_t)(k0 + q * kstep) << lb] = mk<T>(vr[q], vi[q]);
  }
}

template <typename T, int H, int NS, int NR, int F0, int REG, int HB>
__device__ __forceinline__ void xstage_in(C<T>* lds, const C<T>* const (&src)[NS], int64_t s0,
                                          int R, int lb, int tid, int nthr) {
  const int lr = __builtin_ctz((unsigned)R);
  if (nthr >= R) {
    const int r = tid & (R - 1);
    const int64_t row = xstage_row<H>(s0 + r, lb);
    const int kstep = nthr >> lr;
    const int per = (H * R) / nthr;
#pragma unroll
    for (int f = 0; f < NS; ++f) {
      const C<T>* g = src[f] + row;
      C<T>* lrow = lds + ((r >> 1) * NR + F0 + f) * REG + (r & 1) * HB;
      if (per % 8 == 0) xstage_in_run<T, 8>(lrow, g, per, tid >> lr, kstep, lb);
      else xstage_in_run<T, 4>(lrow, g, per, tid >> lr, kstep, lb);
    }
  } else {
#pragma unroll
    for (int f = 0; f < NS; ++f) {
      for (int i = tid; i < H * R; i += nthr) {
        const int r = i & (R - 1), kx = i >> lr;
        lds[((r >> 1) * NR + F0 + f) * REG + (r & 1) * HB + kx] =
            src[f][xstage_row<H>(s0 + r, lb) + ((int64_t)kx << lb)];
      }
    }
  }
}

template <typename T, int H, int NS, int NR, int F0, int REG, int HB>
__device__ __forceinline__ void xstage_out(C<T>* const (&dst)[NS], const C<T>* lds, int64_t s0,
                                           int R, int lb, int tid, int nthr) {
  const int lr = __builtin_ctz((unsigned)R);
  if (nthr >= R) {
    const int r = tid & (R - 1);
    const int64_t row = xstage_row<H>(s0 + r, lb);
    const int kstep = nthr >> lr;
    const int per = (H * R) / nthr;
#pragma unroll
    for (int f = 0; f < NS; ++f) {
      C<T>* g = dst[f] + row;
      const C<T>* lrow = lds + ((r >> 1) * NR + F0 + f) * REG + (r & 1) * HB;
      if (per % 8 == 0) xstage_out_run<T, 8>(g, lrow, per, tid >> lr, kstep, lb);
      else xstage_out_run<T, 4>(g, lrow, per, tid >> lr, kstep, lb);
    }
  } else {
#pragma unroll
    for (int f = 0; f < NS; ++f) {
      for (int i = tid; i < H * R; i += nthr) {
        const int r = i & (R - 1), kx = i >> lr;
        dst[f][xstage_row<H>(s0 + r, lb) + ((int64_t)kx << lb)] =
            lds[((r >> 1) * NR + F0 + f) * REG + (r & 1) * HB + kx];
      }
    }
  }
}

template <typename T, int NLM>
__device__ __forceinline__ void nonlinear(C<T>* c0, C<T>* c1, T p0, T p1, T p2) {
  if constexpr (NLM == NLIN_POLY) {
    // f = a2 psi^2 + a3 psi^3 on both packed rows
    const T a2 = p0, a3 = p1;
    T x = c0->x, y = c0->y;
    c0->x = x * x * (a2 + a3 * x);
    c0->y = y * y * (a2 + a3 * y);
  } else if constexpr (NLM == NLIN_GS) {
    // g_u = F - u v^2, g_v = u v^2
    const T F = p0;
    T ux = c0->x, uy = c0->y, vx = c1->x, vy = c1->y;
    T wx = ux * vx * vx, wy = uy * vy * vy;
    c0->x = F - wx; c0->y = F - wy;
    c1->x = wx;     c1->y = wy;
  } else if constexpr (NLM == NLIN_THRESH) {
    // occupancy rho = 1 where psi > 0, else 0, on both packed rows
    c0->x = c0->x > (T)0 ? (T)1 : (T)0;
    c0->y = c0->y > (T)0 ? (T)1 : (T)0;
  } else {
    // model C: f_psi = -c2 psi^3 + 2 c5 psi m ; f_m = -c4 m^3 + c5 psi^2
    const T c2 = p0, c4 = p1, c5 = p2;
    T px = c0->x, py = c0->y, mx = c1->x, my = c1->y;
    c0->x = px * (-c2 * px * px + (T)2 * c5 * mx);
    c0->y = py * (-c2 * py * py + (T)2 * c5 * my);
    c1->x = mx * mx * (-c4 * mx) + c5 * px * px;
    c1->y = my * my * (-c4 * my) + c5 * py * py;
  }
}

// E_j of the table on W values at once: Horner in u for each power of v
// (the coefficients unrolled over their 8 slots with uniform guards, so
// their loads sit at fixed offsets and serve all W values), then Horner
// in v.
template <typename T, int NF, int W>
__device__ __forceinline__ void ntab_eval(const NTab& tb, int j, const T (&u)[W], const T (&v)[W], T (&acc)[W]) {
#pragma unroll
  for (int w = 0; w < W; ++w) acc[w] = (T)0;
  const int kmax = NF == 2 ? tb.dv[j] : 0;
  for (int k = kmax; k >= 0; --k) {
    const int dk = tb.du[j][k];
    T ak[8];   // the row, loaded whole before the guards: one batch of loads
#pragma unroll
    for (int i = 0; i < 8; ++i) ak[i] = sizeof(T) == 8 ? (T)tb.a[j][k][i] : (T)tb.af[j][k][i];
    T h[W];
#pragma unroll
    for (int w = 0; w < W; ++w) h[w] = (T)0;
#pragma unroll
    for (int i = 7; i >= 0; --i) {
      if (i <= dk) {
#pragma unroll
        for (int w = 0; w < W; ++w) h[w] = h[w] * u[w] + ak[i];
      }
    }
#pragma unroll
    for (int w = 0; w < W; ++w) acc[w] = NF == 2 ? acc[w] * v[w] + h[w] : h[w];
  }
}

// NLIN_TABLE over a thread's PT cells (two packed rows each), in chunks
// of 4 cells; every E_j reads the fields of the current step (a chunk's
// inputs are all read before its outputs are written).
template <typename T, int NF, int PT>
__device__ __forceinline__ void nonlinear_table(C<T> (&c)[NF][PT], const NTab& tb) {
  constexpr int CH = 4, W = 2 * CH;
  static_assert(PT % CH == 0, "chunk size");
#pragma unroll
  for (int e0 = 0; e0 < PT; e0 += CH) {
    T u[W], v[W], r0[W], r1[W];
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      u[2 * q] = c[0][e0 + q].x;
      u[2 * q + 1] = c[0][e0 + q].y;
      v[2 * q] = c[NF - 1][e0 + q].x;
      v[2 * q + 1] = c[NF - 1][e0 + q].y;
    }
    ntab_eval<T, NF, W>(tb, 0, u, v, r0);
    if constexpr (NF == 2) ntab_eval<T, NF, W>(tb, 1, u, v, r1);
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      c[0][e0 + q] = mk<T>(r0[2 * q], r0[2 * q + 1]);
      if constexpr (NF == 2) c[1][e0 + q] = mk<T>(r1[2 * q], r1[2 * q + 1]);
    }
  }
}

// threads per block of the x pass (launch bound)
template <typename T, int NX, int NF, bool SP = false>
struct XThreads {
  static constexpr int value = x_block_threads((int)sizeof(C<T>), NX, NF, SP);
};

// One x-pass tile: rows blk*R .. blk*R+R-1 of the spectral layout.  The
// block's threads form G = blockDim/S groups of S threads, G dividing R/2.
// PRELOADED: the caller has already staged the tile's spectral rows in LDS
// (the persistent kernel below does, from registers it filled earlier).
// tid: the thread's index in the block (a caller that loops over tiles
// passes a copy the compiler cannot see through, so that nothing derived
// from it is hoisted out of the loop).
// SP: the small grids' 4 points per thread (x_small).
template <typename T, int NX, int NF, int MODE, int NLM, bool PRELOADED = false, bool SP = false>
__device__ __forceinline__ void xpass_body(const XArgs& a, int64_t blk, C<T>* lds, int tid = threadIdx.x) {
  typedef XCfg<T, NX, NF, SP> K;
  constexpr int S = K::S, H = K::H, HB = K::HB, PT = K::P;
  constexpr int REG = K::reg_for(NF);

  const int R = a.rows_per_block;
  const int P = R >> 1;
  const int G = (int)blockDim.x / S;         // thread groups (lines in flight)
  const int g = tid / S, t = tid - g * S;
  const int64_t s0 = blk * R;
  const int64_t rows = a.rows;
  const Twiddles<T, NX, PT> tw = make_twiddles<T, NX, PT>(t);

  if constexpr (MODE != XMODE_FWD && !PRELOADED) {
    const C<T>* src[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) src[f] = (const C<T>*)a.spec_in[f];
    xstage_in<T, H, NF, NF, 0, REG, HB>(lds, src, s0, R, a.lb, tid, (int)blockDim.x);
    __syncthreads();
  }

  const int iters = P / G;
  for (int it = 0; it < iters; ++it) {
    const int pr = it * G + g;                 // row pair handled by this group
    C<T>* x[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) x[f] = lds + (pr * NF + f) * REG;
    C<T> c[NF][PT];
    const int64_t sa = s0 + 2 * pr;            // spectral row of the pair's first row

    if constexpr (MODE == XMODE_FWD) {
      const T* rin = (const T*)a.real_in;
      const int64_t za = sa % a.nz, ya = sa / a.nz;
      const int64_t zb = (sa + 1) % a.nz, yb = (sa + 1) / a.nz;
      const T* ra = rin + (za * a.ny + ya) * NX;
      const T* rb = rin + (zb * a.ny + yb) * NX;
#pragma unroll
      for (int e = 0; e < PT; ++e) c[0][e] = mk<T>(ra[t + e * S], rb[t + e * S]);
    } else {
      // Z[k] = X_a[k] + i X_b[k] over the full length from the half spectra
#pragma unroll
      for (int f = 0; f < NF; ++f) {
#pragma unroll
        for (int e = 0; e < PT; ++e) {
          const int k = t + e * S;
          C<T> z;
          if (k == 0) {
            C<T> ta = x[f][0], tb = x[f][HB];
            z = mk<T>(ta.x, tb.x);
          } else if (k == H) {
            C<T> ta = x[f][0], tb = x[f][HB];
            z = mk<T>(ta.y, tb.y);
          } else if (k < H) {
            C<T> ta = x[f][k], tb = x[f][HB + k];
            z = mk<T>(ta.x - tb.y, ta.y + tb.x);
          } else {
            C<T> ta = x[f][NX - k], tb = x[f][HB + NX - k];
            z = mk<T>(ta.x + tb.y, tb.x - ta.y);
          }
          c[f][e] = z;
        }
      }
      __syncthreads();
      fft_lines<T, NX, +1, NF, PT>(c, x, t, tw);
      if constexpr (MODE == XMODE_INV) {
        T* rout = (T*)a.real_out;
        const int64_t za = sa % a.nz, ya = sa / a.nz;
        const int64_t zb = (sa + 1) % a.nz, yb = (sa + 1) / a.nz;
        T* ra = rout + (za * a.ny + ya) * NX;
        T* rb = rout + (zb * a.ny + yb) * NX;
#pragma unroll
        for (int e = 0; e < PT; ++e) {
          ra[t + e * S] = c[0][e].x;
          rb[t + e * S] = c[0][e].y;
        }
        continue;
      } else {
        if constexpr (NLM == NLIN_TABLE) {
          nonlinear_table<T, NF, PT>(c, a.tab);
        } else {
          const T p0 = (T)a.p[0], p1 = (T)a.p[1], p2 = (T)a.p[2];
#pragma unroll
          for (int e = 0; e < PT; ++e) {
            if constexpr (NF == 1) nonlinear<T, NLM>(&c[0][e], &c[0][e], p0, p1, p2);
            else nonlinear<T, NLM>(&c[0][e], &c[NF - 1][e], p0, p1, p2);
          }
        }
      }
    }
    if constexpr (MODE != XMODE_INV) {
      fft_lines<T, NX, -1, NF, PT>(c, x, t, tw);
      // natural-order spectrum to LDS, then split the two rows
#pragma unroll
      for (int f = 0; f < NF; ++f) {
#pragma unroll
        for (int e = 0; e < PT; ++e) x[f][pidx<T>(t + e * S)] = c[f][e];
      }
      __syncthreads();
      const T sc = (T)a.scale;
      const T half = (T)0.5 * sc;
      C<T> fa[NF][PT / 2], fb[NF][PT / 2];
#pragma unroll
      for (int f = 0; f < NF; ++f) {
#pragma unroll
        for (int e = 0; e < PT / 2; ++e) {
          const int k = t + e * S;               // 0 .. H-1
          C<T> w = x[f][pidx<T>(k)];
          if (k == 0) {
            C<T> wn = x[f][pidx<T>(H)];
            fa[f][e] = mk<T>(w.x * sc, wn.x * sc);
            fb[f][e] = mk<T>(w.y * sc, wn.y * sc);
          } else {
            C<T> wm = x[f][pidx<T>(NX - k)];
            fa[f][e] = mk<T>((w.x + wm.x) * half, (w.y - wm.y) * half);
            fb[f][e] = mk<T>((w.y + wm.y) * half, (wm.x - w.x) * half);
          }
        }
      }
      __syncthreads();
#pragma unroll
      for (int f = 0; f < NF; ++f) {
#pragma unroll
        for (int e = 0; e < PT / 2; ++e) {
          const int k = t + e * S;
          x[f][k] = fa[f][e];
          x[f][HB + k] = fb[f][e];
        }
      }
    }
  }

  if constexpr (MODE != XMODE_INV) {
    __syncthreads();
    C<T>* dst[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) dst[f] = (C<T>*)a.spec_out[f];
    xstage_out<T, H, NF, NF, 0, REG, HB>(dst, lds, s0, R, a.lb, tid, (int)blockDim.x);
  }
}

template <typename T, int NX, int NF, int MODE, int NLM, bool SP = false>
__global__ void __launch_bounds__((XThreads<T, NX, NF, SP>::value)) xpass_kernel(XArgs a) {
  extern __shared__ __align__(16) unsigned char ss_dyn_lds[];
  xpass_body<T, NX, NF, MODE, NLM, false, SP>(a, xcd_block(blockIdx.x, gridDim.x, a.xcd_remap),
                                              reinterpret_cast<C<T>*>(ss_dyn_lds));
}

// Register prefetch of one x-pass tile for the persistent kernel: the
// element order and thread mapping of xstage_in (fast path, nthr >= R),
// exactly P elements per thread and field (PER = P * fields).
template <typename T, int H, int P, int PER>
__device__ __forceinline__ void xpass_prefetch(T (&pre_re)[PER], T (&pre_im)[PER], const C<T>* in0,
                                               const C<T>* in1, int tid, int nthr, int R, int lb,
                                               int64_t s0) {
  const int lr = __builtin_ctz((unsigned)R);
  const int64_t row = xstage_row<H>(s0 + (tid & (R - 1)), lb);
  const int kstep = nthr >> lr;
  const int k0 = tid >> lr;
  static_for<0, PER>([&](auto qc) __attribute__((always_inline)) {
    constexpr int q = decltype(qc)::value;
    const C<T>* src = (q < P ? in0 : in1) + row;
    const C<T> v = src[(int64_t)(k0 + (q % P) * kstep) << lb];
    pre_re[q] = v.x;
    pre_im[q] = v.y;
  });
}

// Persistent x pass (STEP): block b takes tiles b, b + gridDim, ... and
// loads the next tile's spectral rows into registers while it transforms
// the current one, so the loads of one tile overlap the transforms of the
// previous.  Requires blockDim = (R/2)*S (every pair in flight at once):
// then each thread stages exactly P elements per field.
template <typename T, int NX, int NF, int NLM>
__global__ void __launch_bounds__(512) xpass_pp_kernel(XArgs a, int ntiles) {
  typedef XCfg<T, NX, NF> K;
  constexpr int HB = K::HB, P = K::P;
  constexpr int REG = K::reg_for(NF);
  constexpr int PER = P * NF;
  extern __shared__ __align__(16) unsigned char ss_dyn_lds[];
  C<T>* lds = reinterpret_cast<C<T>*>(ss_dyn_lds);
  const int R = a.rows_per_block;
  const int tid = threadIdx.x;
  const int nthr = (int)blockDim.x;
  const int lr = __builtin_ctz((unsigned)R);
  const int r = tid & (R - 1);
  C<T>* lrow = lds + (r >> 1) * NF * REG + (r & 1) * HB;
  const int kstep = nthr >> lr;
  const int k0 = tid >> lr;
  T pre_re[PER], pre_im[PER];   // scalar arrays: kept in registers
  int tile = blockIdx.x;
  const C<T>* in0 = (const C<T>*)a.spec_in[0];
  const C<T>* in1 = (const C<T>*)a.spec_in[1];
  const int remap = a.xcd_remap;
  if (tile < ntiles)
    xpass_prefetch<T, K::H, P, PER>(pre_re, pre_im, in0, in1, tid, nthr, R, a.lb,
                                    xcd_block(tile, ntiles, remap) * R);
  for (; tile < ntiles; tile += gridDim.x) {
    __syncthreads();
    static_for<0, PER>([&](auto qc) __attribute__((always_inline)) {
      constexpr int q = decltype(qc)::value;
      lrow[(q / P) * REG + k0 + (q % P) * kstep] = mk<T>(pre_re[q], pre_im[q]);
    });
    __syncthreads();
    const int next = tile + gridDim.x;
    if (next < ntiles)
      xpass_prefetch<T, K::H, P, PER>(pre_re, pre_im, in0, in1, tid, nthr, R, a.lb,
                                      xcd_block(next, ntiles, remap) * R);
    xpass_body<T, NX, NF, XMODE_STEP, NLM, true>(a, xcd_block(tile, ntiles, a.xcd_remap), lds);
  }
}

// ---------------------------------------------------------------------------
// y pass (3D): complex FFT along y of T[kx][y][z] on chunks of R
// consecutive z; block = (kx, z chunk).  In place is allowed.
// ---------------------------------------------------------------------------
struct YArgs {
  const void* in;
  void* out;
  int ny, nz;
  int hx;                  // Nx/2 (kx count of the spectral layout)
  int lb;                  // log2 of the row block of the spectral layout
  int lines_per_block;     // R (divides nz)
  double scale;
};

template <typename T, int NY>
struct YCfg {
  static constexpr int S = NY / 8;
  static constexpr int ESZ = (int)sizeof(C<T>);
  static constexpr int REG = y_reg(ESZ, NY);
};

template <typename T, int NY, int DIR>
__global__ void __launch_bounds__(1024) ypass_kernel(YArgs a) {
  typedef YCfg<T, NY> K;
  constexpr int S = K::S, REG = K::REG;
  extern __shared__ __align__(16) unsigned char ss_dyn_lds[];
  C<T>* lds = reinterpret_cast<C<T>*>(ss_dyn_lds);
  const int R = a.lines_per_block;
  const int G = (int)blockDim.x / S;
  const int tid = threadIdx.x;
  const int g = tid / S, t = tid - g * S;
  const int64_t chunks_per_kx = a.nz / R;
  const int64_t kx = blockIdx.x / chunks_per_kx;
  const int64_t z0 = (blockIdx.x - kx * chunks_per_kx) * R;

  const C<T>* src = (const C<T>*)a.in;
  C<T>* dst = (C<T>*)a.out;
  const Twiddles<T, NY> tw = make_twiddles<T, NY>(t);

  // staged copies: element (y, r) with r fastest; thread tid keeps line
  // r = tid mod R (nthr = G*S is a multiple of R) and y advances by nthr/R.
  // The row block B divides nz, so sidx(kx, y*nz + z) = y*nz*hx + sidx(kx, z).
  const int nthr = (int)blockDim.x;
  const int lr = __builtin_ctz((unsigned)R);
  const int r = tid & (R - 1);
  const int64_t ystride = (int64_t)a.nz * a.hx;
  const int64_t zoff = sidx(kx, z0 + r, a.hx, a.lb);
  const int ystep = nthr >> lr;
  const int per = (NY * R) / nthr;          // a multiple of 8
  C<T>* lline = lds + r * REG;
  for (int c = 0, y0 = tid >> lr; c < per; c += 8, y0 += 8 * ystep) {
    T vr[8], vi[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const C<T> v = src[zoff + (int64_t)(y0 + q * ystep) * ystride];
      vr[q] = v.x;
      vi[q] = v.y;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) lline[y0 + q * ystep] = mk<T>(vr[q], vi[q]);
  }
  __syncthreads();
  const T sc = (T)a.scale;
  const int iters = R / G;
  for (int it = 0; it < iters; ++it) {
    const int ln = it * G + g;
    C<T>* x[1] = {lds + ln * REG};
    C<T> c[1][8];
#pragma unroll
    for (int e = 0; e < 8; ++e) c[0][e] = x[0][t + e * S];
    __syncthreads();
    fft_lines<T, NY, DIR, 1>(c, x, t, tw);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 8; ++e) x[0][t + e * S] = cscale<T>(c[0][e], sc);
  }
  __syncthreads();
  for (int c = 0, y0 = tid >> lr; c < per; c += 8, y0 += 8 * ystep) {
    T vr[8], vi[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const C<T> v = lline[y0 + q * ystep];
      vr[q] = v.x;
      vi[q] = v.y;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) dst[zoff + (int64_t)(y0 + q * ystep) * ystride] = mk<T>(vr[q], vi[q]);
  }
}

// ---------------------------------------------------------------------------
// k-space pass: lines along the last axis (length NL), ETD1 update.
// ---------------------------------------------------------------------------
struct KField {
  void* state;              // T (read; written too unless `out` is set)
  const void* nonlin;       // G
  const void* nonlin2;      // a second explicit channel's G (stepping form; null: none)
  void* out;                // where the new T goes (null: in place)
  void* shat;               // stepping form: the state's full spectrum S^, read and rewritten
  double l[4];              // L(k^2) = l0 + l1 k^2 + l2 k^4 + l3 k^6
  double n[4];              // N(k^2) = n0 + n1 k^2 + n2 k^4 + n3 k^6 (the channel's derivative)
  double n2[4];             // the second channel's N(k^2)
};

struct KArgs {
  KField fld[2];
  int nlines;               // Nx/2 * J  (J = Ny in 3D, 1 in 2D)
  int J;                    // lines per kx plane
  int lines_per_block;
  int nx;                   // grid size along x (for the Nyquist plane)
  double sx, sy, sz;        // 2 pi / (N_axis dx_axis)
  double dt;
  double a_scale, b_scale;  // 1/N_last and 1/N
  double* mass_log;         // may be null
  int64_t log_index;        // row of mass_log for this step (per field stride nf)
  int64_t log_capacity;
  int nf;
  int three_d;
  int lb;                   // log2 of the row block of the spectral layout
  int scheme;               // 0: ETD1 factors; 1: linearly implicit (selects the kernel)
};

// A = exp(z) and phi1(z) = (e^z - 1)/z of one mode (Eq. 4; phi1(0) = 1).
// FP64: one expm1 serves both.  FP32: the library exponential for A;
// phi1 from its Taylor series where |z| < 1/2 (degree 7: truncation below
// 2e-8 relative) and from A and the hardware reciprocal elsewhere, where
// e^z - 1 has no cancellation; both are evaluated and one is selected, so
// z = 0 needs no special case.  The forward step and its adjoint share
// this; em is e^z - 1 as the adjoint uses it.
template <typename T>
__device__ __forceinline__ void etd1_aphi(T z, T& A, T& phi, T& em) {
  if constexpr (sizeof(T) == 8) {
    em = expm1(z);
    A = 1.0 + em;
    phi = (z != 0.0) ? em / z : 1.0;
  } else {
    A = SS_FAST_EXPF ? __expf(z) : expf(z);
    float ps = 1.0f / 40320.0f;
    ps = fmaf(ps, z, 1.0f / 5040.0f);
    ps = fmaf(ps, z, 1.0f / 720.0f);
    ps = fmaf(ps, z, 1.0f / 120.0f);
    ps = fmaf(ps, z, 1.0f / 24.0f);
    ps = fmaf(ps, z, 1.0f / 6.0f);
    ps = fmaf(ps, z, 0.5f);
    ps = fmaf(ps, z, 1.0f);
    const float pl = (A - 1.0f) * __builtin_amdgcn_rcpf(z);
    phi = __builtin_fabsf(z) < 0.5f ? ps : pl;
    em = A - 1.0f;
  }
}

// Step factors of one mode, with the k-space pass scalings folded in.
// scheme 0, ETD1 (Eq. 4): A = exp(L dt), B = dt phi1(L dt) N.
// scheme 1, linearly implicit (the first-order semi-implicit scheme):
// A = 1/(1 - L dt), B = dt A N (the host has checked 1 - L dt > 0).
// The scheme is a compile-time choice: a run-time branch here costs the
// FP64 k-space kernels registers they do not have.
template <typename T>
__device__ __forceinline__ T kpoly3(const double (&c)[4], T k2) {
  return (T)c[0] + k2 * ((T)c[1] + k2 * ((T)c[2] + k2 * (T)c[3]));
}

template <typename T, int SCH = 0>
__device__ __forceinline__ void etd1_coeffs(const KField& f, T k2, double dt, double as, double bs,
                                            T& ao, T& bo) {
  const T L = kpoly3<T>(f.l, k2);
  const T z = L * (T)dt;
  T A, phi, em;
  if constexpr (SCH == 1) {
    A = (T)1 / ((T)1 - z);
    phi = A;
  } else {
    etd1_aphi<T>(z, A, phi, em);
  }
  ao = A * (T)as;
  bo = (T)dt * phi * kpoly3<T>(f.n, k2) * (T)bs;
}

// The same with two explicit channels: B N_1 and B N_2 (Eq. 8, a sum over
// the channels i of B_i = B d_i).
template <typename T, int SCH = 0>
__device__ __forceinline__ void etd1_coeffs2(const KField& f, T k2, double dt, double as, double bs,
                                             T& ao, T& bo, T& bo2) {
  const T L = kpoly3<T>(f.l, k2);
  const T z = L * (T)dt;
  T A, phi, em;
  if constexpr (SCH == 1) {
    A = (T)1 / ((T)1 - z);
    phi = A;
  } else {
    etd1_aphi<T>(z, A, phi, em);
  }
  ao = A * (T)as;
  const T b = (T)dt * phi * (T)bs;
  bo = b * kpoly3<T>(f.n, k2);
  bo2 = b * kpoly3<T>(f.n2, k2);
}

// Offset of element u (0 <= u < N_last) of a k-space line from the line's
// first element: g(u) = ((u >> lb) * hx << lb) + (u mod B).  For t < S and
// S, B powers of two (B at most the line length, the line start a multiple
// of B): g(t + e S) = g(t) + g(e S), a per-thread part plus a part that is
// the same for every thread of the line.
__device__ __forceinline__ int64_t kline_off(int64_t u, int64_t hx, int lb) {
  return (((u >> lb) * hx) << lb) + (u & ((int64_t(1) << lb) - 1));
}

// Uniform 64-bit value across the wave (the line of a k-space thread is the
// same for all 64 lanes when the line has at least 64 threads).
__device__ __forceinline__ int64_t wave_uniform(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// base + uo (elements, wave uniform) + tb (bytes, per thread, < 4 GiB)
template <typename P>
__device__ __forceinline__ P* kline_at(P* base, int64_t uo, uint32_t tb) {
  typedef typename std::conditional<std::is_const<P>::value, const char, char>::type B;
  return reinterpret_cast<P*>(reinterpret_cast<B*>(base + uo) + tb);
}

// Twiddle bases of a k-space thread: from registers (FP32) or from its LDS
// entries (FP64).
template <typename T, int NL, int P = 8>
__device__ __forceinline__ Twiddles<T, NL, P> ktw(const Twiddles<T, NL, P>& tw, const C<T>* twl, int stride) {
  if constexpr (sizeof(T) == 8) {
    Twiddles<T, NL, P> r;
#pragma unroll
    for (int i = 0; i < Twiddles<T, NL, P>::NW; ++i) r.w[i] = twl[i * stride];
    return r;
  } else {
    return tw;
  }
}

// Line slot -> (kx index, mid-axis index).  Slots 0 .. J-1 are the packed
// kx = 0 plane; in 3D they are ordered so that each line sits next to its
// mirror (-k_mid): pairs (0, J/2), then (j, J - j).
__device__ __forceinline__ void kline_slot(int slot, int J, int three_d, int& kxi, int& kyi) {
  if (slot < J) {
    kxi = 0;
    if (!three_d) {
      kyi = 0;
    } else {
      const int pi = slot >> 1, mem = slot & 1;
      kyi = (pi == 0) ? (mem ? J / 2 : 0) : (mem ? J - pi : pi);
    }
  } else {
    kxi = slot / J;
    kyi = slot - kxi * J;
  }
}

template <typename T, int NL, int P = 8>
struct KCfg {
  static constexpr int S = NL / P;
  static constexpr int ESZ = (int)sizeof(C<T>);
  static constexpr int REG = k_reg(ESZ, NL);
};

// One k-space tile: lines bx*L .. bx*L+L-1 of field `fi`.
// HAT = false: the state's spectrum is formed here (forward FFT of T, three
// transforms per line).  HAT = true (stepping form): the full spectrum S^ of
// the state is carried between steps (S^ = FFT(T)/N_last), so only the
// nonlinear term is transformed; U = A S^ + B N G^ is written back as the
// new S^ and, inverse transformed, as the new T (two transforms per line;
// the host passes a_scale = 1).
// CH2 (stepping form only): the field has a second explicit channel whose
// term G2 (F.nonlin2) is transformed too: U = A S^ + B (N_1 G^ + N_2 G2^).
template <typename T, int NL, bool HAT = false, int SCH = 0, int P = 8, bool CH2 = false>
__device__ __forceinline__ void kpass_body(const KArgs& a, int bx, int fi, C<T>* lds, int tid = threadIdx.x) {
  static_assert(!CH2 || HAT, "a second channel needs the stepping form");
  typedef KCfg<T, NL, P> K;
  constexpr int S = K::S, REG = K::REG;
  const int ls = tid / S, t = tid - ls * S;
  const KField F = fi == 0 ? a.fld[0] : a.fld[1];
  const int line0 = bx * a.lines_per_block;
  const int slot = line0 + ls;               // global line slot
  const bool packed_block = line0 < a.J;     // block holds kx = 0 lines
  int kxi, kyi;
  kline_slot(slot, a.J, a.three_d, kxi, kyi);
  // element p of this line is row s = kyi*NL + p of plane kxi; the line
  // start is a multiple of NL, and the row block B is at most NL
  const int64_t hx = a.nx / 2;
  const int lb = a.lb;
  int64_t lbase = sidx(kxi, (int64_t)kyi * NL, hx, lb);
  if constexpr (S >= 64) lbase = wave_uniform(lbase);
  const uint32_t tb = (uint32_t)(kline_off(t, hx, lb) * (int64_t)sizeof(C<T>));
  const C<T>* st = (const C<T>*)(HAT ? F.shat : F.state) + lbase;
  const C<T>* gn = (const C<T>*)F.nonlin + lbase;
  C<T>* so = (C<T>*)(F.out ? F.out : F.state) + lbase;

  C<T> ct[1][P], cg[1][P], cg2[1][CH2 ? P : 1];
  // the three-transform form transforms the state first; the stepping
  // form reads S^ only for the update, after the nonlinear term's
  // transform (fewer live registers during it)
  if constexpr (!HAT) {
#pragma unroll
    for (int e = 0; e < P; ++e) ct[0][e] = *kline_at(st, kline_off(e * S, hx, lb), tb);
  }
  // one LDS region per line serves all three transforms in turn
  C<T>* x[1] = {lds + ls * REG};
  // FP64 parks the twiddle bases in LDS between the transforms (entry i of
  // thread j at i * L*S + j): the registers they free let three waves share
  // a SIMD.  Each thread reads back only what it wrote.
  C<T>* const twl = lds + a.lines_per_block * REG + ls * S + t;
  const int twstride = a.lines_per_block * S;
  static_assert(Twiddles<T, NL, P>::NW == k_nw(NL, P), "LDS twiddle table size");
  static_assert(sizeof(T) != 8 || (NL / P) * k_nw(NL, P) <= k_twl(16, NL), "LDS twiddle table size");
  const Twiddles<T, NL, P> tw = make_twiddles<T, NL, P>(t);
  if constexpr (sizeof(T) == 8) {
#pragma unroll
    for (int i = 0; i < Twiddles<T, NL, P>::NW; ++i) twl[i * twstride] = tw.w[i];
  }
  if constexpr (!HAT) fft_lines<T, NL, -1, 1, P>(ct, x, t, ktw<T, NL, P>(tw, twl, twstride));
  if constexpr (CH2) {
    const C<T>* gn2 = (const C<T>*)F.nonlin2 + lbase;
#pragma unroll
    for (int e = 0; e < P; ++e) cg2[0][e] = *kline_at(gn2, kline_off(e * S, hx, lb), tb);
    fft_lines<T, NL, -1, 1, P>(cg2, x, t, ktw<T, NL, P>(tw, twl, twstride));
  }
#pragma unroll
  for (int e = 0; e < P; ++e) cg[0][e] = *kline_at(gn, kline_off(e * S, hx, lb), tb);
  fft_lines<T, NL, -1, 1, P>(cg, x, t, ktw<T, NL, P>(tw, twl, twstride));
  if constexpr (HAT) {
#pragma unroll
    for (int e = 0; e < P; ++e) ct[0][e] = *kline_at(st, kline_off(e * S, hx, lb), tb);
  }

  // wavenumbers: k_last from the position, k_mid from kyi (3D), k_x from kxi
  const T kxv = (T)kxi * (T)a.sx;
  T kmid2 = (T)0;
  if (a.three_d) {
    const int m = kyi <= a.J / 2 ? kyi : kyi - a.J;
    kmid2 = ((T)m * (T)a.sy) * ((T)m * (T)a.sy);
  }
  const T klast_s = (T)(a.three_d ? a.sz : a.sy);

  if (packed_block) {
    // The kx = 0 lines hold S(0) + i S(Nx/2).  With the mirror mode m(-k):
    //   U = (a0+an)/2 C + (a0-an)/2 conj(C(-k)) + (b0+bn)/2 D + (b0-bn)/2 conj(D(-k))
    // (C, D: transformed state and nonlinear term).  The two halves are
    // formed one after the other through the single LDS region.
    const bool packed = slot < a.J;
    int mls = ls;
    if (a.three_d && (slot >> 1) != 0) mls = ls ^ 1;
    const C<T>* xm = lds + mls * REG;
    const T kny = (T)(a.nx / 2) * (T)a.sx;
#pragma unroll
    for (int e = 0; e < P; ++e) x[0][pidx<T>(t + e * S)] = ct[0][e];
    __syncthreads();
    if (packed) {
#pragma unroll
      for (int e = 0; e < P; ++e) {
        __builtin_amdgcn_sched_barrier(0);
        const int p = t + e * S;
        const int m = p <= NL / 2 ? p : p - NL;
        const T kl = (T)m * klast_s;
        const T k2_0 = kmid2 + kl * kl;
        T a0, b0, an, bn;
        etd1_coeffs<T, SCH>(F, k2_0, a.dt, a.a_scale, a.b_scale, a0, b0);
        etd1_coeffs<T, SCH>(F, k2_0 + kny * kny, a.dt, a.a_scale, a.b_scale, an, bn);
        const C<T> cm = cconj<T>(xm[pidx<T>((NL - p) & (NL - 1))]);
        const T ap = (T)0.5 * (a0 + an), am = (T)0.5 * (a0 - an);
        ct[0][e] = mk<T>(ap * ct[0][e].x + am * cm.x, ap * ct[0][e].y + am * cm.y);
      }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < P; ++e) x[0][pidx<T>(t + e * S)] = cg[0][e];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < P; ++e) {
      __builtin_amdgcn_sched_barrier(0);
      const int p = t + e * S;
      const int m = p <= NL / 2 ? p : p - NL;
      const T kl = (T)m * klast_s;
      if (packed) {
        const T k2_0 = kmid2 + kl * kl;
        T a0, b0, an, bn;
        etd1_coeffs<T, SCH>(F, k2_0, a.dt, a.a_scale, a.b_scale, a0, b0);
        etd1_coeffs<T, SCH>(F, k2_0 + kny * kny, a.dt, a.a_scale, a.b_scale, an, bn);
        const C<T> dm = cconj<T>(xm[pidx<T>((NL - p) & (NL - 1))]);
        const T bp = (T)0.5 * (b0 + bn), bmn = (T)0.5 * (b0 - bn);
        ct[0][e] = mk<T>(ct[0][e].x + bp * cg[0][e].x + bmn * dm.x,
                         ct[0][e].y + bp * cg[0][e].y + bmn * dm.y);
      } else if constexpr (CH2) {
        const T k2 = kxv * kxv + kmid2 + kl * kl;
        T av, bv, bv2;
        etd1_coeffs2<T, SCH>(F, k2, a.dt, a.a_scale, a.b_scale, av, bv, bv2);
        ct[0][e] = mk<T>(av * ct[0][e].x + bv * cg[0][e].x + bv2 * cg2[0][e].x,
                         av * ct[0][e].y + bv * cg[0][e].y + bv2 * cg2[0][e].y);
      } else {
        const T k2 = kxv * kxv + kmid2 + kl * kl;
        T av, bv;
        etd1_coeffs<T, SCH>(F, k2, a.dt, a.a_scale, a.b_scale, av, bv);
        ct[0][e] = mk<T>(av * ct[0][e].x + bv * cg[0][e].x, av * ct[0][e].y + bv * cg[0][e].y);
      }
    }
    if constexpr (CH2) {
      // the second channel's two packed halves, through the same region
      __syncthreads();
#pragma unroll
      for (int e = 0; e < P; ++e) x[0][pidx<T>(t + e * S)] = cg2[0][e];
      __syncthreads();
      if (packed) {
#pragma unroll
        for (int e = 0; e < P; ++e) {
          __builtin_amdgcn_sched_barrier(0);
          const int p = t + e * S;
          const int m = p <= NL / 2 ? p : p - NL;
          const T kl = (T)m * klast_s;
          const T k2_0 = kmid2 + kl * kl;
          T a0, b0, b20, an, bn, b2n;
          etd1_coeffs2<T, SCH>(F, k2_0, a.dt, a.a_scale, a.b_scale, a0, b0, b20);
          etd1_coeffs2<T, SCH>(F, k2_0 + kny * kny, a.dt, a.a_scale, a.b_scale, an, bn, b2n);
          const C<T> dm = cconj<T>(xm[pidx<T>((NL - p) & (NL - 1))]);
          const T bp = (T)0.5 * (b20 + b2n), bmn = (T)0.5 * (b20 - b2n);
          ct[0][e] = mk<T>(ct[0][e].x + bp * cg2[0][e].x + bmn * dm.x,
                           ct[0][e].y + bp * cg2[0][e].y + bmn * dm.y);
        }
      }
    }
    if (packed && a.mass_log && kyi == 0 && t == 0 && a.log_index < a.log_capacity)
      a.mass_log[a.log_index * a.nf + fi] = (double)ct[0][0].x;
    __syncthreads();
  } else {
#pragma unroll
    for (int e = 0; e < P; ++e) {
      __builtin_amdgcn_sched_barrier(0);
      const int p = t + e * S;
      const int m = p <= NL / 2 ? p : p - NL;
      const T kl = (T)m * klast_s;
      const T k2 = kxv * kxv + kmid2 + kl * kl;
      if constexpr (CH2) {
        T av, bv, bv2;
        etd1_coeffs2<T, SCH>(F, k2, a.dt, a.a_scale, a.b_scale, av, bv, bv2);
        ct[0][e] = mk<T>(av * ct[0][e].x + bv * cg[0][e].x + bv2 * cg2[0][e].x,
                         av * ct[0][e].y + bv * cg[0][e].y + bv2 * cg2[0][e].y);
      } else {
        T av, bv;
        etd1_coeffs<T, SCH>(F, k2, a.dt, a.a_scale, a.b_scale, av, bv);
        ct[0][e] = mk<T>(av * ct[0][e].x + bv * cg[0][e].x, av * ct[0][e].y + bv * cg[0][e].y);
      }
    }
  }

  if constexpr (HAT) {
    C<T>* sh = (C<T>*)F.shat + lbase;
#pragma unroll
    for (int e = 0; e < P; ++e) *kline_at(sh, kline_off(e * S, hx, lb), tb) = ct[0][e];
  }
  fft_lines<T, NL, +1, 1, P>(ct, x, t, ktw<T, NL, P>(tw, twl, twstride));
#pragma unroll
  for (int e = 0; e < P; ++e) *kline_at(so, kline_off(e * S, hx, lb), tb) = ct[0][e];
}

// FP64: three waves per SIMD (168 VGPRs), except 128- and 256-point lines,
// whose 3D plane pairing needs ~176 VGPRs (spills under the cap of three).
// Two explicit channels (CH2) hold a third line of registers: FP64 takes
// two waves per SIMD there.
template <typename T, int NL, bool HAT, int SCH = 0, bool CH2 = false>
__global__ void __launch_bounds__(512)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? ((NL == 128 || NL == 256 || CH2) ? 2 : 3) : SS_KWAVES)))
kpass_kernel(KArgs a) {
  extern __shared__ __align__(16) unsigned char ss_dyn_lds[];
  kpass_body<T, NL, HAT, SCH, HAT ? k_pts((int)sizeof(C<T>), NL) : 8, CH2>(a, blockIdx.x, blockIdx.y,
                                                                           reinterpret_cast<C<T>*>(ss_dyn_lds));
}

// S^ = FFT(T) / N_last along every line of field blockIdx.y (the stepping
// form's spectrum, refreshed after the fields change outside a step).
template <typename T, int NL>
__global__ void __launch_bounds__(512) kfwd_kernel(KArgs a) {
  typedef KCfg<T, NL> K;
  constexpr int S = K::S, REG = K::REG;
  extern __shared__ __align__(16) unsigned char ss_dyn_lds[];
  C<T>* lds = reinterpret_cast<C<T>*>(ss_dyn_lds);
  const int tid = threadIdx.x;
  const int ls = tid / S, t = tid - ls * S;
  const KField& F = blockIdx.y == 0 ? a.fld[0] : a.fld[1];
  int kxi, kyi;
  kline_slot(blockIdx.x * a.lines_per_block + ls, a.J, a.three_d, kxi, kyi);
  const int64_t hx = a.nx / 2;
  const int lb = a.lb;
  const int64_t lbase = sidx(kxi, (int64_t)kyi * NL, hx, lb);
  const uint32_t tb = (uint32_t)(kline_off(t, hx, lb) * (int64_t)sizeof(C<T>));
  const C<T>* st = (const C<T>*)F.state + lbase;
  C<T>* sh = (C<T>*)F.shat + lbase;
  C<T> c[1][8];
#pragma unroll
  for (int e = 0; e < 8; ++e) c[0][e] = *kline_at(st, kline_off(e * S, hx, lb), tb);
  C<T>* x[1] = {lds + ls * REG};
  fft_lines<T, NL, -1, 1>(c, x, t, make_twiddles<T, NL>(t));
  const T sc = (T)1 / (T)NL;
#pragma unroll
  for (int e = 0; e < 8; ++e) *kline_at(sh, kline_off(e * S, hx, lb), tb) = cscale<T>(c[0][e], sc);
}

// ---------------------------------------------------------------------------
// Structure factor (Sec. 3): radial average of S(k) = |rho_hat_k|^2 / N for
// the occupancy rho = [psi > 0].  The x pass (NLIN_THRESH) has already
// formed the x-spectrum of rho (3D: also transformed along y) in the layout
// of the state; this pass transforms each line along the last axis and
// bins every mode by b = round(|m|), m the integer mode vector (the box has
// the same length along every axis, so |k| = 2 pi |m| / L).  Each block
// accumulates a histogram in LDS over its lines (several, persistently) and
// writes it to its own row of a partials array; sf_reduce adds the rows in
// block order.  The histogram's sums are kept in fixed point (sf_add), so
// that no part of the result depends on the order of the atomic adds.
// ---------------------------------------------------------------------------
struct SFArgs {
  const void* spec;        // transformed occupancy, layout of the state
  double* part_sum;        // [gridDim.x][pstride] per-block sums of |rho_hat|^2 / N
  uint32_t* part_cnt;      // [gridDim.x][pstride] per-block mode counts
  double* s_out;           // [nbins] radial average (sf_reduce)
  int64_t* n_out;          // [nbins] modes per bin (sf_reduce)
  int nbins;
  int pstride;             // row stride of the partials: nbins rounded up to 32 (whole lines)
  int nblocks;             // rows of the partials
  int nlines, J, lines_per_block, nx, three_d, lb;
  double inv_n;            // 1/N
};

constexpr int64_t sf_lds(int esz, int nl, int lines, int nbins) {
  return (int64_t)lines * k_reg(esz, nl) * esz + (int64_t)nbins * (24 + 4);
}

// Per-bin sums in fixed point.  A contribution v = |rho_hat|^2 / N (twice
// that for a +-kx pair) lies in [0, 2^35): |rho_hat| <= N <= 2^34.  It is
// added as floor(v 2^85) in three 40-bit chunks, each to its own 64-bit LDS
// counter with an integer atomic; integer sums do not depend on the order
// of the adds, and up to 2^24 adds per bin and block leave every counter
// below 2^64.  The truncation costs at most 2^-85 per contribution.
__device__ __forceinline__ void sf_add(unsigned long long* h, int b, double v) {
  const double x = v * 0x1p85;                 // exact scaling, below 2^120
  const double hi = floor(x * 0x1p-80);
  const double r = x - hi * 0x1p80;            // exact
  const double mid = floor(r * 0x1p-40);
  const double lo = floor(r - mid * 0x1p40);
  atomicAdd(&h[3 * b], (unsigned long long)hi);
  atomicAdd(&h[3 * b + 1], (unsigned long long)mid);
  atomicAdd(&h[3 * b + 2], (unsigned long long)lo);
}
__device__ __forceinline__ double sf_value(const unsigned long long* h, int b) {
  return (double)h[3 * b] * 0x1p-5 + (double)h[3 * b + 1] * 0x1p-45 + (double)h[3 * b + 2] * 0x1p-85;
}

// b = round(sqrt(m2)) for an integer m2 >= 0: the b with b^2 - b < m2 <= b^2 + b
__device__ __forceinline__ int sf_bin(int64_t m2) {
  int64_t b = (int64_t)sqrt((double)m2);
  while (b * b + b < m2) ++b;
  while (b > 0 && b * b - b >= m2) --b;
  return (int)b;
}

template <typename T, int NL>
__device__ __forceinline__ void sf_tile(const SFArgs& a, int tile, C<T>* lds, unsigned long long* hs, uint32_t* hc) {
  typedef KCfg<T, NL> K;
  constexpr int S = K::S, REG = K::REG;
  const int tid = threadIdx.x;
  const int ls = tid / S, t = tid - ls * S;
  const int line0 = tile * a.lines_per_block;
  const int slot = line0 + ls;
  const bool packed_block = line0 < a.J;
  int kxi, kyi;
  kline_slot(slot, a.J, a.three_d, kxi, kyi);
  const int64_t hx = a.nx / 2;
  const int lb = a.lb;
  const int64_t lbase = sidx(kxi, (int64_t)kyi * NL, hx, lb);
  const C<T>* src = (const C<T>*)a.spec + lbase;
  const uint32_t tb = (uint32_t)(kline_off(t, hx, lb) * (int64_t)sizeof(C<T>));
  C<T> c[1][8];
#pragma unroll
  for (int e = 0; e < 8; ++e) c[0][e] = *kline_at(src, kline_off(e * S, hx, lb), tb);
  C<T>* x[1] = {lds + ls * REG};
  fft_lines<T, NL, -1, 1>(c, x, t, make_twiddles<T, NL>(t));
  // integer mode components other than x
  int64_t mmid2 = 0;
  if (a.three_d) {
    const int64_t m = kyi <= a.J / 2 ? kyi : kyi - a.J;
    mmid2 = m * m;
  }
  const double w = a.inv_n;
  bool done = false;
  if (packed_block) {
    // the kx = 0 plane holds C = rho_hat(0, .) + i rho_hat(Nx/2, .); with the
    // mirror mode C(-k): rho_hat(0, k) = (C + conj C(-k))/2,
    // rho_hat(Nx/2, k) = (C - conj C(-k))/(2i).  Lines of the block that
    // are not in that plane fall through to the general case below.
    const bool packed = slot < a.J;
    int mls = ls;
    if (a.three_d && (slot >> 1) != 0) mls = ls ^ 1;
    const C<T>* xm = lds + mls * REG;
#pragma unroll
    for (int e = 0; e < 8; ++e) x[0][pidx<T>(t + e * S)] = c[0][e];
    __syncthreads();
    if (packed) {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int p = t + e * S;
        const int64_t ml = p <= NL / 2 ? p : p - NL;
        const C<T> cm = xm[pidx<T>((NL - p) & (NL - 1))];
        const double ar = 0.5 * ((double)c[0][e].x + (double)cm.x), ai = 0.5 * ((double)c[0][e].y - (double)cm.y);
        const double br = 0.5 * ((double)c[0][e].y + (double)cm.y), bi = 0.5 * ((double)cm.x - (double)c[0][e].x);
        const int b0 = sf_bin(mmid2 + ml * ml);
        const int bn = sf_bin(hx * hx + mmid2 + ml * ml);
        sf_add(hs, b0, (ar * ar + ai * ai) * w);
        atomicAdd(&hc[b0], 1u);
        sf_add(hs, bn, (br * br + bi * bi) * w);
        atomicAdd(&hc[bn], 1u);
      }
      done = true;
    }
  }
  if (!done) {
    // kx and -kx have the same |rho_hat| and |m|: weight 2
    const int64_t mx2 = (int64_t)kxi * kxi;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int p = t + e * S;
      const int64_t ml = p <= NL / 2 ? p : p - NL;
      const double re = (double)c[0][e].x, im = (double)c[0][e].y;
      const int b = sf_bin(mx2 + mmid2 + ml * ml);
      sf_add(hs, b, 2.0 * (re * re + im * im) * w);
      atomicAdd(&hc[b], 2u);
    }
  }
  __syncthreads();
}

template <typename T, int NL>
__global__ void __launch_bounds__(512) sfpass_kernel(SFArgs a) {
  typedef KCfg<T, NL> K;
  extern __shared__ __align__(16) unsigned char ss_dyn_lds[];
  C<T>* lds = reinterpret_cast<C<T>*>(ss_dyn_lds);
  unsigned long long* hs = reinterpret_cast<unsigned long long*>(lds + a.lines_per_block * K::REG);
  uint32_t* hc = reinterpret_cast<uint32_t*>(hs + 3 * a.nbins);
  for (int i = threadIdx.x; i < a.nbins; i += blockDim.x) {
    hs[3 * i] = 0ull;
    hs[3 * i + 1] = 0ull;
    hs[3 * i + 2] = 0ull;
    hc[i] = 0u;
  }
  __syncthreads();
  const int ntiles = a.nlines / a.lines_per_block;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) sf_tile<T, NL>(a, tile, lds, hs, hc);
  __syncthreads();
  double* ps = a.part_sum + (int64_t)blockIdx.x * a.pstride;
  uint32_t* pc = a.part_cnt + (int64_t)blockIdx.x * a.pstride;
  for (int i = threadIdx.x; i < a.nbins; i += blockDim.x) {
    ps[i] = sf_value(hs, i);
    pc[i] = hc[i];
  }
}

// Reduction of the partials: a block takes 32 bins (a row segment of 256
// bytes of sums and 128 of counts: whole cache lines, the rows being
// padded to a multiple of 32 bins, which the block reads alone); thread (slice j, bin i) adds rows j, j + 32, j + 64, ... of
// bin i in order, then the 32 slice sums of each bin are added in slice
// order (the same order every call).
template <typename T>
__global__ void __launch_bounds__(1024) sf_reduce_kernel(SFArgs a) {
  __shared__ double ps[32][32];
  __shared__ int64_t pn[32][32];
  const int i = threadIdx.x & 31, j = threadIdx.x >> 5;
  const int b = blockIdx.x * 32 + i;
  double s = 0.0;
  int64_t n = 0;
  if (b < a.nbins) {
    for (int k = j; k < a.nblocks; k += 32) {
      s += a.part_sum[(int64_t)k * a.pstride + b];
      n += a.part_cnt[(int64_t)k * a.pstride + b];
    }
  }
  ps[j][i] = s;
  pn[j][i] = n;
  __syncthreads();
  if (j == 0 && b < a.nbins) {
    double t = 0.0;
    int64_t m = 0;
#pragma unroll
    for (int q = 0; q < 32; ++q) {
      t += ps[q][i];
      m += pn[q][i];
    }
    a.s_out[b] = m ? t / (double)m : 0.0;
    a.n_out[b] = m;
  }
}

// ---------------------------------------------------------------------------
// Finite check: flag[0] counts the arrays (of narr, n values each) holding
// a NaN or an infinity; one atomic per offending block.
// ---------------------------------------------------------------------------
struct FiniteArgs {
  const void* arr[2];
  int narr;
  int64_t n;
  unsigned* flag;   // flag[a] != 0: array a is not finite
};

template <typename T>
__global__ void __launch_bounds__(64) finite_clear_kernel(FiniteArgs a) {
  if (threadIdx.x < 2) a.flag[threadIdx.x] = 0u;
}

template <typename T>
__global__ void __launch_bounds__(256) finite_kernel(FiniteArgs a) {
  const T* v = (const T*)a.arr[blockIdx.y];
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * blockDim.x)
    bad |= !__builtin_isfinite(v[i]);
  if (__syncthreads_or(bad) && threadIdx.x == 0) atomicOr(&a.flag[blockIdx.y], 1u);
}

}  // namespace ss
