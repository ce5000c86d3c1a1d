// One-workgroup spectral step for small 2D grids.
//
// On a small grid the two passes of a step are latency-bound: each is a
// handful of waves on an otherwise idle GPU, and a step pays two kernel
// launches.  Here one workgroup holds the whole spectral state of a
// one-field grid for a run of steps: the carried spectrum S^ in registers
// (lines along y, 2 to 8 points per thread), the row pass's data and every
// exchange in LDS.  A run reads the state once and writes it once; a step
// costs no launch and no HBM traffic.  The ETD1 factors of every mode do
// not change between steps: a small kernel computes them once per run into
// a table the step kernel reads (L2-resident).
//
// Per step (Sec. 2.4.2, Eqs. 3-4 and 8, as the two-pass step):
//   T -> LDS in row-pair layout; per row pair: inverse x FFT, f(psi),
//   forward x FFT, split into the two rows' half spectra (G) in LDS;
//   per k-space line: forward y FFT of G, U = A S^ + B N G^ (the packed
//   kx = 0 / Nyquist line with its mirror mode), S^ = U, T = inverse y FFT
//   of U.  Scalings as the two-pass step: S^ = FFT_xy(psi)/N, T =
//   FFT_x(psi)/Nx.
#pragma once

#include "ss_kernels.hpp"

namespace ss {

struct SmallArgs {
  void* state;          // T, spectral layout (row block 2^lb)
  void* shat;           // S^, same layout
  void* coef;           // factor table (small_coef_kernel): 2 x (N/2) x N values
  void* coef_nyq;       // the packed line's second factors: 2 x N values
  int lb;
  int nsteps;
  int load_shat;        // 1: S^ is current and is read; 0: formed from T
  double sx, sy;        // 2 pi / (N_axis dx_axis)
  double dt, b_scale;   // time step, 1/N
  KField f;             // L(k^2) and N(k^2)
  double p[3];          // coefficients of the pointwise term
  double* mass_log;     // may be null
  int64_t log_index;    // row of the first step of the run
  int64_t log_capacity;
};

// Square grids N x N, N = 16 .. 128.  Points per thread: as few as keep
// the workgroup's lines in registers, so that the step spreads over the
// CU's four SIMDs (one workgroup has no other waves to hide its latencies
// behind).  Measured per step (Allen-Cahn, FP64 / FP32, one MI355X):
//   N = 16:  2 points (64 threads)          2.3 / 2.0 us (16 points: 5.9 / 5.1)
//   N = 32:  4 / 2 points (128 / 256)       4.2 / 3.4 us (16 points: 11.7 / 10.6)
//   N = 64:  4 points (512 threads)         7.9 / 5.5 us (16 points: 13.6 / 10.9)
//   N = 128: 8 points (1024 threads)        23.6 / 14.8 us (FP32, 16 points: 16.0)
// (the FP64 128 line of 16 points beside the carried spectrum spills).
template <typename T, int N>
struct SmallCfg {
  static constexpr int P = N == 16 ? 2 : N == 32 ? (sizeof(T) == 8 ? 4 : 2) : N == 64 ? 4 : 8;
  static constexpr int H = N / 2;     // k-space lines (kx = 0 .. N/2 - 1, kx = 0 packed with Nyquist)
  static constexpr int S = N / P;     // threads per k-space line = threads per row pair
  static constexpr int W = H * S;     // threads of the workgroup (also (N/2) row pairs x S)
  static constexpr int HB = H + 1;    // offset of a pair's second row in its region
};

// LDS bytes: the row-pair regions or the line regions, whichever is larger
constexpr int64_t small_lds(int esz, int n) {
  return (int64_t)(n / 2) * (x_reg(esz, n, 1) > k_reg(esz, n) ? x_reg(esz, n, 1) : k_reg(esz, n)) * esz;
}
// factor tables (entries of the element type): (a, b) for every element
// of every thread, N^2 (one field array); (a-, b-) for the packed line's
// elements, 2 N (any points per thread)
constexpr int64_t small_coef_len(int n) { return (int64_t)n * n; }
constexpr int64_t small_coef_nyq_len(int n) { return 2 * (int64_t)n; }

// Factors of the elements of thread tid: for lines kx >= 1, (A, B N) of
// the mode; for the packed line, ((a0 + an)/2, (b0 + bn)/2) and
// ((a0 - an)/2, (b0 - bn)/2), a0/b0 of kx = 0 and an/bn of the Nyquist
// plane (the pairing the two-pass step applies).
template <typename T, int N>
__global__ void __launch_bounds__((SmallCfg<T, N>::W)) small_coef_kernel(SmallArgs a) {
  typedef SmallCfg<T, N> K;
  constexpr int P = K::P, S = K::S, W = K::W;
  const int tid = threadIdx.x;
  const int kx = tid / S, t = tid - kx * S;
  T* main_tab = (T*)a.coef;
  T* nyq_tab = (T*)a.coef_nyq;
  const T kny = (T)(N / 2) * (T)a.sx;
  const T kxv = (T)kx * (T)a.sx;
  for (int e = 0; e < P; ++e) {
    const int p = t + e * S;
    const int m = p <= N / 2 ? p : p - N;
    const T kl = (T)m * (T)a.sy;
    const int64_t i = (int64_t)e * W + tid;
    if (kx == 0) {
      const T k2_0 = kl * kl;
      T a0, b0, an, bn;
      etd1_coeffs<T, 0>(a.f, k2_0, a.dt, 1.0, a.b_scale, a0, b0);
      etd1_coeffs<T, 0>(a.f, k2_0 + kny * kny, a.dt, 1.0, a.b_scale, an, bn);
      main_tab[2 * i] = (T)0.5 * (a0 + an);
      main_tab[2 * i + 1] = (T)0.5 * (b0 + bn);
      nyq_tab[2 * (e * S + t)] = (T)0.5 * (a0 - an);
      nyq_tab[2 * (e * S + t) + 1] = (T)0.5 * (b0 - bn);
    } else {
      const T k2 = kxv * kxv + kl * kl;
      T av, bv;
      etd1_coeffs<T, 0>(a.f, k2, a.dt, 1.0, a.b_scale, av, bv);
      main_tab[2 * i] = av;
      main_tab[2 * i + 1] = bv;
    }
  }
}

template <typename T, int N>
__global__ void __launch_bounds__((SmallCfg<T, N>::W)) small_step_kernel(SmallArgs a) {
  typedef SmallCfg<T, N> K;
  constexpr int P = K::P, H = K::H, S = K::S, W = K::W, HB = K::HB;
  constexpr int ESZ = (int)sizeof(C<T>);
  constexpr int REGX = x_reg(ESZ, N, 1), REGK = k_reg(ESZ, N);
  extern __shared__ __align__(16) unsigned char ss_dyn_lds[];
  C<T>* lds = reinterpret_cast<C<T>*>(ss_dyn_lds);
  // k-space line kx, its elements y = t + e S; row pair pr, elements k =
  // t + e S (the same split of the threads serves both passes).  Indices
  // and addresses are formed again inside the step loop from a copy of
  // the thread index the compiler cannot see through, so that they are not
  // held in registers across the loop beside the two lines of data.
  const int tid0 = threadIdx.x;
  const Twiddles<T, N, P> tw = make_twiddles<T, N, P>(tid0 % S);
  const T* main_tab = (const T*)a.coef;
  const T* nyq_tab = (const T*)a.coef_nyq;
  const T p0 = (T)a.p[0], p1 = (T)a.p[1], p2 = (T)a.p[2];

  C<T> s[1][P], c[1][P];
  const int kx0 = tid0 / S, t0 = tid0 - kx0 * S;
  const C<T>* gT = (const C<T>*)a.state;
#pragma unroll
  for (int e = 0; e < P; ++e) c[0][e] = gT[sidx(kx0, t0 + e * S, H, a.lb)];
  if (a.load_shat) {
    const C<T>* gS = (const C<T>*)a.shat;
#pragma unroll
    for (int e = 0; e < P; ++e) s[0][e] = gS[sidx(kx0, t0 + e * S, H, a.lb)];
  } else {
#pragma unroll
    for (int e = 0; e < P; ++e) s[0][e] = c[0][e];
    C<T>* xk0[1] = {lds + kx0 * REGK};
    fft_lines<T, N, -1, 1, P>(s, xk0, t0, tw);
    const T sc = (T)1 / (T)N;
#pragma unroll
    for (int e = 0; e < P; ++e) s[0][e] = cscale<T>(s[0][e], sc);
  }

  for (int step = 0; step < a.nsteps; ++step) {
    int tid = tid0;
    asm volatile("" : "+v"(tid));
    const int kx = tid / S, t = tid - kx * S;
    const int pr = kx;
    const bool packed = kx == 0;
    C<T>* xk[1] = {lds + kx * REGK};
    C<T>* xr[1] = {lds + pr * REGX};
    // T (k-space layout) -> LDS (row-pair layout: row y of plane kx)
    __syncthreads();
#pragma unroll
    for (int e = 0; e < P; ++e) {
      const int y = t + e * S;
      lds[(y >> 1) * REGX + (y & 1) * HB + kx] = c[0][e];
    }
    __syncthreads();
    // row pair pr: Z[k] = X_a[k] + i X_b[k] over the full length
#pragma unroll
    for (int e = 0; e < P; ++e) {
      const int k = t + e * S;
      C<T> z;
      if (k == 0) {
        C<T> ta = xr[0][0], tb = xr[0][HB];
        z = mk<T>(ta.x, tb.x);
      } else if (k == H) {
        C<T> ta = xr[0][0], tb = xr[0][HB];
        z = mk<T>(ta.y, tb.y);
      } else if (k < H) {
        C<T> ta = xr[0][k], tb = xr[0][HB + k];
        z = mk<T>(ta.x - tb.y, ta.y + tb.x);
      } else {
        C<T> ta = xr[0][N - k], tb = xr[0][HB + N - k];
        z = mk<T>(ta.x + tb.y, tb.x - ta.y);
      }
      c[0][e] = z;
    }
    __syncthreads();
    fft_lines<T, N, +1, 1, P>(c, xr, t, tw);
#pragma unroll
    for (int e = 0; e < P; ++e) nonlinear<T, NLIN_POLY>(&c[0][e], &c[0][e], p0, p1, p2);
    fft_lines<T, N, -1, 1, P>(c, xr, t, tw);
    // split the two rows: G_a[k], G_b[k] for k < H (kx = 0 packs Nyquist)
#pragma unroll
    for (int e = 0; e < P; ++e) xr[0][pidx<T>(t + e * S)] = c[0][e];
    __syncthreads();
    C<T> fa[P / 2], fb[P / 2];
#pragma unroll
    for (int e = 0; e < P / 2; ++e) {
      const int k = t + e * S;
      C<T> w = xr[0][pidx<T>(k)];
      if (k == 0) {
        C<T> wn = xr[0][pidx<T>(H)];
        fa[e] = mk<T>(w.x, wn.x);
        fb[e] = mk<T>(w.y, wn.y);
      } else {
        C<T> wm = xr[0][pidx<T>(N - k)];
        const T half = (T)0.5;
        fa[e] = mk<T>((w.x + wm.x) * half, (w.y - wm.y) * half);
        fb[e] = mk<T>((w.y + wm.y) * half, (wm.x - w.x) * half);
      }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < P / 2; ++e) {
      const int k = t + e * S;
      xr[0][k] = fa[e];
      xr[0][HB + k] = fb[e];
    }
    __syncthreads();
    // line kx of G, then its forward transform along y
#pragma unroll
    for (int e = 0; e < P; ++e) {
      const int y = t + e * S;
      c[0][e] = lds[(y >> 1) * REGX + (y & 1) * HB + kx];
    }
    __syncthreads();
    fft_lines<T, N, -1, 1, P>(c, xk, t, tw);
    // U = A S^ + B N G^; the packed line pairs each mode with its mirror
#pragma unroll
    for (int e = 0; e < P; ++e) xk[0][pidx<T>(t + e * S)] = s[0][e];
    __syncthreads();
    if (packed) {
#pragma unroll
      for (int e = 0; e < P; ++e) {
        const int p = t + e * S;
        const int64_t i = (int64_t)e * W + tid;
        const T ap = main_tab[2 * i], am = nyq_tab[2 * (e * S + t)];
        const C<T> cm = cconj<T>(xk[0][pidx<T>((N - p) & (N - 1))]);
        s[0][e] = mk<T>(ap * s[0][e].x + am * cm.x, ap * s[0][e].y + am * cm.y);
      }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < P; ++e) xk[0][pidx<T>(t + e * S)] = c[0][e];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < P; ++e) {
      const int p = t + e * S;
      const int64_t i = (int64_t)e * W + tid;
      const T av = main_tab[2 * i], bv = main_tab[2 * i + 1];
      if (packed) {
        const T bmn = nyq_tab[2 * (e * S + t) + 1];
        const C<T> dm = cconj<T>(xk[0][pidx<T>((N - p) & (N - 1))]);
        s[0][e] = mk<T>(s[0][e].x + bv * c[0][e].x + bmn * dm.x, s[0][e].y + bv * c[0][e].y + bmn * dm.y);
      } else {
        s[0][e] = mk<T>(av * s[0][e].x + bv * c[0][e].x, av * s[0][e].y + bv * c[0][e].y);
      }
    }
    if (tid == 0 && a.mass_log && a.log_index + step < a.log_capacity)
      a.mass_log[a.log_index + step] = (double)s[0][0].x;
    __syncthreads();
    // T = inverse y transform of U
#pragma unroll
    for (int e = 0; e < P; ++e) c[0][e] = s[0][e];
    fft_lines<T, N, +1, 1, P>(c, xk, t, tw);
  }

  int tid = tid0;
  asm volatile("" : "+v"(tid));
  const int kx = tid / S, t = tid - kx * S;
  C<T>* oT = (C<T>*)a.state;
  C<T>* oS = (C<T>*)a.shat;
#pragma unroll
  for (int e = 0; e < P; ++e) {
    const int64_t g = sidx(kx, t + e * S, H, a.lb);
    oT[g] = c[0][e];
    oS[g] = s[0][e];
  }
}

}  // namespace ss
