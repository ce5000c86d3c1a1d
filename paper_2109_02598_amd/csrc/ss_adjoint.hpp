// Reverse mode of the 2D Gray-Scott spectral step (the exact transpose of
// the discrete forward map, not of the continuous equations).
//
// Forward, per field j (u, v):  q_j' = Acal_j q_j + Bcal_j g_j(q),
//   g_u = F - u v^2, g_v = u v^2, Acal = IFFT A FFT, Bcal = IFFT B FFT,
//   with A = exp(L dt), B = (exp(L dt) - 1)/L of Sec. 2.4.2 (Eq. 4).
// A and B are real and even in k, so Acal and Bcal are symmetric and the
// transposed step is
//   mu_j     = Bcal_j lambda_j'
//   lambda_u = Acal_u lambda_u' + v^2 (mu_v - mu_u)
//   lambda_v = Acal_v lambda_v' + 2 u v (mu_v - mu_u)
// with u, v at the step's input level.  Coefficient gradients collect
//   <lambda_j', dAcal_j/dtheta q_j + dBcal_j/dtheta g_j> + <mu_j, dg_j/dtheta>
// with dA/dL = dt A and dB/dL = dt^2 phi1'(L dt).
//
// kadj  (k-space, per field): forward y FFTs of lambda', q, g; outputs the
//        x-spectra of Acal lambda' and of mu = Bcal lambda'; adds the
//        block's share of the spectral inner products to its accumulator.
// xadj  (x pass, both fields): inverse x FFTs of mu_u, mu_v, q_u, q_v;
//        pointwise Jacobian transpose; forward x FFT; plus Acal lambda'.
// All arrays use the layout and scaling of the forward state (x-spectrum
// / Nx, kx = 0 and Nyquist packed, transposed).
#pragma once

#include "ss_kernels.hpp"

namespace ss {

struct KAdjField {
  const void* lam;     // lambda' (adjoint of the step's output)
  const void* q;       // forward state at the step's input level
  const void* g;       // its nonlinear term (x-spectrum, unscaled)
  void* out_a;         // x-spectrum of Acal lambda'
  void* out_m;         // x-spectrum of mu = Bcal lambda'
  double l[2];         // L = l0 + l1 k^2
};

struct KAdjArgs {
  KAdjField fld[2];
  int nlines;          // Nx/2
  int lines_per_block;
  int nx;
  double sx, sy, dt;
  double a_scale;      // 1/Ny
  double nxd;          // Nx
  double* acc;         // [gridDim.y][gridDim.x][2]: sums of w (Nx dA P + dB Q) and k^2 times it
  double* dc;          // [1]: sum of mu_u over the grid (F-derivative of g_u)
  int lb;              // log2 of the row block of the spectral layout
};

// dphi1(z) = (z e^z - expm1(z)) / z^2 = 1/2 + z/3 + z^2/8 + z^3/30 + z^4/144 + ...
template <typename T>
__device__ __forceinline__ T dphi1_of(T z, T em) {
  const T lim = sizeof(T) == 8 ? (T)1e-3 : (T)0.1;
  if (z < lim && z > -lim) {
    return (T)0.5 + z * ((T)(1.0 / 3.0) + z * ((T)0.125 + z * ((T)(1.0 / 30.0) +
                    z * ((T)(1.0 / 144.0) + z * (T)(1.0 / 840.0)))));
  }
  return (z * ((T)1 + em) - em) / (z * z);
}

template <typename T>
struct AdjCoef {
  T a, b, da, db;   // A, B, dt A, dt^2 dphi1
};

template <typename T>
__device__ __forceinline__ AdjCoef<T> adj_coeffs(const KAdjField& f, double k2, double dt) {
  AdjCoef<T> r;
  const T z = (T)((f.l[0] + f.l[1] * k2) * dt);
  T A, phi, em;
  etd1_aphi<T>(z, A, phi, em);   // the forward step's own factors
  const T dtt = (T)dt;
  r.a = A;
  r.b = dtt * phi;
  r.da = dtt * r.a;
  r.db = dtt * dtt * dphi1_of<T>(z, em);
  return r;
}

template <typename T>
__device__ __forceinline__ T re_conj_mul(C<T> a, C<T> b) { return a.x * b.x + a.y * b.y; }

// Points per thread of the reverse sweep's transforms along an axis of n
// points: four up to 512 (twice the waves in flight, as the forward passes
// take on small grids), eight above.
constexpr int adj_pts(int n) { return n <= 512 ? 4 : 8; }

template <typename T, int NL>
__device__ __forceinline__ void kadj_body(const KAdjArgs& a, int bx, int fi, C<T>* lds, double* red) {
  constexpr int PT = adj_pts(NL), S = NL / PT;
  constexpr int REG = k_reg((int)sizeof(C<T>), NL);
  const int tid = threadIdx.x;
  const int ls = tid / S, t = tid - ls * S;
  const KAdjField F = fi == 0 ? a.fld[0] : a.fld[1];
  const int kxi = bx * a.lines_per_block + ls;
  const int64_t hx = a.nx / 2;
  const C<T>* pl = (const C<T>*)F.lam;
  const C<T>* pq = (const C<T>*)F.q;
  const C<T>* pg = (const C<T>*)F.g;
  const int L = a.lines_per_block;
  // three regions per block: lambda^, q^, g^ (each L lines)
  C<T>* xl = lds + (0 * L + ls) * REG;
  C<T>* xq = lds + (1 * L + ls) * REG;
  C<T>* xg = lds + (2 * L + ls) * REG;
  const Twiddles<T, NL, PT> tw = make_twiddles<T, NL, PT>(t);

  C<T> cl[1][PT], cq[1][PT], cg[1][PT];
#pragma unroll
  for (int e = 0; e < PT; ++e) {
    const int64_t ix = sidx(kxi, t + e * S, hx, a.lb);
    cl[0][e] = pl[ix];
    cq[0][e] = pq[ix];
    cg[0][e] = pg[ix];
  }
  {
    C<T>* x1[1] = {xl};
    fft_lines<T, NL, -1, 1, PT>(cl, x1, t, tw);
    fft_lines<T, NL, -1, 1, PT>(cq, x1, t, tw);
    fft_lines<T, NL, -1, 1, PT>(cg, x1, t, tw);
  }
  const bool packed_block = bx == 0;   // line kx = 0 holds kx = 0 and Nyquist
  const bool packed = kxi == 0;
  const double kxv = (double)kxi * a.sx;
  const double kny = (double)(a.nx / 2) * a.sx;
  const T nxd = (T)a.nxd;
  const T as = (T)a.a_scale;
  double s0 = 0.0, s1 = 0.0, dcs = 0.0;
  C<T> oa[1][PT], om[1][PT];
  if (packed_block) {
#pragma unroll
    for (int e = 0; e < PT; ++e) {
      xl[pidx<T>(t + e * S)] = cl[0][e];
      xq[pidx<T>(t + e * S)] = cq[0][e];
      xg[pidx<T>(t + e * S)] = cg[0][e];
    }
    __syncthreads();
  }
#pragma unroll
  for (int e = 0; e < PT; ++e) {
    const int p = t + e * S;
    const int m = p <= NL / 2 ? p : p - NL;
    const double ky = (double)m * a.sy;
    if (packed) {
      const int pm = (NL - p) & (NL - 1);
      const C<T> lm = cconj<T>(xl[pidx<T>(pm)]), qm = cconj<T>(xq[pidx<T>(pm)]), gm = cconj<T>(xg[pidx<T>(pm)]);
      const T h = (T)0.5;
      // kx = 0 parts (X + conj X(-k))/2 and Nyquist parts (X - conj X(-k))/(2i)
      const C<T> l0 = mk<T>(h * (cl[0][e].x + lm.x), h * (cl[0][e].y + lm.y));
      const C<T> ln = mk<T>(h * (cl[0][e].y - lm.y), -h * (cl[0][e].x - lm.x));
      const C<T> q0 = mk<T>(h * (cq[0][e].x + qm.x), h * (cq[0][e].y + qm.y));
      const C<T> qn = mk<T>(h * (cq[0][e].y - qm.y), -h * (cq[0][e].x - qm.x));
      const C<T> g0 = mk<T>(h * (cg[0][e].x + gm.x), h * (cg[0][e].y + gm.y));
      const C<T> gn = mk<T>(h * (cg[0][e].y - gm.y), -h * (cg[0][e].x - gm.x));
      const double k20 = ky * ky, k2n = ky * ky + kny * kny;
      const AdjCoef<T> c0 = adj_coeffs<T>(F, k20, a.dt), cn = adj_coeffs<T>(F, k2n, a.dt);
      const T v0 = nxd * c0.da * re_conj_mul<T>(l0, q0) + c0.db * re_conj_mul<T>(l0, g0);
      const T vn = nxd * cn.da * re_conj_mul<T>(ln, qn) + cn.db * re_conj_mul<T>(ln, gn);
      s0 += (double)v0 + (double)vn;
      s1 += k20 * (double)v0 + k2n * (double)vn;
      // outputs re-packed: X0 + i Xn with X0 = c0 * l0, Xn = cn * ln
      oa[0][e] = mk<T>(as * (c0.a * l0.x - cn.a * ln.y), as * (c0.a * l0.y + cn.a * ln.x));
      om[0][e] = mk<T>(as * (c0.b * l0.x - cn.b * ln.y), as * (c0.b * l0.y + cn.b * ln.x));
      if (p == 0) dcs = (double)a.nxd * (double)c0.b * (double)l0.x;
    } else {
      const double k2 = kxv * kxv + ky * ky;
      const AdjCoef<T> c = adj_coeffs<T>(F, k2, a.dt);
      const T v = nxd * c.da * re_conj_mul<T>(cl[0][e], cq[0][e]) + c.db * re_conj_mul<T>(cl[0][e], cg[0][e]);
      // interior kx planes stand for +kx and -kx of the full spectrum
      s0 += 2.0 * (double)v;
      s1 += 2.0 * k2 * (double)v;
      oa[0][e] = cscale<T>(cl[0][e], as * c.a);
      om[0][e] = cscale<T>(cl[0][e], as * c.b);
    }
  }
  if (packed_block) __syncthreads();
  {
    C<T>* x1[1] = {xl};
    fft_lines<T, NL, +1, 1, PT>(oa, x1, t, tw);
    fft_lines<T, NL, +1, 1, PT>(om, x1, t, tw);
  }
  C<T>* pa = (C<T>*)F.out_a;
  C<T>* pm = (C<T>*)F.out_m;
#pragma unroll
  for (int e = 0; e < PT; ++e) {
    const int64_t ix = sidx(kxi, t + e * S, hx, a.lb);
    pa[ix] = oa[0][e];
    pm[ix] = om[0][e];
  }
  // deterministic block reduction of (s0, s1)
  red[2 * tid] = s0;
  red[2 * tid + 1] = s1;
  __syncthreads();
  for (int w = (int)blockDim.x / 2; w > 0; w >>= 1) {
    if (tid < w) {
      red[2 * tid] += red[2 * (tid + w)];
      red[2 * tid + 1] += red[2 * (tid + w) + 1];
    }
    __syncthreads();
  }
  if (tid == 0) {
    double* acc = a.acc + 2 * ((int64_t)fi * gridDim.x + blockIdx.x);
    acc[0] += red[0];
    acc[1] += red[1];
  }
  if (packed && fi == 0 && t == 0 && a.dc) a.dc[0] += dcs;
}

template <typename T, int NL>
__global__ void __launch_bounds__(512) kadj_kernel(KAdjArgs a) {
  extern __shared__ __align__(16) unsigned char ss_dyn_lds[];
  constexpr int REG = k_reg((int)sizeof(C<T>), NL);
  C<T>* lds = reinterpret_cast<C<T>*>(ss_dyn_lds);
  double* red = reinterpret_cast<double*>(ss_dyn_lds + (size_t)3 * a.lines_per_block * REG * sizeof(C<T>));
  kadj_body<T, NL>(a, blockIdx.x, blockIdx.y, lds, red);
}

constexpr int64_t kadj_lds(int esz, int nl, int lines, int threads) {
  return (int64_t)3 * lines * k_reg(esz, nl) * esz + (int64_t)threads * 2 * 8;
}

// ---------------------------------------------------------------------------
struct XAdjArgs {
  const void* m[2];    // mu_u, mu_v (x-spectra)
  const void* q[2];    // u, v at the input level
  const void* la[2];   // Acal lambda' (x-spectra)
  void* out[2];        // lambda at the input level
  int64_t rows;
  int rows_per_block;
  int lb;              // log2 of the row block of the spectral layout
};

// six staged arrays per row pair: mu_u, mu_v, q_u, q_v, la_u, la_v
constexpr int64_t xadj_lds(int esz, int nx, int rows) { return (int64_t)(rows / 2) * 6 * x_reg(esz, nx, 6) * esz; }

template <typename T, int NX>
__global__ void __launch_bounds__(512) xadj_kernel(XAdjArgs a) {
  constexpr int PT = adj_pts(NX), S = NX / PT, H = NX / 2, HB = H + 1;
  constexpr int NA = 6;
  constexpr int REG = x_reg((int)sizeof(C<T>), NX, NA);
  extern __shared__ __align__(16) unsigned char ss_dyn_lds[];
  C<T>* lds = reinterpret_cast<C<T>*>(ss_dyn_lds);
  const int R = a.rows_per_block;
  const int NP = R >> 1;                      // row pairs of the tile
  const int G = (int)blockDim.x / S;
  const int tid = threadIdx.x;
  const int g = tid / S, t = tid - g * S;
  const int64_t s0 = (int64_t)blockIdx.x * R;
  const int64_t rows = a.rows;
  const Twiddles<T, NX, PT> tw = make_twiddles<T, NX, PT>(t);

  {
    const C<T>* src[NA] = {(const C<T>*)a.m[0], (const C<T>*)a.m[1], (const C<T>*)a.q[0],
                           (const C<T>*)a.q[1], (const C<T>*)a.la[0], (const C<T>*)a.la[1]};
    xstage_in<T, H, NA, NA, 0, REG, HB>(lds, src, s0, R, a.lb, tid, (int)blockDim.x);
  }
  __syncthreads();
  for (int it = 0; it < NP / G; ++it) {
    const int pr = it * G + g;
    C<T>* x[NA];
#pragma unroll
    for (int f = 0; f < NA; ++f) x[f] = lds + (pr * NA + f) * REG;
    C<T> c[4][PT];
#pragma unroll
    for (int f = 0; f < 4; ++f) {
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
    {
      C<T>* const xi[4] = {x[0], x[1], x[2], x[3]};
      fft_lines<T, NX, +1, 4, PT>(c, xi, t, tw);
    }
    // pointwise transpose of the Jacobian of (g_u, g_v) = (F - u v^2, u v^2)
    C<T> w[2][PT];
#pragma unroll
    for (int e = 0; e < PT; ++e) {
      const C<T> mu = c[0][e], mv = c[1][e], u = c[2][e], v = c[3][e];
      const T dx = mv.x - mu.x, dy = mv.y - mu.y;
      w[0][e] = mk<T>(v.x * v.x * dx, v.y * v.y * dy);
      w[1][e] = mk<T>((T)2 * u.x * v.x * dx, (T)2 * u.y * v.y * dy);
    }
    {
      C<T>* const xo[2] = {x[0], x[1]};
      fft_lines<T, NX, -1, 2, PT>(w, xo, t, tw);
    }
#pragma unroll
    for (int f = 0; f < 2; ++f) {
#pragma unroll
      for (int e = 0; e < PT; ++e) x[f][pidx<T>(t + e * S)] = w[f][e];
    }
    __syncthreads();
    const T sc = (T)1 / (T)NX;
    const T half = (T)0.5 * sc;
    C<T> fa[2][PT / 2], fb[2][PT / 2];
#pragma unroll
    for (int f = 0; f < 2; ++f) {
#pragma unroll
      for (int e = 0; e < PT / 2; ++e) {
        const int k = t + e * S;               // 0 .. H-1
        C<T> wk = x[f][pidx<T>(k)];
        C<T> ra, rb;
        if (k == 0) {
          C<T> wn = x[f][pidx<T>(H)];
          ra = mk<T>(wk.x * sc, wn.x * sc);
          rb = mk<T>(wk.y * sc, wn.y * sc);
        } else {
          C<T> wm = x[f][pidx<T>(NX - k)];
          ra = mk<T>((wk.x + wm.x) * half, (wk.y - wm.y) * half);
          rb = mk<T>((wk.y + wm.y) * half, (wm.x - wk.x) * half);
        }
        const C<T> la_a = x[4 + f][k], la_b = x[4 + f][HB + k];
        fa[f][e] = cadd<T>(ra, la_a);
        fb[f][e] = cadd<T>(rb, la_b);
      }
    }
    __syncthreads();
#pragma unroll
    for (int f = 0; f < 2; ++f) {
#pragma unroll
      for (int e = 0; e < PT / 2; ++e) {
        const int k = t + e * S;
        x[4 + f][k] = fa[f][e];
        x[4 + f][HB + k] = fb[f][e];
      }
    }
  }
  __syncthreads();
  {
    C<T>* dst[2] = {(C<T>*)a.out[0], (C<T>*)a.out[1]};
    xstage_out<T, H, 2, NA, 4, REG, HB>(dst, lds, s0, R, a.lb, tid, (int)blockDim.x);
  }
}

}  // namespace ss
