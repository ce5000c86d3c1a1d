// Register-resident Stockham FFT for gfx950, exchanged through LDS.
//
// One line of N (power of two, 8..4096) complex points is owned by S = N/P
// consecutive threads (P = 2, 4, 8 or 16 points per thread; the kernels take
// 4 on short lines of small grids, 8 or 16 otherwise); thread t holds the P
// points x[t + e*S], e = 0..P-1.  Every stage of the Stockham autosort
// reads that same set of positions, so the first stage can take its
// operands straight from global memory (coalesced) and, because the last
// stage writes each output back to the thread that holds its position, the
// result is again x[t + e*S] in natural order, in registers.  A forward
// transform followed by a pointwise operation and an inverse transform
// therefore touches LDS only between inner stages.
//
// Stage plan: one stage of radix 2^(log2 N mod log2 P) first (no twiddles)
// when log2 N is not a multiple of log2 P, then radix-P stages; P = 16 needs
// one LDS exchange fewer than P = 8 for N = 128, 1024, 2048 and 4096.  The
// twiddles exp(-+2 pi i r k/(Ns P)) of a radix-P butterfly are powers of one
// base value per thread and stage (computed once with sincospi); the powers
// are formed by multiplication.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ss {

template <typename T> struct cplx_of;
template <> struct cplx_of<float> { typedef float2 type; };
template <> struct cplx_of<double> { typedef double2 type; };
template <typename T> using C = typename cplx_of<T>::type;

template <typename T>
__device__ __forceinline__ C<T> mk(T x, T y) { C<T> r; r.x = x; r.y = y; return r; }
template <typename T>
__device__ __forceinline__ C<T> cadd(C<T> a, C<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ C<T> csub(C<T> a, C<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T>
__device__ __forceinline__ C<T> cmul(C<T> a, C<T> b) {
  return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T>
__device__ __forceinline__ C<T> cscale(C<T> a, T s) { return mk<T>(a.x * s, a.y * s); }
template <typename T>
__device__ __forceinline__ C<T> cconj(C<T> a) { return mk<T>(a.x, -a.y); }

// (a.x + i a.y) * (DIR * i)
template <typename T, int DIR>
__device__ __forceinline__ C<T> mul_diri(C<T> a) {
  return DIR > 0 ? mk<T>(-a.y, a.x) : mk<T>(a.y, -a.x);
}

__device__ __forceinline__ double2 cis_pi(double x) {
  double s, c;
  sincospi(x, &s, &c);
  return make_double2(c, s);
}
__device__ __forceinline__ float2 cis_pi(float x) {
  float s, c;
  sincospif(x, &s, &c);
  return make_float2(c, s);
}

// LDS index padding: one spare slot every 8 (16-byte elements) or 16
// (8-byte elements) points keeps the strided Stockham writes spread over
// the banks.
template <typename T>
__device__ __forceinline__ int pidx(int i) {
  return sizeof(T) == 8 ? i + (i >> 3) : i + (i >> 4);
}
template <typename T>
__host__ __device__ constexpr int padded_len(int n) {
  return sizeof(T) == 8 ? n + (n >> 3) + 1 : n + (n >> 4) + 1;
}

constexpr int ilog2c(int n) { return n <= 1 ? 0 : 1 + ilog2c(n >> 1); }
constexpr int ipow(int b, int e) { return e <= 0 ? 1 : b * ipow(b, e - 1); }

template <int N, int P = 8>
struct Plan {
  static_assert(P == 2 || P == 4 || P == 8 || P == 16, "2, 4, 8 or 16 points per thread");
  static constexpr int LOG = ilog2c(N);
  static constexpr int LP = ilog2c(P);
  static constexpr int FIRST = (LOG % LP == 0) ? P : (1 << (LOG % LP));
  static constexpr int NST = (LOG + LP - 1) / LP;
};

// ---- small DFTs, in place, sign DIR (-1 forward, +1 inverse) ------------
template <typename T, int DIR>
__device__ __forceinline__ void dft2(C<T>* v) {
  C<T> a = v[0];
  v[0] = cadd<T>(a, v[1]);
  v[1] = csub<T>(a, v[1]);
}

template <typename T, int DIR>
__device__ __forceinline__ void dft4(C<T>& x0, C<T>& x1, C<T>& x2, C<T>& x3) {
  C<T> t0 = cadd<T>(x0, x2), t1 = csub<T>(x0, x2);
  C<T> t2 = cadd<T>(x1, x3), t3 = mul_diri<T, DIR>(csub<T>(x1, x3));
  x0 = cadd<T>(t0, t2);
  x2 = csub<T>(t0, t2);
  x1 = cadd<T>(t1, t3);
  x3 = csub<T>(t1, t3);
}

template <typename T, int DIR>
__device__ __forceinline__ void dft4v(C<T>* v) { dft4<T, DIR>(v[0], v[1], v[2], v[3]); }

template <typename T, int DIR>
__device__ __forceinline__ void dft8(C<T>* v) {
  // even/odd split: E = DFT4(v0,v2,v4,v6), O = DFT4(v1,v3,v5,v7)
  C<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  C<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4<T, DIR>(e0, e1, e2, e3);
  dft4<T, DIR>(o0, o1, o2, o3);
  const T r = (T)0.70710678118654752440084436210484903928;
  // o1 *= w8, o2 *= w8^2, o3 *= w8^3 with w8 = exp(DIR 2 pi i / 8)
  C<T> p1 = mk<T>(r * (o1.x - (T)DIR * o1.y), r * (o1.y + (T)DIR * o1.x));
  C<T> p2 = mul_diri<T, DIR>(o2);
  C<T> p3 = mk<T>(r * (-o3.x - (T)DIR * o3.y), r * ((T)DIR * o3.x - o3.y));
  v[0] = cadd<T>(e0, o0);
  v[4] = csub<T>(e0, o0);
  v[1] = cadd<T>(e1, p1);
  v[5] = csub<T>(e1, p1);
  v[2] = cadd<T>(e2, p2);
  v[6] = csub<T>(e2, p2);
  v[3] = cadd<T>(e3, p3);
  v[7] = csub<T>(e3, p3);
}

// a * exp(DIR 2 pi i M / 16)
template <typename T, int DIR, int M>
__device__ __forceinline__ C<T> mul_w16(C<T> a) {
  constexpr double c1 = 0.92387953251128675612818318939678828682;   // cos(pi/8)
  constexpr double s1 = 0.38268343236508977172845998403039886676;   // sin(pi/8)
  constexpr double r2 = 0.70710678118654752440084436210484903928;   // cos(pi/4)
  if constexpr (M == 0) {
    return a;
  } else if constexpr (M == 4) {
    return mul_diri<T, DIR>(a);
  } else if constexpr (M == 2 || M == 6) {
    const T c = (T)(M == 2 ? r2 : -r2), sn = (T)r2;
    return mk<T>(c * a.x - (T)DIR * sn * a.y, c * a.y + (T)DIR * sn * a.x);
  } else {
    const T c = (T)(M == 1 ? c1 : M == 3 ? s1 : -c1);
    const T sn = (T)(M == 1 ? s1 : M == 3 ? c1 : -s1);
    return mk<T>(c * a.x - (T)DIR * sn * a.y, c * a.y + (T)DIR * sn * a.x);
  }
}

// 16-point DFT as 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2;
// X[k1 + 4 k2] = sum_n2 w16^(n2 k1) w4^(n2 k2) sum_n1 w4^(n1 k1) x[4 n1 + n2]
template <typename T, int DIR>
__device__ __forceinline__ void dft16(C<T>* v) {
  C<T> a[4][4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    C<T> x0 = v[n2], x1 = v[4 + n2], x2 = v[8 + n2], x3 = v[12 + n2];
    dft4<T, DIR>(x0, x1, x2, x3);
    a[n2][0] = x0;
    a[n2][1] = x1;
    a[n2][2] = x2;
    a[n2][3] = x3;
  }
  a[1][1] = mul_w16<T, DIR, 1>(a[1][1]);
  a[1][2] = mul_w16<T, DIR, 2>(a[1][2]);
  a[1][3] = mul_w16<T, DIR, 3>(a[1][3]);
  a[2][1] = mul_w16<T, DIR, 2>(a[2][1]);
  a[2][2] = mul_w16<T, DIR, 4>(a[2][2]);
  a[2][3] = mul_w16<T, DIR, 6>(a[2][3]);
  a[3][1] = mul_w16<T, DIR, 3>(a[3][1]);
  a[3][2] = mul_w16<T, DIR, 6>(a[3][2]);
  a[3][3] = mul_w16<T, DIR, 9>(a[3][3]);
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    C<T> y0 = a[0][k1], y1 = a[1][k1], y2 = a[2][k1], y3 = a[3][k1];
    dft4<T, DIR>(y0, y1, y2, y3);
    v[k1] = y0;
    v[k1 + 4] = y1;
    v[k1 + 8] = y2;
    v[k1 + 12] = y3;
  }
}

template <typename T, int DIR, int R>
__device__ __forceinline__ void dftR(C<T>* v) {
  if constexpr (R == 2) dft2<T, DIR>(v);
  else if constexpr (R == 4) dft4v<T, DIR>(v);
  else if constexpr (R == 8) dft8<T, DIR>(v);
  else dft16<T, DIR>(v);
}

// Base twiddles of one thread: for every radix-P stage after the first,
// w = exp(-2 pi i k / (Ns P)) with k = t mod Ns (forward sign; the inverse
// uses the conjugate).  Computed once per kernel and reused for every line
// the thread transforms.
template <typename T, int N, int P = 8>
struct Twiddles {
  static constexpr int NW = Plan<N, P>::NST > 1 ? Plan<N, P>::NST - 1 : 1;
  C<T> w[NW];
};

template <typename T, int N, int P = 8>
__device__ __forceinline__ Twiddles<T, N, P> make_twiddles(int t) {
  typedef Plan<N, P> PL;
  Twiddles<T, N, P> tw;
#pragma unroll
  for (int s = 1; s < PL::NST; ++s) {
    int ns = PL::FIRST;
#pragma unroll
    for (int u = 1; u < s; ++u) ns *= P;
    const int k = t & (ns - 1);
    tw.w[s - 1] = cis_pi((T)(-2 * k) / (T)(ns * P));
  }
  if (PL::NST == 1) tw.w[0] = mk<T>((T)1, (T)0);
  return tw;
}

// Keeps the compiler from hoisting values derived from x out of the
// caller's loops (which would hold every twiddle power live at once).
template <typename T>
__device__ __forceinline__ C<T> opaque(C<T> x) {
  asm volatile("" : "+v"(x.x), "+v"(x.y));
  return x;
}

// One Stockham stage of radix R over NL lines held by this thread.
// x[l] is the LDS exchange region of line l (padded indices).  On entry
// the regions must be free (no thread still reading them).  w1 is the
// forward base twiddle of this thread for the stage (unused when NS = 1).
template <typename T, int N, int DIR, int R, int NS, bool LAST, int NL, int P>
__device__ __forceinline__ void stockham_stage(C<T> (&c)[NL][P], C<T>* const (&x)[NL], int t,
                                               C<T> w1) {
  constexpr int S = N / P;
  constexpr int Q = P / R;
  static_assert(NS == 1 || Q == 1, "only the first stage may have radix < P");
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int j = t + q * S;
    const int k = j & (NS - 1);
    C<T> w[R];
    if constexpr (NS > 1 && NL > 1) {
      // several lines share the powers: form them once
      w[1] = opaque<T>(DIR > 0 ? cconj<T>(w1) : w1);
#pragma unroll
      for (int r = 2; r < R; ++r) w[r] = cmul<T>(w[r >> 1], w[r - (r >> 1)]);
    }
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      C<T> v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = c[l][q + r * Q];
      if constexpr (NS > 1 && NL > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) v[r] = cmul<T>(v[r], w[r]);
      } else if constexpr (NS > 1) {
        // one line: walk the powers while applying them (two live values)
        const C<T> wb = opaque<T>(DIR > 0 ? cconj<T>(w1) : w1);
        C<T> wr = wb;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          v[r] = cmul<T>(v[r], wr);
          if (r + 1 < R) wr = cmul<T>(wr, wb);
        }
      }
      dftR<T, DIR, R>(v);
      if constexpr (LAST) {
#pragma unroll
        for (int r = 0; r < R; ++r) c[l][q + r * Q] = v[r];
      } else {
        const int base = (j - k) * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) x[l][pidx<T>(base + r * NS)] = v[r];
      }
    }
  }
  if constexpr (!LAST) {
    __syncthreads();
#pragma unroll
    for (int l = 0; l < NL; ++l) {
#pragma unroll
      for (int e = 0; e < P; ++e) c[l][e] = x[l][pidx<T>(t + e * S)];
    }
    __syncthreads();
  }
}

// Stage s of the plan (first: radix FIRST, no twiddles; then radix P).
template <typename T, int N, int DIR, int NL, int P, int ST>
__device__ __forceinline__ void fft_stages(C<T> (&c)[NL][P], C<T>* const (&x)[NL], int t,
                                           const Twiddles<T, N, P>& tw) {
  typedef Plan<N, P> PL;
  if constexpr (ST < PL::NST) {
    constexpr int R = ST == 0 ? PL::FIRST : P;
    constexpr int NS = ST == 0 ? 1 : PL::FIRST * ipow(P, ST - 1);
    stockham_stage<T, N, DIR, R, NS, ST == PL::NST - 1, NL, P>(c, x, t, tw.w[ST == 0 ? 0 : ST - 1]);
    fft_stages<T, N, DIR, NL, P, ST + 1>(c, x, t, tw);
  }
}

// Unnormalised DFT of NL lines of length N: sign DIR (-1 forward).
template <typename T, int N, int DIR, int NL, int P = 8>
__device__ __forceinline__ void fft_lines(C<T> (&c)[NL][P], C<T>* const (&x)[NL], int t,
                                          const Twiddles<T, N, P>& tw) {
  static_assert(N >= P && N <= 4096 && (N & (N - 1)) == 0, "power of two in [P, 4096]");
  fft_stages<T, N, DIR, NL, P, 0>(c, x, t, tw);
}

}  // namespace ss
