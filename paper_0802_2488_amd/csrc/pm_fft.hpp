// Register/LDS radix FFT building blocks for CDNA4 (gfx950, wave64).
//
// One transform of length N is carried out by a team of TPF = N / RMAX
// threads.  Between kernels' compute phases the data sits in registers in the
// "pattern A" layout: thread t of the team holds elements t + TPF * s,
// s = 0..RMAX-1, in register slot s.  The Stockham autosort decomposition
// (radix RMAX, a smaller middle radix when N is not a power of RMAX, radix
// RMAX last) both starts from and ends in pattern A, in natural order, so a
// kernel can
//   load pattern A from HBM -> FFT -> pointwise work -> FFT -> store
// with LDS used only for the exchanges between radix stages.
//
// Conventions: forward transform DIR = -1, X[k] = sum_n x[n] exp(-2 pi i nk/N);
// inverse DIR = +1, unnormalised.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pm {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T re, im;
};

// Pointer into global memory.  Buffers reached through a descriptor read
// from memory are generic pointers to the compiler, and generic accesses
// become flat instructions, which also count against the LDS wait counter;
// kernels convert such pointers with glb() so their accesses are global.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gptr<T> glb(T* p) {
  return (gptr<T>)p;
}

// Complex loads and stores through LDS (generic) or global pointers; the
// global forms move both parts as one 2-vector.
template <typename T>
using vec2 = T __attribute__((ext_vector_type(2)));
template <typename T>
__device__ __forceinline__ cx<T> ldc(const cx<T>* p) { return *p; }
template <typename T>
__device__ __forceinline__ cx<T> ldc(gptr<const cx<T>> p) {
  const vec2<T> v = *(gptr<const vec2<T>>)p;
  return {v.x, v.y};
}
template <typename T>
__device__ __forceinline__ cx<T> ldc(gptr<cx<T>> p) { return ldc((gptr<const cx<T>>)p); }
template <typename T>
__device__ __forceinline__ void stc(cx<T>* p, cx<T> a) { *p = a; }
template <typename T>
__device__ __forceinline__ void stc(gptr<cx<T>> p, cx<T> a) {
  vec2<T> v;
  v.x = a.re;
  v.y = a.im;
  *(gptr<vec2<T>>)p = v;
}

template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cx<T> cconj(cx<T> a) { return {a.re, -a.im}; }
template <typename T>
__device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return {a.re * s, a.im * s}; }
// multiply by DIR * i
template <int DIR, typename T>
__device__ __forceinline__ cx<T> mul_diri(cx<T> a) {
  if constexpr (DIR < 0) return {a.im, -a.re};
  else return {-a.im, a.re};
}

// cos(2 pi m / 16) and sin(2 pi m / 16), m = 0..15 (exact mathematical values).
constexpr double kC16[16] = {
    1.0, 0.923879532511286756128183189396788933, 0.707106781186547524400844362104849039,
    0.382683432365089771728459984030398866, 0.0, -0.382683432365089771728459984030398866,
    -0.707106781186547524400844362104849039, -0.923879532511286756128183189396788933, -1.0,
    -0.923879532511286756128183189396788933, -0.707106781186547524400844362104849039,
    -0.382683432365089771728459984030398866, 0.0, 0.382683432365089771728459984030398866,
    0.707106781186547524400844362104849039, 0.923879532511286756128183189396788933};
constexpr double kS16[16] = {
    0.0, 0.382683432365089771728459984030398866, 0.707106781186547524400844362104849039,
    0.923879532511286756128183189396788933, 1.0, 0.923879532511286756128183189396788933,
    0.707106781186547524400844362104849039, 0.382683432365089771728459984030398866, 0.0,
    -0.382683432365089771728459984030398866, -0.707106781186547524400844362104849039,
    -0.923879532511286756128183189396788933, -1.0, -0.923879532511286756128183189396788933,
    -0.707106781186547524400844362104849039, -0.382683432365089771728459984030398866};

// a * exp(DIR * 2 pi i m / R) for a compile-time m, R in {2, 4, 8, 16}.
template <int DIR, int R, int M, typename T>
__device__ __forceinline__ cx<T> twc(cx<T> a) {
  constexpr int m16 = ((M * (16 / R)) % 16 + 16) % 16;
  if constexpr (m16 == 0) return a;
  else if constexpr (m16 == 8) return {-a.re, -a.im};
  else if constexpr (m16 == 4) return mul_diri<DIR>(a);
  else if constexpr (m16 == 12) return mul_diri<-DIR>(a);
  else {
    constexpr double cd = kC16[m16];
    constexpr double sd = DIR * kS16[m16];
    const T c = (T)cd;
    const T s = (T)sd;
    return {a.re * c - a.im * s, a.re * s + a.im * c};
  }
}

template <int DIR, typename T>
__device__ __forceinline__ void dft2(cx<T>* v) {
  cx<T> a = v[0], b = v[1];
  v[0] = a + b;
  v[1] = a - b;
}

template <int DIR, typename T>
__device__ __forceinline__ void dft4(cx<T>* v) {
  cx<T> a0 = v[0] + v[2], a1 = v[0] - v[2];
  cx<T> a2 = v[1] + v[3], a3 = mul_diri<DIR>(v[1] - v[3]);
  v[0] = a0 + a2;
  v[2] = a0 - a2;
  v[1] = a1 + a3;
  v[3] = a1 - a3;
}

// Two-level split R = R1 * R2: n = R2 n1 + n2, k = k1 + R1 k2.
template <int DIR, int R1, int R2, typename T>
__device__ __forceinline__ void dft_split(cx<T>* v);

template <int DIR, int R, typename T>
__device__ __forceinline__ void dft(cx<T>* v) {
  if constexpr (R == 2) dft2<DIR>(v);
  else if constexpr (R == 4) dft4<DIR>(v);
  else if constexpr (R == 8) dft_split<DIR, 2, 4>(v);
  else if constexpr (R == 16) dft_split<DIR, 4, 4>(v);
  else static_assert(R == 2 || R == 4 || R == 8 || R == 16, "unsupported radix");
}

template <int DIR, int R1, int R2, int N2, int K1, typename T>
__device__ __forceinline__ void split_tw(cx<T> (&y)[R2][R1]) {
  y[N2][K1] = twc<DIR, R1 * R2, N2 * K1>(y[N2][K1]);
  if constexpr (K1 + 1 < R1) split_tw<DIR, R1, R2, N2, K1 + 1>(y);
  else if constexpr (N2 + 1 < R2) split_tw<DIR, R1, R2, N2 + 1, 0>(y);
}

template <int DIR, int R1, int R2, typename T>
__device__ __forceinline__ void dft_split(cx<T>* v) {
  cx<T> y[R2][R1];
#pragma unroll
  for (int n2 = 0; n2 < R2; ++n2) {
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) y[n2][n1] = v[R2 * n1 + n2];
    dft<DIR, R1>(y[n2]);
  }
  split_tw<DIR, R1, R2, 0, 0>(y);
#pragma unroll
  for (int k1 = 0; k1 < R1; ++k1) {
    cx<T> z[R2];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) z[n2] = y[n2][k1];
    dft<DIR, R2>(z);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) v[k1 + R1 * k2] = z[k2];
  }
}

// Dependency fence on register-resident values: the empty asm "redefines"
// every element, so no arithmetic can move across it in either direction.
// Used between the phases of a fused kernel (load, transform, pointwise
// work) to keep the compiler from interleaving them, which otherwise raises
// register pressure into spills.
template <typename T, int R>
__device__ __forceinline__ void fence(cx<T> (&z)[R]) {
#pragma unroll
  for (int i = 0; i < R; ++i) asm volatile("" : "+v"(z[i].re), "+v"(z[i].im));
}

// ---------------------------------------------------------------------------
// Radix plan: N = RMAX^s * rem (rem < RMAX); stages RMAX, ..., rem, RMAX.
template <int N, int RMAX>
struct Plan {
  static constexpr int log2i(int x) { return x <= 1 ? 0 : 1 + log2i(x / 2); }
  static constexpr int LN = log2i(N);
  static constexpr int LR = log2i(RMAX);
  static constexpr int NFULL = LN / LR;           // number of radix-RMAX stages
  static constexpr int REM = 1 << (LN - NFULL * LR);
  static constexpr int NSTAGE = NFULL + (REM > 1 ? 1 : 0);
  static constexpr int TPF = N / RMAX;
  static_assert((1 << LN) == N, "N must be a power of two");
  static_assert(N >= RMAX, "N must be at least RMAX");
  // radix of stage i: the middle factor sits just before the last stage
  static constexpr int radix(int i) {
    return (REM > 1 && NSTAGE >= 2 && i == NSTAGE - 2) ? REM : (REM > 1 && NSTAGE == 1 ? REM : RMAX);
  }
  static constexpr int ns(int i) { return i == 0 ? 1 : ns(i - 1) * radix(i - 1); }
};

// LDS index with one padding element every 16 (breaks power-of-two strides).
__device__ __forceinline__ int lpad(int i) { return i + (i >> 4); }
template <int N>
struct LdsSize {
  static constexpr int value = N + N / 16;
};

// Twiddle exp(DIR * 2 pi i * idx / N) from a forward table tw[i] = exp(-2 pi i i / N).
template <int DIR, typename T>
__device__ __forceinline__ cx<T> twl(gptr<const cx<T>> __restrict__ tw, int idx) {
  cx<T> w = ldc(tw + idx);
  if constexpr (DIR > 0) w.im = -w.im;
  return w;
}

// Twiddle seeds of one stage for one thread: for each of its B butterflies
// the powers w, w^2, w^4, w^8 (as far as the radix needs) of
// w = exp(DIR 2 pi i base / N), read from the table.  A stage's seeds are
// loaded while the previous stage computes, so the table reads overlap work.
template <typename T, int B>
struct Seeds {
  cx<T> w[B][4];
};

template <int DIR, typename T, int N, int RMAX, int STAGE>
using StageSeeds = Seeds<T, RMAX / Plan<N, RMAX>::radix(STAGE)>;

template <int DIR, typename T, int N, int RMAX, int STAGE>
__device__ __forceinline__ void load_seeds(StageSeeds<DIR, T, N, RMAX, STAGE>& sd, gptr<const cx<T>> __restrict__ tw,
                                           int t) {
  using P = Plan<N, RMAX>;
  constexpr int R = P::radix(STAGE);
  constexpr int NS = P::ns(STAGE);
  constexpr int B = RMAX / R;
  if constexpr (NS > 1) {
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int j = t + b * P::TPF;
      const int base = (j % NS) * (N / (NS * R));
      sd.w[b][0] = twl<DIR>(tw, base);
      if constexpr (R >= 4) sd.w[b][1] = twl<DIR>(tw, 2 * base);
      if constexpr (R >= 8) sd.w[b][2] = twl<DIR>(tw, 4 * base);
      if constexpr (R >= 16) sd.w[b][3] = twl<DIR>(tw, 8 * base);
    }
  }
}

// Multiply u[1..R-1] by w^r from the seeds w, w^2, w^4, w^8; the other
// powers take at most three products.
template <int R, typename T>
__device__ __forceinline__ void apply_seeds(cx<T>* u, const cx<T> (&sd)[4]) {
  if constexpr (R == 2) {
    u[1] = cmul(u[1], sd[0]);
  } else if constexpr (R == 4) {
    const cx<T> w3 = cmul(sd[0], sd[1]);
    u[1] = cmul(u[1], sd[0]);
    u[2] = cmul(u[2], sd[1]);
    u[3] = cmul(u[3], w3);
  } else {
    cx<T> w[R];
    w[1] = sd[0];
    w[2] = sd[1];
    w[4] = sd[2];
    w[3] = cmul(w[1], w[2]);
    w[5] = cmul(w[4], w[1]);
    w[6] = cmul(w[4], w[2]);
    w[7] = cmul(w[4], w[3]);
    if constexpr (R == 16) {
      w[8] = sd[3];
#pragma unroll
      for (int r = 9; r < 16; ++r) w[r] = cmul(w[8], w[r - 8]);
    }
#pragma unroll
    for (int r = 1; r < R; ++r) u[r] = cmul(u[r], w[r]);
  }
}

// LDS exchange buffers of one transform team, from a base pointer: buffer
// b holds S = LdsSize<N>::value complex values (real and imaginary part
// side by side, one LDS access each) at base + 2 b S.  With one buffer a
// stage's writes wait at a barrier
// until every thread has read the previous stage; with two (DB),
// consecutive exchanges alternate between the buffers, so only the barrier
// between an exchange's writes and its reads remains.
//
// One Stockham stage, the X-th exchange of a chain of transforms.  Input:
// stage 0 takes pattern A from v; later stages read exchange X - 1 from LDS.
// Output: the last stage writes pattern A to v; earlier stages write
// exchange X to LDS.
template <int DIR, typename T, int N, int RMAX, int STAGE, bool DB, int X>
__device__ __forceinline__ void stockham_stage(cx<T> (&v)[RMAX], T* __restrict__ xb, int t,
                                               const StageSeeds<DIR, T, N, RMAX, STAGE>& sd) {
  using P = Plan<N, RMAX>;
  constexpr int R = P::radix(STAGE);
  constexpr int NS = P::ns(STAGE);
  constexpr int TPF = P::TPF;
  constexpr int B = RMAX / R;
  constexpr bool FIRST = STAGE == 0;
  constexpr bool LAST = STAGE == P::NSTAGE - 1;
  constexpr int S = LdsSize<N>::value;
  constexpr int RD = DB ? ((X - 1) & 1) : 0, WR = DB ? (X & 1) : 0;
  cx<T> u[RMAX];
#pragma unroll
  for (int b = 0; b < B; ++b) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if constexpr (FIRST) {
        u[b * R + r] = v[b + B * r];
      } else {
        const int j = t + b * TPF;
        const int idx = lpad(j + r * (N / R));
        u[b * R + r] = reinterpret_cast<const cx<T>*>(xb + 2 * RD * S)[idx];
      }
    }
  }
#pragma unroll
  for (int b = 0; b < B; ++b) {
    if constexpr (NS > 1) apply_seeds<R>(&u[b * R], sd.w[b]);
    dft<DIR, R>(&u[b * R]);
  }
  if constexpr (LAST) {
#pragma unroll
    for (int b = 0; b < B; ++b)
#pragma unroll
      for (int r = 0; r < R; ++r) v[b + B * r] = u[b * R + r];
  } else {
    if constexpr (!DB) __syncthreads();
    cx<T>* __restrict__ wb = reinterpret_cast<cx<T>*>(xb + 2 * WR * S);
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int j = t + b * TPF;
      const int base = (j / NS) * NS * R + (j % NS);
#pragma unroll
      for (int r = 0; r < R; ++r) wb[lpad(base + r * NS)] = u[b * R + r];
    }
    __syncthreads();
  }
}

template <int DIR, typename T, int N, int RMAX, int STAGE, bool DB, int X0>
__device__ __forceinline__ void fft_stages(cx<T> (&v)[RMAX], T* xb, int t, gptr<const cx<T>> tw,
                                           const StageSeeds<DIR, T, N, RMAX, STAGE>& cur) {
  if constexpr (STAGE + 1 < Plan<N, RMAX>::NSTAGE) {
    StageSeeds<DIR, T, N, RMAX, STAGE + 1> nxt;
    load_seeds<DIR, T, N, RMAX, STAGE + 1>(nxt, tw, t);
    stockham_stage<DIR, T, N, RMAX, STAGE, DB, X0 + STAGE>(v, xb, t, cur);
    fft_stages<DIR, T, N, RMAX, STAGE + 1, DB, X0>(v, xb, t, tw, nxt);
  } else {
    stockham_stage<DIR, T, N, RMAX, STAGE, DB, X0 + STAGE>(v, xb, t, cur);
  }
}

// Exchanges (LDS round trips) of one length-N transform.
template <int N, int RMAX>
constexpr int fft_exchanges() {
  return Plan<N, RMAX>::NSTAGE - 1;
}

// Length-N transform of one signal held in pattern A by a team of Plan::TPF
// threads; every thread of the block must call it (it contains barriers).
// X0 numbers its first exchange within a chain of transforms.  With two
// buffers the first write is not preceded by a barrier: the caller either
// starts a chain behind one, or continues a chain (X0 = exchanges so far),
// in which case the buffer it writes was last read before the barrier of
// the previous exchange.
template <int DIR, typename T, int N, int RMAX, bool DB = false, int X0 = 0>
__device__ __forceinline__ void fft(cx<T> (&v)[RMAX], T* xb, int t, gptr<const cx<T>> tw) {
  // An opaque copy of the table pointer behind a compiler memory barrier:
  // twiddle loads cannot be hoisted out of the transform and held live
  // across unrelated work.
  gptr<const cx<T>> twp = tw;
  asm volatile("" : "+s"(twp) : : "memory");
  StageSeeds<DIR, T, N, RMAX, 0> none;   // stage 0 has no twiddles
  fft_stages<DIR, T, N, RMAX, 0, DB, X0>(v, xb, t, twp, none);
}

// Three transforms in a chain (one barrier in front when double-buffered).
template <int DIR, typename T, int N, int RMAX, bool DB>
__device__ __forceinline__ void fft3(cx<T> (&a)[RMAX], cx<T> (&b)[RMAX], cx<T> (&c)[RMAX], T* xb,
                                     int t, gptr<const cx<T>> tw) {
  constexpr int E = fft_exchanges<N, RMAX>();
  if constexpr (DB) __syncthreads();
  fft<DIR, T, N, RMAX, DB, 0>(a, xb, t, tw);
  fft<DIR, T, N, RMAX, DB, E>(b, xb, t, tw);
  fft<DIR, T, N, RMAX, DB, 2 * E>(c, xb, t, tw);
}

}  // namespace pm
