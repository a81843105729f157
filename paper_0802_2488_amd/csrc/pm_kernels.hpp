// HIP kernels of the discrete-Green augmented-Lagrangian FFT solver (gfx950).
//
// Per iteration the device runs
//   column pass : column FFT of the row spectra of tau, discrete Green tensor
//                 of eq. 3 applied per momentum (q = 0 carries E), inverse
//                 column FFT                                   (k_column)
//   row pass    : per row pair, inverse real FFT -> compatible strain e,
//                 pointwise augmented-Lagrangian step (Hencky-Mises law,
//                 voids stress free), new polarisation tau, forward real FFT
//                 back into the row spectra; FP64 partial sums   (k_row)
//   reductions  : fixed-order FP64 sums, convergence indicators, and the
//                 equilibrium residual, with the divergence that belongs to
//                 the Green tensor in use (backward differences of eq. 1,
//                 forward ones along a DG2 variant's flipped directions, the
//                 continuum form for CG1), when the other two indicators
//                 already pass                  (k_reduce*, k_div, k_div_continuum)
// The persistent state is the stress of the last iterate ((11, 22, 33, 12)
// of each pixel side by side), which is also the augmented-Lagrangian
// multiplier, and the half
// spectrum of the polarisation tau; the strain is recovered from both when
// outputs are written.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "pm_fft.hpp"
#include "pm_internal.h"

// Tuning knobs (compile-time; the defaults are the measured best on MI355X).
#ifndef PM_ROW_R32
#define PM_ROW_R32 16         // row-pass radix, FP32
#endif
#ifndef PM_ROW_R64
#define PM_ROW_R64 4          // row-pass radix, FP64
#endif
#ifndef PM_ROW_TPF_MAX
#define PM_ROW_TPF_MAX 512    // most threads per row-pass transform
#endif
#ifndef PM_ROW_WPE
#define PM_ROW_WPE 2          // minimum waves per SIMD requested for the row pass
#endif
#ifndef PM_ROW_PREFETCH
#define PM_ROW_PREFETCH 2     // pixel pairs of stress fetched ahead in the FP32 row pass
#endif
#ifndef PM_ROW_PREFETCH64
#define PM_ROW_PREFETCH64 1   // the same for FP64 (twice the registers per pair)
#endif
#ifndef PM_STAGE_INFLIGHT
#define PM_STAGE_INFLIGHT 6   // 16-byte loads per thread in flight while staging a row
#endif
#ifndef PM_COL_R32
#define PM_COL_R32 16         // column-pass radix, FP32, L >= 2048
#endif
#ifndef PM_COL_R64
#define PM_COL_R64 8          // column-pass radix, FP64, L >= 2048
#endif
#ifndef PM_COL_W32
#define PM_COL_W32 2          // columns per block (= spectrum tile width), FP32, long columns
#endif
#ifndef PM_COL_CB32
#define PM_COL_CB32 2         // columns per block, FP32, columns of 256 threads
#endif
#ifndef PM_COL_LDS_SKEW
#define PM_COL_LDS_SKEW 16    // words between the FFT buffers of a block's columns, beyond their size
#endif
#ifndef PM_COL_PAIRV
#define PM_COL_PAIRV 1   // 16-byte accesses for FP32 column pairs
#endif
#ifndef PM_LDS_DB
#define PM_LDS_DB 1   // double-buffered FFT exchanges where the LDS share allows
#endif
#ifndef PM_COL_WPE
#define PM_COL_WPE 2
#endif

namespace pm {

// ---------------------------------------------------------------------------
// Material constants in the field precision.
template <typename T>
struct Mat {
  T mu, lam, Y, mu0, lam0, K, K0;
  T sy;        // sqrt(2/3) Y: Frobenius norm of the capped stress deviator
  T cel;       // mu / (mu + mu0): deviator ratio s / dev R on the elastic branch
  T inv2mu0, inv3KK0, inv3K, inv2lm0;
};

template <typename T>
__device__ __forceinline__ Mat<T> make_mat(const DevParams& p) {
  Mat<T> m;
  m.mu = (T)p.mu; m.lam = (T)p.lam; m.Y = (T)p.Y; m.mu0 = (T)p.mu0; m.lam0 = (T)p.lam0;
  m.K = (T)p.K; m.K0 = (T)p.K0; m.sy = (T)p.sy;
  m.cel = (T)(p.mu / (p.mu + p.mu0));
  m.inv2mu0 = (T)(1.0 / (2.0 * p.mu0));
  m.inv3KK0 = (T)(1.0 / (3.0 * (p.K + p.K0)));
  m.inv3K = (T)(1.0 / (3.0 * p.K));
  m.inv2lm0 = (T)(1.0 / (2.0 * (p.lam0 + p.mu0)));
  return m;
}

// The stored stress of a void is exactly zero; its 33 component is kept as
// a negative zero, which marks the pixel as a void for the iteration pass
// (so that pass does not read the mask).  Matrix pixels store their 33
// component plus +0, which turns a negative zero into a positive one and
// leaves every other value unchanged.
__device__ __forceinline__ bool void_flagged(float v) { return __float_as_uint(v) == 0x80000000u; }
__device__ __forceinline__ bool void_flagged(double v) {
  return (unsigned long long)__double_as_longlong(v) == 0x8000000000000000ull;
}
template <typename T>
__device__ __forceinline__ T flag33(T s33, bool is_void) {
  return is_void ? -(T)0 : s33 + (T)0;
}

// 1 / x: the hardware estimate in FP32 (1 ulp; det of a positive definite
// acoustic tensor, never 0, inf or denormal), correctly rounded in FP64.
#ifndef PM_PRECISE_F32
#define PM_PRECISE_F32 0      // 1: correctly rounded FP32 division and square root
#endif
__device__ __forceinline__ float recip(float x) { return PM_PRECISE_F32 ? 1.0f / x : __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

// 1 / sqrt(x): the hardware estimate in FP32 (~1 ulp), exact in FP64.
__device__ __forceinline__ float rsq(float x) { return PM_PRECISE_F32 ? 1.0f / __fsqrt_rn(x) : rsqrtf(x); }
__device__ __forceinline__ double rsq(double x) { return 1.0 / sqrt(x); }

// Hencky-Mises stress of a matrix pixel; eps = (11, 22, 33, 12).  The
// deviator is 2 mu dev(eps) capped at Frobenius norm sqrt(2/3) Y:
// s = min(2 mu, sqrt(2/3) Y / |dev eps|) dev eps.  Returns the plastic flag
// (strictly beyond the cap).
template <typename T>
__device__ __forceinline__ bool hencky(const T* e, T* s, const Mat<T>& m) {
  const T t3 = (e[0] + e[1] + e[2]) * (T)(1.0 / 3.0);
  const T d0 = e[0] - t3, d1 = e[1] - t3, d2 = e[2] - t3, d3 = e[3];
  const T cap = m.sy * rsq(d0 * d0 + d1 * d1 + d2 * d2 + (T)2 * d3 * d3);
  const T tm = (T)2 * m.mu;
  const bool plastic = cap < tm;
  const T sc = plastic ? cap : tm;
  const T pr = (T)3 * m.K * t3;
  s[0] = pr + sc * d0; s[1] = pr + sc * d1; s[2] = pr + sc * d2; s[3] = sc * d3;
  return plastic;
}

// Plastic phase of the output (Sec. 3: the matrix pixels where the Mises
// stress equals Y), read from the stored stress: |dev sigma|^2 within a few
// rounding units of (2/3) Y^2.  A capped stress has Mises norm Y up to
// rounding; an elastic one has Mises norm Y plus the trial margin (negative),
// so this agrees with the pointwise step's branch except for elastic pixels
// within PLASTIC_TOL Y of yield.  Recovering the strain first and testing it
// instead loses accuracy when the reference medium is soft (the strain is
// (sigma - tau) / C0 up to the trace term).
template <typename T>
struct PlasticTol;
template <>
struct PlasticTol<float> {
  static constexpr float value = 4e-6f;
};
template <>
struct PlasticTol<double> {
  static constexpr double value = 1e-12;
};
template <typename T>
__device__ __forceinline__ bool at_yield(const T* sg, const Mat<T>& m) {
  const T t3 = (sg[0] + sg[1] + sg[2]) * (T)(1.0 / 3.0);
  const T d0 = sg[0] - t3, d1 = sg[1] - t3, d2 = sg[2] - t3, d3 = sg[3];
  const T n2 = d0 * d0 + d1 * d1 + d2 * d2 + (T)2 * d3 * d3;
  return n2 > m.sy * m.sy * ((T)1 - (T)2 * PlasticTol<T>::value);
}

// Pointwise step of one pixel: solve S(eps) + C0:eps = R with
// R = lambda + C0:e, where lambda (the multiplier, equal to the stress of the
// previous iterate) is the stored state and e = (e11, e22, e12), e33 = 0.
// Volumetric part: tr eps = tr R / (3 (K + K0)).  Deviatoric part with
// r = dev R: s = c r, c = min(mu / (mu + mu0), sqrt(2/3) Y / |r|) (the elastic
// and the capped branch in one formula), dev eps = (r - s) / (2 mu0).
// Voids carry no stress: eps = e (in plane), eps33 = 0.
// Outputs the new stress (the next multiplier), eps and tau = sigma - C0:eps;
// returns whether the pixel is on the capped (plastic) branch.
template <typename T>
__device__ __forceinline__ bool alm_point(const T* e, const T* la, bool is_void, const Mat<T>& m, T* en, T* sg,
                                          T* tau) {
  if (is_void) {
    en[0] = e[0]; en[1] = e[1]; en[2] = (T)0; en[3] = e[2];
    sg[0] = sg[1] = sg[2] = sg[3] = (T)0;
    const T tr = m.lam0 * (e[0] + e[1]);
    tau[0] = -(tr + (T)2 * m.mu0 * e[0]);
    tau[1] = -(tr + (T)2 * m.mu0 * e[1]);
    tau[2] = -((T)2 * m.mu0 * e[2]);
    return false;
  }
  const T tre = m.lam0 * (e[0] + e[1]);
  const T R0 = la[0] + tre + (T)2 * m.mu0 * e[0];
  const T R1 = la[1] + tre + (T)2 * m.mu0 * e[1];
  const T R2 = la[2] + tre;
  const T R3 = la[3] + (T)2 * m.mu0 * e[2];
  const T trR3 = (R0 + R1 + R2) * (T)(1.0 / 3.0);
  const T r0 = R0 - trR3, r1 = R1 - trR3, r2 = R2 - trR3, r3 = R3;
  const T cap = m.sy * rsq(r0 * r0 + r1 * r1 + r2 * r2 + (T)2 * r3 * r3);
  const T c = cap < m.cel ? cap : m.cel;
  const T s0 = c * r0, s1 = c * r1, s2 = c * r2, s3 = c * r3;
  const T tr_eps = (T)3 * trR3 * m.inv3KK0;
  const T t3 = tr_eps * (T)(1.0 / 3.0);
  en[0] = (r0 - s0) * m.inv2mu0 + t3;
  en[1] = (r1 - s1) * m.inv2mu0 + t3;
  en[2] = (r2 - s2) * m.inv2mu0 + t3;
  en[3] = (r3 - s3) * m.inv2mu0;
  const T pr = m.K * tr_eps;
  sg[0] = pr + s0; sg[1] = pr + s1; sg[2] = pr + s2; sg[3] = s3;
  const T c0t = m.lam0 * tr_eps;
  tau[0] = sg[0] - (c0t + (T)2 * m.mu0 * en[0]);
  tau[1] = sg[1] - (c0t + (T)2 * m.mu0 * en[1]);
  tau[2] = sg[3] - (T)2 * m.mu0 * en[3];
  return cap < m.cel;
}

// Strain from the stored stress and the polarisation tau = sigma - C0:eps of
// the same iterate.  Matrix: tr eps = tr sigma / (3K); in plane
// eps_ab = (sigma_ab - tau_ab - lambda0 tr eps delta_ab) / (2 mu0);
// eps33 = tr eps - eps11 - eps22.  Voids (sigma = 0, eps = e, eps33 = 0):
// tr = -(tau11 + tau22) / (2 (lambda0 + mu0)), eps_ab = -(tau_ab + lambda0
// tr delta_ab) / (2 mu0).
template <typename T>
__device__ __forceinline__ void strain_from(const T* sg, const T* tau, bool is_void, const Mat<T>& m, T* en) {
  if (is_void) {
    const T tr = -(tau[0] + tau[1]) * m.inv2lm0;
    en[0] = -(tau[0] + m.lam0 * tr) * m.inv2mu0;
    en[1] = -(tau[1] + m.lam0 * tr) * m.inv2mu0;
    en[2] = (T)0;
    en[3] = -tau[2] * m.inv2mu0;
    return;
  }
  const T tr = (sg[0] + sg[1] + sg[2]) * m.inv3K;
  en[0] = (sg[0] - tau[0] - m.lam0 * tr) * m.inv2mu0;
  en[1] = (sg[1] - tau[1] - m.lam0 * tr) * m.inv2mu0;
  en[3] = (sg[3] - tau[2]) * m.inv2mu0;
  en[2] = tr - en[0] - en[1];
}

// ---------------------------------------------------------------------------
// Block reduction of NV doubles in a fixed order (wave shuffles, then LDS).
template <int NV, typename P>
__device__ __forceinline__ void block_reduce_store(double (&v)[NV], P out) {
  __shared__ double red[16][NV];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nwave = (blockDim.x + 63) >> 6;
  // lanes beyond the end of a partial last wave contribute nothing
  const int active = min(64, (int)blockDim.x - wave * 64);
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double x = v[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double y = __shfl_xor(x, off, 64);
      if ((lane ^ off) < active) x += y;
    }
    v[i] = x;
  }
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) red[wave][i] = v[i];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < NV; i += blockDim.x) {
    double s = 0.0;
    for (int w = 0; w < nwave; ++w) s += red[w][i];
    out[i] = s;
  }
}

// ---------------------------------------------------------------------------
// Half-spectrum layout.  Row transforms of real rows have real bins m1 = 0
// and m1 = L/2; the Nyquist value is stored in the imaginary slot of bin 0,
// so a row holds exactly L/2 complex bins per component.  Columns are tiled
// WT at a time so a column block's data is one contiguous run:
//   index(m1, m2, c) = (((m1 / WT) * L + m2) * WT + m1 % WT) * 3 + c.
template <int L, int WT>
__device__ __forceinline__ unsigned sidx(int m1, int m2) {
  return ((unsigned)((m1 / WT) * L + m2) * WT + (unsigned)(m1 % WT)) * 3u;
}

__device__ __forceinline__ int xcd_remap(int b, int nb) {
  // Blocks are dispatched round-robin over the 8 XCDs; give each XCD a
  // contiguous range of logical work items so neighbours, which share cache
  // lines, meet in the same L2 at about the same time.
  const int x = b & 7, q = nb >> 3, r = nb & 7;
  return x * q + (x < r ? x : r) + (b >> 3);
}

// Blocks of `waves` waves that share a CU when each SIMD holds WPE waves,
// and the LDS bytes each of them may take.
constexpr int blocks_per_cu(int waves, int wpe) {
  const int cu = 4 * wpe > waves ? 4 * wpe : waves;
  return cu / waves > 1 ? cu / waves : 1;
}
constexpr size_t lds_budget(int waves, int wpe) {
  return (size_t)160 * 1024 / blocks_per_cu(waves, wpe) - 2048;
}
constexpr size_t zmax(size_t a, size_t b) { return a > b ? a : b; }
// Two exchange buffers stay within about one 64 KiB LDS immediate-offset
// range of one base register; beyond it every access needs its own address
// register and the kernels spill.
template <typename T, int L>
constexpr bool lds_db_near() {
  return (size_t)3 * LdsSize<L>::value * sizeof(T) < 65536;
}

// LDS of one row-pass block.  One region serves in turn as the stage of one
// row of each team's pair (HBM <-> LDS copies in 16-byte units), as the FFT
// exchange buffers and as the per-thread sums of the pointwise step; the
// phases are separated by block barriers.  Rows are staged, and the
// exchanges double-buffered, when the region still fits the LDS share of a
// block at the CU's expected number of blocks.
template <typename T, int L, int TEAMS, int TPF>
struct RowLds {
  static constexpr size_t budget = lds_budget((TEAMS * TPF + 63) / 64, PM_ROW_WPE);
  static constexpr size_t stage = (size_t)TEAMS * (L / 2) * 3 * sizeof(cx<T>);
  static constexpr size_t fftb = (size_t)TEAMS * 2 * LdsSize<L>::value * sizeof(T);   // one buffer per team
  static constexpr size_t sums = (size_t)NSUM * TEAMS * TPF * sizeof(double);   // FP64 per-thread sums
  static constexpr bool staged = zmax(stage, zmax(fftb, sums)) <= budget;
  // FP64 row passes take two buffers wherever they fit (no spills at the
  // sizes where they do: L = 4096 at 228 VGPRs); FP32 ones only within the
  // offset range (L = 8192 spills otherwise)
  static constexpr bool db = PM_LDS_DB && (sizeof(T) == 8 || lds_db_near<T, L>()) &&
                             zmax(staged ? stage : 0, zmax(2 * fftb, sums)) <= budget;
  static constexpr int team_words = (db ? 4 : 2) * LdsSize<L>::value;   // FFT buffers of one team
  static constexpr size_t bytes = zmax(staged ? stage : 0, zmax(db ? 2 * fftb : fftb, sums));
};

// LDS of one column-pass block: the FFT buffers of each of its CB columns,
// skewed by PM_COL_LDS_SKEW words; double-buffered when that fits.
template <typename T, int L, int CB, int TPF>
struct ColLds {
  static constexpr size_t budget = lds_budget((CB * TPF + 63) / 64, PM_COL_WPE);
  static constexpr bool db = PM_LDS_DB && lds_db_near<T, L>() &&
                             (size_t)CB * (4 * LdsSize<L>::value + PM_COL_LDS_SKEW) * sizeof(T) <= budget;
  static constexpr int col_words = (db ? 4 : 2) * LdsSize<L>::value + PM_COL_LDS_SKEW;
  static constexpr size_t bytes = (size_t)CB * col_words * sizeof(T);
};

// A row pair's view of the half spectrum: bins m1 of rows (ra + r), r = 0, 1,
// at base + (m1 / WT) * TSTRIDE + r * WT * 3 + (m1 % WT) * 3 + c.  The same
// accessor addresses the spectrum in HBM (base at row ra, TSTRIDE = L WT 3)
// and a row pair's copy staged in LDS (TSTRIDE = 2 WT 3).
template <int WT, int TSTRIDE>
__device__ __forceinline__ unsigned pidx(int m1, int r, int c) {
  return (unsigned)(m1 / WT) * TSTRIDE + (unsigned)(r * WT * 3 + (m1 % WT) * 3 + c);
}

// Row-pass output: split the complex transform Z of x + i y into the half
// spectra X[m] = (Z[m] + conj Z[L-m]) / 2 and Y[m] = (Z[m] - conj Z[L-m]) / (2i),
// m < L/2, with the real Nyquist values packed into the imaginary slots of
// bin 0.  Thread t gets bins m = t + TPF k, k < RMAX / 2.
template <typename T, int L, int RMAX>
__device__ __forceinline__ void split_regs(const cx<T> (&z)[RMAX], cx<T>* lz, int t, cx<T> (&X)[RMAX / 2],
                                           cx<T> (&Y)[RMAX / 2]) {
  constexpr int TPF = L / RMAX;
  __syncthreads();
#pragma unroll
  for (int s = 0; s < RMAX; ++s) lz[lpad(t + TPF * s)] = z[s];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < RMAX / 2; ++k) {
    const int mm = t + TPF * k;
    const cx<T> zm = lz[lpad(mm)];
    const cx<T> zr = cconj(lz[lpad((L - mm) & (L - 1))]);   // conj Z[L - m]
    const cx<T> d = zm - zr;
    X[k] = cscale(zm + zr, (T)0.5);
    Y[k] = {d.im * (T)0.5, -d.re * (T)0.5};
    if (mm == 0) {
      const cx<T> zh = lz[lpad(L / 2)];
      X[k].im = zh.re;   // Re Z[L/2]: Nyquist bin of x
      Y[k].im = zh.im;   // Im Z[L/2]: Nyquist bin of y
    }
  }
}

// Components 0, 1, 2 of row r of the pair at bins t + TPF k, k < H.
template <typename T, int L, int H, int WT, int TSTRIDE, typename P>
__device__ __forceinline__ void put_row(P base, int t, int r, const cx<T> (&c0)[H],
                                        const cx<T> (&c1)[H], const cx<T> (&c2)[H]) {
  constexpr int TPF = L / (2 * H);
#pragma unroll
  for (int k = 0; k < H; ++k) {
    const int mm = t + TPF * k;
    stc(base + pidx<WT, TSTRIDE>(mm, r, 0), c0[k]);
    stc(base + pidx<WT, TSTRIDE>(mm, r, 1), c1[k]);
    stc(base + pidx<WT, TSTRIDE>(mm, r, 2), c2[k]);
  }
}

// Hermitian extension of a packed row spectrum at bin m in [0, L).
template <typename T, int L, int WT, int TSTRIDE, typename P>
__device__ __forceinline__ cx<T> load_bin(P base, int m, int r, int c) {
  if (m == 0) return {ldc(base + pidx<WT, TSTRIDE>(0, r, c)).re, (T)0};
  if (m == L / 2) return {ldc(base + pidx<WT, TSTRIDE>(0, r, c)).im, (T)0};
  if (m < L / 2) return ldc(base + pidx<WT, TSTRIDE>(m, r, c));
  return cconj(ldc(base + pidx<WT, TSTRIDE>(L - m, r, c)));
}

// An opaque copy of an index: addresses derived from it in one phase of a
// kernel are recomputed in the next instead of being held in registers
// across the phases in between.
__device__ __forceinline__ int opaque(int v) {
  asm volatile("" : "+v"(v));
  return v;
}

// Largest divisor of n that is at most cap.
constexpr int divisor_upto(int n, int cap) {
  int d = cap < n ? cap : n;
  while (n % d != 0) --d;
  return d;
}

// A row pair's slice of the half spectrum in 16-byte units: in tile j each
// row holds WT 3 contiguous complex values (UPT units) and row b follows row
// a.  Unit u of row a sits at unit gidx(u) from the pair's base and the same
// unit of row b UPT units further; the LDS stage keeps one row in tile order.
template <typename T, int L, int WT, int TPF>
struct RowUnits {
  using u4 = unsigned __attribute__((ext_vector_type(4)));
  static constexpr int CPT = WT * 3;                           // complex values per tile and row
  static constexpr int UPT = CPT * (int)sizeof(cx<T>) / 16;    // 16-byte units per tile and row
  static constexpr int NU = (L / 2 / WT) * UPT;
  static constexpr int PER = NU / TPF;                         // units per thread and row
  static_assert((CPT * sizeof(cx<T>)) % 16 == 0, "a tile row must be a whole number of 16-byte units");
  static_assert(NU % TPF == 0, "the copy must split evenly over the team");
  static __device__ __forceinline__ unsigned gidx(int u) {
    const int j = u / UPT, k = u - j * UPT;
    return (unsigned)j * (L * WT * 3 * (int)sizeof(cx<T>) / 16) + k;
  }
};

// Both rows of a pair from HBM: row a into the LDS stage, row b into
// registers.  The two rows of a tile are adjacent, so loading them together
// brings each cache line in once.
template <typename T, int L, int WT, int TPF>
__device__ __forceinline__ void stage_pair_in(gptr<cx<T>> __restrict__ g, cx<T>* __restrict__ st, int t,
                                              typename RowUnits<T, L, WT, TPF>::u4 (&hold)[RowUnits<T, L, WT, TPF>::PER]) {
  using R = RowUnits<T, L, WT, TPF>;
  using u4 = typename R::u4;
  gptr<const u4> __restrict__ gs = (gptr<const u4>)g;
  u4* __restrict__ ls = reinterpret_cast<u4*>(st);
  constexpr int G = divisor_upto(R::PER, PM_STAGE_INFLIGHT);
#pragma unroll
  for (int i0 = 0; i0 < R::PER; i0 += G) {
    u4 buf[G];
#pragma unroll
    for (int i = 0; i < G; ++i) {
      const unsigned gi = R::gidx(t + (i0 + i) * TPF);
      buf[i] = gs[gi];
      hold[i0 + i] = gs[gi + R::UPT];
    }
#pragma unroll
    for (int i = 0; i < G; ++i) ls[t + (i0 + i) * TPF] = buf[i];
  }
}

// Row b, held in registers, into the LDS stage.
template <typename T, int L, int WT, int TPF>
__device__ __forceinline__ void hold_to_stage(cx<T>* __restrict__ st, int t,
                                              const typename RowUnits<T, L, WT, TPF>::u4 (&hold)[RowUnits<T, L, WT, TPF>::PER]) {
  using R = RowUnits<T, L, WT, TPF>;
  using u4 = typename R::u4;
  u4* __restrict__ ls = reinterpret_cast<u4*>(st);
#pragma unroll
  for (int i = 0; i < R::PER; ++i) ls[t + i * TPF] = hold[i];
}

// Row a, staged in LDS, into registers.
template <typename T, int L, int WT, int TPF>
__device__ __forceinline__ void stage_to_hold(const cx<T>* __restrict__ st, int t,
                                              typename RowUnits<T, L, WT, TPF>::u4 (&hold)[RowUnits<T, L, WT, TPF>::PER]) {
  using R = RowUnits<T, L, WT, TPF>;
  using u4 = typename R::u4;
  const u4* __restrict__ ls = reinterpret_cast<const u4*>(st);
#pragma unroll
  for (int i = 0; i < R::PER; ++i) hold[i] = ls[t + i * TPF];
}

// Both rows of a pair to HBM: row a from registers, row b from the LDS stage,
// so each cache line is written whole at once.
template <typename T, int L, int WT, int TPF>
__device__ __forceinline__ void stage_pair_out(gptr<cx<T>> __restrict__ g, const cx<T>* __restrict__ st, int t,
                                               const typename RowUnits<T, L, WT, TPF>::u4 (&hold)[RowUnits<T, L, WT, TPF>::PER]) {
  using R = RowUnits<T, L, WT, TPF>;
  using u4 = typename R::u4;
  gptr<u4> __restrict__ gd = (gptr<u4>)g;
  const u4* __restrict__ ls = reinterpret_cast<const u4*>(st);
#pragma unroll
  for (int i = 0; i < R::PER; ++i) {
    const int u = t + i * TPF;
    const unsigned gi = R::gidx(u);
    gd[gi] = hold[i];
    gd[gi + R::UPT] = ls[u];
  }
}

// ---------------------------------------------------------------------------
// Row pass.  A team of TPF = L / RMAX threads owns rows a = 2p and b = 2p + 1
// and three complex length-L signals: Za = 11a + i 22a, Zb = 11b + i 22b,
// Zc = 12a + i 12b (two real rows per complex transform).  Modes:
//   ROW_ITER  inverse row FFT -> e; pointwise step on the stored stress;
//             new stress stored; tau forward-transformed back
//   ROW_INIT  stress S(E) (0 on voids) stored; tau = sigma - C0:E transformed
//   ROW_EMIT  inverse row FFT of the stored tau; strain recovered from the
//             stress and tau; per-step outputs and sums of the strain
//   ROW_FWD / ROW_INV  plain row transforms of three real planes (checks)
//   ROW_SIGFWD forward row transform of the stored stress (11, 22, 12) into
//             x.spec_alt (the continuum equilibrium indicator of CG1)
template <typename T, int L, int RMAX, int TEAMS, int WT, int MODE, bool NTS>
__global__ void __launch_bounds__(TEAMS*(L / RMAX)) __attribute__((amdgpu_waves_per_eu(PM_ROW_WPE)))
k_row(const Slot<T>* __restrict__ slots, Extra<T> x) {
  constexpr int TPF = L / RMAX;
  constexpr int BS = TEAMS * TPF;
  constexpr int LS = LdsSize<L>::value;
  constexpr int LOAD_GROUP = RMAX >= 4 ? 4 : RMAX;   // unrolled iterations whose loads may be in flight together
  constexpr bool LOADS_SPEC = MODE == ROW_ITER || MODE == ROW_INV || MODE == ROW_EMIT;
  constexpr bool POINTWISE = MODE == ROW_ITER || MODE == ROW_INIT;
  using RL = RowLds<T, L, TEAMS, TPF>;
  constexpr bool STAGED = RL::staged;
  constexpr bool DB = RL::db;
  constexpr int GSTRIDE = L * WT * 3, SSTRIDE = WT * 3;
  constexpr int BPS = (L / 2) / TEAMS;                 // blocks per slot
  const Slot<T>& S = slots[blockIdx.x / BPS];
  if (gated_out(x, S.st)) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int team = threadIdx.x / TPF;
  const int t = threadIdx.x % TPF;
  // one LDS region, used in turn as row stage, FFT buffers and sums
  T* lre = reinterpret_cast<T*>(smem_raw) + team * RL::team_words;
  cx<T>* stg = reinterpret_cast<cx<T>*>(smem_raw) + team * (L / 2) * 3;
  const int p = xcd_remap(blockIdx.x % BPS, BPS) * TEAMS + team;
  const int ra = 2 * p, rb = 2 * p + 1;
  gptr<cx<T>> __restrict__ gbase =
      glb(MODE == ROW_SIGFWD ? x.spec_alt : S.spec) + (size_t)ra * WT * 3;
  gptr<const cx<T>> __restrict__ tw = glb(S.tw);
  gptr<const uint8_t> __restrict__ mask = glb(S.mask);
  // the stress state: (11, 22, 33, 12) of a pixel side by side, one vector.
  // The iteration streams it in and out once per pass.  NTS (set by the host
  // when the states iterated together exceed half the 256 MB Infinity Cache)
  // gives those loads and stores the non-temporal hint (measured: the FP32
  // row pass 8 % faster at L = 4096, 4 % at 8192, the 256-realization batch
  // 5 %); smaller states keep the default policy, which leaves them in the
  // cache for the next pass (there the hint cost 7 % at L = 1024 and 2048
  // FP32, 15-18 % in FP64).  The spectrum always keeps the default policy:
  // adjacent row pairs share its cache lines, and the column pass reads it
  // back from the Infinity Cache where it fits.
  using v4 = T __attribute__((ext_vector_type(4)));
  gptr<v4> __restrict__ sig = (gptr<v4>)glb(S.sig);
  static_assert(!NTS || MODE == ROW_ITER, "the non-temporal state policy belongs to the iteration");
  const Mat<T> m = make_mat<T>(S.prm);
  constexpr unsigned NPX = (unsigned)L * L;

  cx<T> za[RMAX], zb[RMAX], zc[RMAX];

  // Stress and mask of the thread's pixel pairs, fetched PF pairs ahead of
  // the pointwise step; the first PF pairs are issued before the inverse
  // transforms so they arrive while those run.
  constexpr int PF_WANT = sizeof(T) == 4 ? PM_ROW_PREFETCH : PM_ROW_PREFETCH64;
  constexpr int PF = PF_WANT < RMAX ? PF_WANT : RMAX;
  T so[RMAX][2][4];
  uint8_t mk[RMAX][2];
  auto fetch = [&](int s, int tt) {
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const unsigned ix = (unsigned)(half ? rb : ra) * L + tt + TPF * s;
      if constexpr (MODE != ROW_ITER) mk[s][half] = mask[ix];
      if constexpr (MODE == ROW_ITER) {
        v4 q;
        if constexpr (NTS) q = __builtin_nontemporal_load(sig + ix);
        else q = sig[ix];
        so[s][half][0] = q.x; so[s][half][1] = q.y; so[s][half][2] = q.z; so[s][half][3] = q.w;
      }
    }
  };
  if constexpr (POINTWISE) {
#pragma unroll
    for (int s = 0; s < PF; ++s) fetch(s, t);
  }

  if constexpr (LOADS_SPEC) {
    auto build = [&](auto base, auto tstride) {
      constexpr int TS = decltype(tstride)::value;
#pragma unroll
      for (int s = 0; s < RMAX; ++s) {
        const int mm = t + TPF * s;
        const cx<T> a0 = load_bin<T, L, WT, TS>(base, mm, 0, 0), a1 = load_bin<T, L, WT, TS>(base, mm, 0, 1);
        const cx<T> a2 = load_bin<T, L, WT, TS>(base, mm, 0, 2);
        const cx<T> b0 = load_bin<T, L, WT, TS>(base, mm, 1, 0), b1 = load_bin<T, L, WT, TS>(base, mm, 1, 1);
        const cx<T> b2 = load_bin<T, L, WT, TS>(base, mm, 1, 2);
        za[s] = {a0.re - a1.im, a0.im + a1.re};
        zb[s] = {b0.re - b1.im, b0.im + b1.re};
        zc[s] = {a2.re - b2.im, a2.im + b2.re};
        if ((s & (LOAD_GROUP - 1)) == LOAD_GROUP - 1) __builtin_amdgcn_sched_barrier(0);
      }
    };
    if constexpr (STAGED) {
      // row a: Za = 11a + i 22a and the 12a part of Zc; row b waits in registers
      typename RowUnits<T, L, WT, TPF>::u4 hold[RowUnits<T, L, WT, TPF>::PER];
      stage_pair_in<T, L, WT, TPF>(gbase, stg, t, hold);
      __syncthreads();
#pragma unroll
      for (int s = 0; s < RMAX; ++s) {
        const int mm = t + TPF * s;
        const cx<T> a0 = load_bin<T, L, WT, SSTRIDE>(stg, mm, 0, 0), a1 = load_bin<T, L, WT, SSTRIDE>(stg, mm, 0, 1);
        za[s] = {a0.re - a1.im, a0.im + a1.re};
        zc[s] = load_bin<T, L, WT, SSTRIDE>(stg, mm, 0, 2);
      }
      __syncthreads();
      // row b: Zb = 11b + i 22b, and Zc = 12a + i 12b
      hold_to_stage<T, L, WT, TPF>(stg, t, hold);
      __syncthreads();
#pragma unroll
      for (int s = 0; s < RMAX; ++s) {
        const int mm = t + TPF * s;
        const cx<T> b0 = load_bin<T, L, WT, SSTRIDE>(stg, mm, 0, 0), b1 = load_bin<T, L, WT, SSTRIDE>(stg, mm, 0, 1);
        const cx<T> b2 = load_bin<T, L, WT, SSTRIDE>(stg, mm, 0, 2);
        zb[s] = {b0.re - b1.im, b0.im + b1.re};
        zc[s] = {zc[s].re - b2.im, zc[s].im + b2.re};
      }
    } else {
      build(gbase, std::integral_constant<int, GSTRIDE>{});
    }
    fence(za); fence(zb); fence(zc);
    fft3<+1, T, L, RMAX, DB>(za, zb, zc, lre, opaque(t), tw);
    fence(za); fence(zb); fence(zc);
  }

  if constexpr (MODE == ROW_INV) {
    gptr<T> __restrict__ out = glb(x.real_out);
#pragma unroll
    for (int s = 0; s < RMAX; ++s) {
      const int x1 = t + TPF * s;
      const unsigned ia = (unsigned)ra * L + x1, ib = (unsigned)rb * L + x1;
      out[ia] = za[s].re; out[NPX + ia] = za[s].im; out[2 * NPX + ia] = zc[s].re;
      out[ib] = zb[s].re; out[NPX + ib] = zb[s].im; out[2 * NPX + ib] = zc[s].im;
    }
    return;
  }

  if constexpr (MODE == ROW_EMIT) {
    // the stored row spectra hold the forward row transforms of tau
    const T invL = (T)(1.0 / L);
    gptr<T> __restrict__ sig_out = glb(x.sig_out);
    gptr<T> __restrict__ eps_out = glb(x.eps_out);
    gptr<uint8_t> __restrict__ pl_out = glb(x.plastic_out);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < RMAX; ++s) {
      const int x1 = t + TPF * s;
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        const unsigned ix = (unsigned)(half ? rb : ra) * L + x1;
        const bool isv = mask[ix] != 0;
        T tau[3];
        if (half == 0) { tau[0] = za[s].re * invL; tau[1] = za[s].im * invL; tau[2] = zc[s].re * invL; }
        else { tau[0] = zb[s].re * invL; tau[1] = zb[s].im * invL; tau[2] = zc[s].im * invL; }
        const v4 q = sig[ix];
        T sg[4] = {q.x, q.y, q.z, q.w};
        T en[4];
        strain_from(sg, tau, isv, m, en);
        const bool pl = !isv && at_yield(sg, m);
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] += (double)en[c];
        if (sig_out) {
#pragma unroll
          for (int c = 0; c < 4; ++c) sig_out[c * NPX + ix] = sg[c] + (T)0;   // the void flag's -0 as +0
        }
        if (eps_out) {
#pragma unroll
          for (int c = 0; c < 4; ++c) eps_out[c * NPX + ix] = en[c];
        }
        if (pl_out) pl_out[ix] = pl ? 1 : 0;
      }
    }
    block_reduce_store<4>(acc, glb(S.part2) + (size_t)(blockIdx.x % BPS) * 4);
    return;
  }

  if constexpr (MODE == ROW_SIGFWD) {
#pragma unroll
    for (int s = 0; s < RMAX; ++s) {
      const int x1 = t + TPF * s;
      const v4 a = sig[(unsigned)ra * L + x1], b = sig[(unsigned)rb * L + x1];
      za[s] = {a.x, a.y};
      zb[s] = {b.x, b.y};
      zc[s] = {a.w, b.w};
    }
  }

  if constexpr (MODE == ROW_FWD) {
    gptr<const T> __restrict__ in = glb(x.real_in);
#pragma unroll
    for (int s = 0; s < RMAX; ++s) {
      const int x1 = t + TPF * s;
      const unsigned ia = (unsigned)ra * L + x1, ib = (unsigned)rb * L + x1;
      za[s] = {in[ia], in[NPX + ia]};
      zb[s] = {in[ib], in[NPX + ib]};
      zc[s] = {in[2 * NPX + ia], in[2 * NPX + ib]};
    }
  }

  if constexpr (POINTWISE) {
    // Pointwise step per pixel.  Per-thread partial sums
    // (sigma 11, 22, 33, 12, |e - eps|^2 and the plastic count) are FP64
    // from the first pixel on, and kept in LDS rather than registers, which
    // keeps the kernel free of spills; block and global sums are FP64 too.
    double(*lacc)[BS] = reinterpret_cast<double(*)[BS]>(smem_raw);
    __syncthreads();   // the region may still be read by the last FFT stage or the row build
    // ROW_INIT: the load step's E from the slot state, or from the arguments
    T E0 = (T)x.E[0], E1 = (T)x.E[1], E2 = (T)x.E[2];
    if (x.use_state) {
      gptr<const DevState> st = glb(S.st);
      E0 = (T)st->E[0]; E1 = (T)st->E[1]; E2 = (T)st->E[2];
    }
#pragma unroll
    for (int i = 0; i < NSUM; ++i) lacc[i][threadIdx.x] = 0.0;
    const int tp = opaque(t);
#pragma unroll
    for (int s = 0; s < RMAX; ++s) {
      const int x1 = tp + TPF * s;
      if (s + PF < RMAX) fetch(s + PF, tp);
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        const unsigned ix = (unsigned)(half ? rb : ra) * L + x1;
        // iterations read the void flag from the state (a negative zero in
        // the 33 component, see void_flagged) instead of the mask
        bool isv;
        if constexpr (MODE == ROW_ITER) isv = void_flagged(so[s][half][2]);
        else isv = mk[s][half] != 0;
        T e[3], en[4], sg[4], tau[3];
        bool pl = false;
        if constexpr (MODE == ROW_INIT) {
          e[0] = E0; e[1] = E1; e[2] = E2;
          en[0] = E0; en[1] = E1; en[2] = (T)0; en[3] = E2;
          if (isv) {
            sg[0] = sg[1] = sg[2] = sg[3] = (T)0;
          } else {
            pl = hencky(en, sg, m);
          }
          const T c0t = m.lam0 * (E0 + E1);
          tau[0] = sg[0] - (c0t + (T)2 * m.mu0 * E0);
          tau[1] = sg[1] - (c0t + (T)2 * m.mu0 * E1);
          tau[2] = sg[3] - (T)2 * m.mu0 * E2;
        } else {
          if (half == 0) { e[0] = za[s].re; e[1] = za[s].im; e[2] = zc[s].re; }
          else { e[0] = zb[s].re; e[1] = zb[s].im; e[2] = zc[s].im; }
          pl = alm_point(e, so[s][half], isv, m, en, sg, tau);
        }
        const v4 snew = {sg[0], sg[1], flag33(sg[2], isv), sg[3]};
        if constexpr (NTS) __builtin_nontemporal_store(snew, sig + ix);
        else sig[ix] = snew;
        {
          const double c0 = (double)(e[0] - en[0]), c1 = (double)(e[1] - en[1]), c2 = (double)en[2],
                       c3 = (double)(e[2] - en[3]);
          const double v6[NSUM] = {(double)sg[0], (double)sg[1], (double)sg[2], (double)sg[3],
                                   c0 * c0 + c1 * c1 + c2 * c2 + 2.0 * c3 * c3, pl ? 1.0 : 0.0};
#pragma unroll
          for (int i = 0; i < NSUM; ++i) lacc[i][threadIdx.x] += v6[i];
        }
        if (half == 0) { za[s] = {tau[0], tau[1]}; zc[s].re = tau[2]; }
        else { zb[s] = {tau[0], tau[1]}; zc[s].im = tau[2]; }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    fence(za); fence(zb); fence(zc);
    double accd[NSUM];
#pragma unroll
    for (int i = 0; i < NSUM; ++i) accd[i] = lacc[i][threadIdx.x];
    block_reduce_store<NSUM>(accd, glb(S.part) + (size_t)(blockIdx.x % BPS) * NPART);
  }

  fft3<-1, T, L, RMAX, DB>(za, zb, zc, lre, opaque(t), tw);

  // Za -> (11, 22) of row a, Zb -> (11, 22) of row b, Zc -> 12 of rows a, b.
  constexpr int H = RMAX / 2;
  cx<T> xa[H], ya[H], xb[H], yb[H], xc[H], yc[H];
  const int ts = opaque(t);
  cx<T>* lz = reinterpret_cast<cx<T>*>(lre);
  split_regs<T, L, RMAX>(za, lz, ts, xa, ya);
  split_regs<T, L, RMAX>(zb, lz, ts, xb, yb);
  split_regs<T, L, RMAX>(zc, lz, ts, xc, yc);
  if constexpr (STAGED) {
    __syncthreads();
    put_row<T, L, H, WT, SSTRIDE>(stg, ts, 0, xa, ya, xc);
    __syncthreads();
    typename RowUnits<T, L, WT, TPF>::u4 hold[RowUnits<T, L, WT, TPF>::PER];
    stage_to_hold<T, L, WT, TPF>(stg, ts, hold);
    __syncthreads();
    put_row<T, L, H, WT, SSTRIDE>(stg, ts, 0, xb, yb, yc);
    __syncthreads();
    stage_pair_out<T, L, WT, TPF>(gbase, stg, opaque(t), hold);
  } else {
    put_row<T, L, H, WT, GSTRIDE>(gbase, ts, 0, xa, ya, xc);
    put_row<T, L, H, WT, GSTRIDE>(gbase, ts, 1, xb, yb, yc);
  }
}

// ---------------------------------------------------------------------------
// Column pass.
template <typename T>
__device__ __forceinline__ void green_apply(cx<T>* tt, cx<T> k1, cx<T> k2, const T lam0, const T mu0,
                                            const T scale) {
  // N = lam0 conj(k) (x) k + mu0 k (x) conj(k) + mu0 |k|^2 I; w_l = conj(k_k) tau_kl;
  // v = N^-1 w; e_ij = -(k_i v_j + k_j v_i) / 2.
  const T n1 = k1.re * k1.re + k1.im * k1.im;
  const T n2 = k2.re * k2.re + k2.im * k2.im;
  const T nk = n1 + n2;
  const T lm = lam0 + mu0;
  const T A = lm * n1 + mu0 * nk;
  const T D = lm * n2 + mu0 * nk;
  const cx<T> c12 = cmul(cconj(k1), k2);   // conj(k1) k2
  // b = lam0 conj(k1) k2 + mu0 k1 conj(k2) = lam0 c12 + mu0 conj(c12)
  const cx<T> b = {(lam0 + mu0) * c12.re, (lam0 - mu0) * c12.im};
  const T det = A * D - (b.re * b.re + b.im * b.im);
  const T idet = scale * recip(det);
  const cx<T> t11 = tt[0], t22 = tt[1], t12 = tt[2];
  const cx<T> k1c = cconj(k1), k2c = cconj(k2);
  const cx<T> w1 = cmul(k1c, t11) + cmul(k2c, t12);
  const cx<T> w2 = cmul(k1c, t12) + cmul(k2c, t22);
  const cx<T> v1 = cscale(cscale(w1, D) - cmul(b, w2), idet);
  const cx<T> v2 = cscale(cscale(w2, A) - cmul(cconj(b), w1), idet);
  const cx<T> e11 = cmul(k1, v1), e22 = cmul(k2, v2);
  const cx<T> e12 = cmul(k1, v2) + cmul(k2, v1);
  tt[0] = {-e11.re, -e11.im};
  tt[1] = {-e22.re, -e22.im};
  tt[2] = {(T)-0.5 * e12.re, (T)-0.5 * e12.im};
}

// Green tensor at momentum (m1, m2), or E at q = 0.
//   GK_SIGN: eq. 3 at (+-q1, +-q2) (the slot's flips; k(-q) = -conj k(q));
//   GK_DG1:  the symmetrised tensor {G(q1,q2) + G(-q1,-q2)
//            + (-1)^(i+j+k+l) [G(-q1,q2) + G(q1,-q2)]} / 4; the sign pattern
//            is applied as tau12 -> -tau12 before and e12 -> -e12 after;
//   GK_CG1:  the continuum operator -Gamma0(xi) at the bins' continuum
//            frequencies (real momenta); modes with a Nyquist component carry
//            no strain.
template <int GK, typename T>
__device__ __forceinline__ void green_at(cx<T>* tt, int m1, int m2, const Slot<T>& S, const Extra<T>& x,
                                         const T lam0, const T mu0, const T scale) {
  const int L = S.prm.L;
  if (m1 == 0 && m2 == 0) {
    double E0 = x.E[0], E1 = x.E[1], E2 = x.E[2];
    if (x.use_state) {
      gptr<const DevState> st = glb(S.st);
      E0 = st->E[0]; E1 = st->E[1]; E2 = st->E[2];
    }
    tt[0] = {(T)E0, (T)0};
    tt[1] = {(T)E1, (T)0};
    tt[2] = {(T)E2, (T)0};
    return;
  }
  if constexpr (GK == GK_CG1) {
    if (m1 == L / 2 || m2 == L / 2) {
      tt[0] = tt[1] = tt[2] = {(T)0, (T)0};
      return;
    }
    const double w = 6.283185307179586476925286766559 / (double)L;
    const cx<T> k1 = {(T)(w * (double)(m1 < L / 2 ? m1 : m1 - L)), (T)0};
    const cx<T> k2 = {(T)(w * (double)(m2 < L / 2 ? m2 : m2 - L)), (T)0};
    green_apply(tt, k1, k2, lam0, mu0, scale);
    return;
  }
  gptr<const cx<T>> ktab = glb(S.ktab);
  cx<T> k1 = ldc(ktab + m1), k2 = ldc(ktab + m2);
  if constexpr (GK == GK_DG1) {
    const cx<T> f1 = {-k1.re, k1.im}, f2 = {-k2.re, k2.im};   // k(-q) = -conj k(q)
    cx<T> acc[3], u[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) u[c] = tt[c];
    green_apply(u, k1, k2, lam0, mu0, scale);
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[c] = u[c];
#pragma unroll
    for (int c = 0; c < 3; ++c) u[c] = tt[c];
    green_apply(u, f1, f2, lam0, mu0, scale);
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[c] = acc[c] + u[c];
    u[0] = tt[0]; u[1] = tt[1]; u[2] = {-tt[2].re, -tt[2].im};
    green_apply(u, f1, k2, lam0, mu0, scale);
    acc[0] = acc[0] + u[0]; acc[1] = acc[1] + u[1]; acc[2] = acc[2] - u[2];
    u[0] = tt[0]; u[1] = tt[1]; u[2] = {-tt[2].re, -tt[2].im};
    green_apply(u, k1, f2, lam0, mu0, scale);
    acc[0] = acc[0] + u[0]; acc[1] = acc[1] + u[1]; acc[2] = acc[2] - u[2];
#pragma unroll
    for (int c = 0; c < 3; ++c) tt[c] = cscale(acc[c], (T)0.25);
    return;
  }
  if (S.flip1) k1 = {-k1.re, k1.im};   // k(-q) = -conj(k(q))
  if (S.flip2) k2 = {-k2.re, k2.im};
  green_apply(tt, k1, k2, lam0, mu0, scale);
}

// A team of TPF threads owns one column m1 of the packed row spectra; a
// block owns CB adjacent columns, with the column index fastest across
// lanes.  Columns are stored in tiles of W (contiguous in memory); CB divides
// W, or equals it.  Column 0 carries the real bins m1 = 0 (real part) and
// m1 = L/2 (imaginary part): its transform is split with conj-symmetry into
// the two real-signal spectra, each gets its own Green tensor, and the
// results are packed again before the inverse.
template <typename T, int L, int RMAX, int W, int CB, int MODE_GK>
__global__ void __launch_bounds__(CB*(L / RMAX)) __attribute__((amdgpu_waves_per_eu(PM_COL_WPE)))
k_column(const Slot<T>* __restrict__ slots, Extra<T> x) {
  constexpr int MODE = MODE_GK & 0xff;
  constexpr int GK = MODE_GK >> 8;
  static_assert(W % CB == 0, "columns per block must divide the tile width");
  constexpr int TPF = L / RMAX;
  constexpr int LS = LdsSize<L>::value;
  constexpr int BPS = (L / 2) / CB;                    // blocks per slot
  const Slot<T>& S = slots[blockIdx.x / BPS];
  if (gated_out(x, S.st)) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // The column index runs fastest across lanes, so a wave's loads cover
  // whole tile rows.  Neighbouring lanes then address two columns' FFT
  // buffers at the same index; the buffers are skewed by PM_COL_LDS_SKEW
  // words so those accesses fall in different banks.
  const int wb = threadIdx.x % CB;        // column within the block
  const int t = threadIdx.x / CB;
  using CL = ColLds<T, L, CB, TPF>;
  T* const lre = reinterpret_cast<T*>(smem_raw) + wb * CL::col_words;
  const int g = xcd_remap(blockIdx.x % BPS, BPS);
  const int m1 = g * CB + wb;
  const int w = m1 % W;                   // column within its tile
  const bool packed = (g == 0);           // block-uniform: block 0 holds column 0
  gptr<const cx<T>> __restrict__ tw = glb(S.tw);
  gptr<cx<T>> __restrict__ tile = glb(x.spec_alt ? x.spec_alt : S.spec) + (size_t)(m1 / W) * L * W * 3;
  gptr<cx<T>> __restrict__ xbuf = glb(S.xbuf);

  // FP32 tiles of two columns, one per lane of a pair: the pair's six
  // complex values of row m2 are 48 contiguous bytes.  Each lane moves its
  // own 16-byte end and the middle 16 bytes (read by both, written as two
  // 8-byte halves), two accesses per row instead of three 8-byte ones.
  constexpr bool PAIRV = PM_COL_PAIRV && sizeof(T) == 4 && W == 2 && CB == 2;
  using f4 = float __attribute__((ext_vector_type(4)));
  cx<T> v[3][RMAX];
#pragma unroll
  for (int s = 0; s < RMAX; ++s) {
    const int m2 = t + TPF * s;
    if constexpr (PAIRV) {
      gptr<const f4> row = (gptr<const f4>)(tile + (unsigned)m2 * 6u);
      const f4 a = row[w ? 2 : 0];
      const f4 b = row[1];
      v[0][s] = w ? cx<T>{b.z, b.w} : cx<T>{a.x, a.y};
      v[1][s] = w ? cx<T>{a.x, a.y} : cx<T>{a.z, a.w};
      v[2][s] = w ? cx<T>{a.z, a.w} : cx<T>{b.x, b.y};
      if ((s & 3) == 3) __builtin_amdgcn_sched_barrier(0);   // bounds the loads in flight
    } else {
      gptr<const cx<T>> q = tile + ((unsigned)m2 * W + w) * 3u;
      v[0][s] = ldc(q); v[1][s] = ldc(q + 1); v[2][s] = ldc(q + 2);
    }
  }
  if constexpr ((MODE & COL_FWD) != 0) {
    fft3<-1, T, L, RMAX, CL::db>(v[0], v[1], v[2], lre, t, tw);
  }
  if constexpr ((MODE & COL_GREEN) != 0) {
    const T lam0 = (T)S.prm.lam0, mu0 = (T)S.prm.mu0, scale = (T)x.scale;
    if (packed) {
      // Column 0 (bins m1 = 0 and L/2 packed) passes its transform through a
      // small global buffer to read the partners conj Z[L - m2]; the branch is
      // uniform over the block, and the barrier orders the global writes
      // before the reads within the block.
      if (wb == 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int s = 0; s < RMAX; ++s) stc(xbuf + (c * L + t + TPF * s), v[c][s]);
      }
      __threadfence_block();
      __syncthreads();
      if (wb == 0) {
#pragma unroll
        for (int s = 0; s < RMAX; ++s) {
          const int m2 = t + TPF * s;
          const int mr = (L - m2) & (L - 1);
          cx<T> x0[3], xn[3];
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const cx<T> zr = cconj(ldc(xbuf + (c * L + mr)));
            const cx<T> d = v[c][s] - zr;
            x0[c] = cscale(v[c][s] + zr, (T)0.5);
            xn[c] = {d.im * (T)0.5, -d.re * (T)0.5};
          }
          green_at<GK>(x0, 0, m2, S, x, lam0, mu0, scale);
          green_at<GK>(xn, L / 2, m2, S, x, lam0, mu0, scale);
#pragma unroll
          for (int c = 0; c < 3; ++c) v[c][s] = {x0[c].re - xn[c].im, x0[c].im + xn[c].re};
        }
      }
    }
    if (!packed || wb != 0) {
#pragma unroll
      for (int s = 0; s < RMAX; ++s) {
        const int m2 = t + TPF * s;
        cx<T> tt[3] = {v[0][s], v[1][s], v[2][s]};
        green_at<GK>(tt, m1, m2, S, x, lam0, mu0, scale);
        v[0][s] = tt[0]; v[1][s] = tt[1]; v[2][s] = tt[2];
      }
    }
  }
  if constexpr ((MODE & COL_INV) != 0) {
    fft3<+1, T, L, RMAX, CL::db>(v[0], v[1], v[2], lre, t, tw);
  }
  // Opaque copies of the lane's indices: the store addresses are recomputed
  // here instead of being held in registers from the loads.
  int ts = t, ws = w;
  asm volatile("" : "+v"(ts), "+v"(ws));
#pragma unroll
  for (int s = 0; s < RMAX; ++s) {
    const int m2 = ts + TPF * s;
    const int w = ws;
    if constexpr (PAIRV) {
      // lane 0: (c0, c1) at bytes 0-15, c2 at 16-23; lane 1: c0 at 24-31, (c1, c2) at 32-47
      const cx<T> p0 = w ? v[1][s] : v[0][s], p1 = w ? v[2][s] : v[1][s], q1 = w ? v[0][s] : v[2][s];
      gptr<f4> row = (gptr<f4>)(tile + (unsigned)m2 * 6u);
      row[w ? 2 : 0] = f4{p0.re, p0.im, p1.re, p1.im};
      stc(tile + (unsigned)m2 * 6u + (w ? 3u : 2u), q1);
      if ((s & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    } else {
      gptr<cx<T>> q = tile + ((unsigned)m2 * W + w) * 3u;
      stc(q, v[0][s]); stc(q + 1, v[1][s]); stc(q + 2, v[2][s]);
    }
  }
}

// ---------------------------------------------------------------------------
// Launch configuration per (precision, L, variant).  Variant 0 is the
// default; variant 1 the alternative the autotuner may choose for the
// iteration kernels (another row radix, another column radix).  The
// spectrum's tile width W is that of variant 0 for every variant, and the
// columns per block of any variant divide it, so the data layout never
// depends on the tuning.
template <typename T, int L>
struct ColTile {
  static constexpr int CDEF = L < 8 ? 4 : (sizeof(T) == 8 ? (L >= 2048 ? PM_COL_R64 : 4) : (L >= 2048 ? PM_COL_R32 : 8));
  static constexpr int CB = CDEF > L ? L : CDEF;
  static constexpr int COL_RMAX = CB * 512 >= L ? CB : L / 512;
  static constexpr int COL_TPF = L / COL_RMAX;
  static constexpr int W_RAW = COL_TPF >= 256 ? (sizeof(T) == 8 ? 1 : PM_COL_W32) : (256 / COL_TPF > 16 ? 16 : 256 / COL_TPF);
  static constexpr int W_CAP = W_RAW * COL_TPF > 1024 ? (1024 / COL_TPF > 0 ? 1024 / COL_TPF : 1) : W_RAW;
  static constexpr int W = W_CAP > L / 2 ? L / 2 : W_CAP;
};

template <typename T, int L, int V>
struct Cfg {
  static constexpr bool F64 = sizeof(T) == 8;
  // Row pass.
  static constexpr int RDEF = F64 ? PM_ROW_R64 : PM_ROW_R32;
  static constexpr int RALT = F64 ? (PM_ROW_R64 == 4 ? 8 : 4) : (PM_ROW_R32 == 16 ? 8 : 16);
  static constexpr int RBASE = L < 8 ? 4 : (V == 0 ? RDEF : RALT);
  static constexpr int RB = RBASE > L ? L : RBASE;
  static constexpr int RMAX = RB * PM_ROW_TPF_MAX >= L ? RB : L / PM_ROW_TPF_MAX;
  static constexpr int TPF = L / RMAX;
  static constexpr int ROW_TEAMS_RAW = TPF >= 256 ? 1 : 256 / TPF;
  static constexpr int ROW_TEAMS = ROW_TEAMS_RAW > L / 2 ? L / 2 : ROW_TEAMS_RAW;
  // Column pass: larger radix for long columns, blocks of at most 512 threads
  // (1024 for short columns).
  static constexpr int CDEF = ColTile<T, L>::CDEF;
  static constexpr int CALT = L < 8 ? 4 : (CDEF == 16 ? 8 : (CDEF == 8 ? (F64 ? 4 : 16) : 8));
  static constexpr int CBASE = V == 0 ? CDEF : CALT;
  static constexpr int CB = CBASE > L ? L : CBASE;
  static constexpr int COL_RMAX = CB * 512 >= L ? CB : L / 512;
  static constexpr int COL_TPF = L / COL_RMAX;
  static constexpr int COL_W = ColTile<T, L>::W;
  // columns per block: the tile width, except FP32 columns of 256 threads or
  // more (PM_COL_CB32 per block; one per block at 512 threads); always a
  // divisor of the tile width and at most 1024 threads per block
  static constexpr int CB_RAW = COL_TPF >= 512 ? 1
                                : (sizeof(T) == 4 && COL_TPF >= 256) ? PM_COL_CB32
                                : (V == 0 ? COL_W : (256 / COL_TPF > 0 ? 256 / COL_TPF : 1));
  static constexpr int CB_W = CB_RAW < COL_W ? CB_RAW : COL_W;
  static constexpr int COL_CB = CB_W * COL_TPF > 1024 ? 1024 / COL_TPF : CB_W;
  static_assert(COL_W % COL_CB == 0, "columns per block must divide the tile width");
};

template <typename T, int L, int V>
static size_t row_lds() {
  using C = Cfg<T, L, V>;
  return RowLds<T, L, C::ROW_TEAMS, C::TPF>::bytes;
}
template <typename T, int L, int V>
static size_t col_lds() {
  using C = Cfg<T, L, V>;
  return ColLds<T, L, C::COL_CB, C::COL_TPF>::bytes;
}

template <typename T, int L, int V, int MODE, bool NTS = false>
static hipError_t launch_row_LM(const Slot<T>* slots, int nslots, const Extra<T>& x, hipStream_t st) {
  using C = Cfg<T, L, V>;
  auto kern = k_row<T, L, C::RMAX, C::ROW_TEAMS, C::COL_W, MODE, NTS>;
  static bool attr = false;
  const size_t lds = row_lds<T, L, V>();
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr = true;
  }
  const int grid = nslots * ((L / 2) / C::ROW_TEAMS);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(C::ROW_TEAMS * C::TPF), lds, st, slots, x);
  return hipGetLastError();
}

template <typename T, int L, int V, int MODE>
static hipError_t launch_col_LM(const Slot<T>* slots, int nslots, const Extra<T>& x, hipStream_t st) {
  using C = Cfg<T, L, V>;
  auto kern = k_column<T, L, C::COL_RMAX, C::COL_W, C::COL_CB, MODE>;
  static bool attr = false;
  const size_t lds = col_lds<T, L, V>();
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr = true;
  }
  const int grid = nslots * ((L / 2) / C::COL_CB);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(C::COL_CB * C::COL_TPF), lds, st, slots, x);
  return hipGetLastError();
}

// The tuned variant applies to the iteration kernels (ROW_ITER, COL_ALL of
// every Green kind); the other modes always run variant 0.
template <typename T, int L>
static hipError_t launch_row_L(int mode, int v, const Slot<T>* slots, int nslots, const Extra<T>& x, hipStream_t st) {
  switch (mode) {
    case ROW_ITER:
      if (x.stream_state)
        return v ? launch_row_LM<T, L, 1, ROW_ITER, true>(slots, nslots, x, st)
                 : launch_row_LM<T, L, 0, ROW_ITER, true>(slots, nslots, x, st);
      return v ? launch_row_LM<T, L, 1, ROW_ITER>(slots, nslots, x, st)
               : launch_row_LM<T, L, 0, ROW_ITER>(slots, nslots, x, st);
    case ROW_INIT: return launch_row_LM<T, L, 0, ROW_INIT>(slots, nslots, x, st);
    case ROW_FWD: return launch_row_LM<T, L, 0, ROW_FWD>(slots, nslots, x, st);
    case ROW_SIGFWD: return launch_row_LM<T, L, 0, ROW_SIGFWD>(slots, nslots, x, st);
    case ROW_INV: return launch_row_LM<T, L, 0, ROW_INV>(slots, nslots, x, st);
    case ROW_EMIT: return launch_row_LM<T, L, 0, ROW_EMIT>(slots, nslots, x, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int L>
static hipError_t launch_col_L(int mode, int v, const Slot<T>* slots, int nslots, const Extra<T>& x, hipStream_t st) {
  switch (mode) {
    case COL_ALL:
      return v ? launch_col_LM<T, L, 1, COL_ALL>(slots, nslots, x, st)
               : launch_col_LM<T, L, 0, COL_ALL>(slots, nslots, x, st);
    case col_mode(COL_ALL, GK_DG1):
      return v ? launch_col_LM<T, L, 1, col_mode(COL_ALL, GK_DG1)>(slots, nslots, x, st)
               : launch_col_LM<T, L, 0, col_mode(COL_ALL, GK_DG1)>(slots, nslots, x, st);
    case col_mode(COL_ALL, GK_CG1):
      return v ? launch_col_LM<T, L, 1, col_mode(COL_ALL, GK_CG1)>(slots, nslots, x, st)
               : launch_col_LM<T, L, 0, col_mode(COL_ALL, GK_CG1)>(slots, nslots, x, st);
    case COL_FWD: return launch_col_LM<T, L, 0, COL_FWD>(slots, nslots, x, st);
    case COL_INV: return launch_col_LM<T, L, 0, COL_INV>(slots, nslots, x, st);
    case COL_GREEN: return launch_col_LM<T, L, 0, COL_GREEN>(slots, nslots, x, st);
    case col_mode(COL_GREEN, GK_DG1): return launch_col_LM<T, L, 0, col_mode(COL_GREEN, GK_DG1)>(slots, nslots, x, st);
    case col_mode(COL_GREEN, GK_CG1): return launch_col_LM<T, L, 0, col_mode(COL_GREEN, GK_CG1)>(slots, nslots, x, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int L>
static int row_grid_L(int v) {
  return v ? (L / 2) / Cfg<T, L, 1>::ROW_TEAMS : (L / 2) / Cfg<T, L, 0>::ROW_TEAMS;
}
template <typename T, int L>
static int tile_w_L(int) { return ColTile<T, L>::W; }

#define PM_DISPATCH_L(FN, T, L, ...)            \
  switch (L) {                                  \
    case 4: return FN<T, 4>(__VA_ARGS__);       \
    case 8: return FN<T, 8>(__VA_ARGS__);       \
    case 16: return FN<T, 16>(__VA_ARGS__);     \
    case 32: return FN<T, 32>(__VA_ARGS__);     \
    case 64: return FN<T, 64>(__VA_ARGS__);     \
    case 128: return FN<T, 128>(__VA_ARGS__);   \
    case 256: return FN<T, 256>(__VA_ARGS__);   \
    case 512: return FN<T, 512>(__VA_ARGS__);   \
    case 1024: return FN<T, 1024>(__VA_ARGS__); \
    case 2048: return FN<T, 2048>(__VA_ARGS__); \
    case 4096: return FN<T, 4096>(__VA_ARGS__); \
    case 8192: return FN<T, 8192>(__VA_ARGS__); \
    default: return hipErrorInvalidValue;       \
  }

template <typename T>
hipError_t launch_row(int L, int mode, int variant, const Slot<T>* slots, int nslots, const Extra<T>& x,
                      hipStream_t st) {
  PM_DISPATCH_L(launch_row_L, T, L, mode, variant, slots, nslots, x, st)
}
template <typename T>
hipError_t launch_col(int L, int mode, int variant, const Slot<T>* slots, int nslots, const Extra<T>& x,
                      hipStream_t st) {
  PM_DISPATCH_L(launch_col_L, T, L, mode, variant, slots, nslots, x, st)
}

#define PM_DISPATCH_INT(FN, T, L, V)    \
  switch (L) {                          \
    case 4: return FN<T, 4>(V);         \
    case 8: return FN<T, 8>(V);         \
    case 16: return FN<T, 16>(V);       \
    case 32: return FN<T, 32>(V);       \
    case 64: return FN<T, 64>(V);       \
    case 128: return FN<T, 128>(V);     \
    case 256: return FN<T, 256>(V);     \
    case 512: return FN<T, 512>(V);     \
    case 1024: return FN<T, 1024>(V);   \
    case 2048: return FN<T, 2048>(V);   \
    case 4096: return FN<T, 4096>(V);   \
    case 8192: return FN<T, 8192>(V);   \
    default: return -1;                 \
  }

template <typename T>
int row_blocks(int L, int variant) {
  PM_DISPATCH_INT(row_grid_L, T, L, variant)
}
template <typename T>
int tile_width(int L) {
  PM_DISPATCH_INT(tile_w_L, T, L, 0)
}

}  // namespace pm
