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
//                 backward-difference equilibrium residual when the other two
//                 indicators already pass                      (k_reduce*, k_div)
// The persistent state is the strain eps (4 planes: 11, 22, 33, 12) and the
// half spectrum; the Lagrange multiplier equals S(eps) after every iteration
// and is recomputed instead of stored.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pm_fft.hpp"
#include "pm_internal.h"

namespace pm {

// ---------------------------------------------------------------------------
// Material constants in the field precision.
template <typename T>
struct Mat {
  T mu, lam, Y, mu0, lam0, K, K0;
  T sy;        // sqrt(2/3) Y: Frobenius norm of the capped stress deviator
  T thr_rho;   // sqrt(2/3) Y (mu + mu0) / mu: plastic iff |dev R| exceeds it
  T inv2mu_mu0, inv2mu0, inv3KK0;
};

template <typename T>
__device__ __forceinline__ Mat<T> make_mat(const DevParams& p) {
  Mat<T> m;
  m.mu = (T)p.mu; m.lam = (T)p.lam; m.Y = (T)p.Y; m.mu0 = (T)p.mu0; m.lam0 = (T)p.lam0;
  m.K = (T)p.K; m.K0 = (T)p.K0; m.sy = (T)p.sy; m.thr_rho = (T)p.thr_rho;
  m.inv2mu_mu0 = (T)(1.0 / (2.0 * (p.mu + p.mu0)));
  m.inv2mu0 = (T)(1.0 / (2.0 * p.mu0));
  m.inv3KK0 = (T)(1.0 / (3.0 * (p.K + p.K0)));
  return m;
}

// Hencky-Mises stress of a matrix pixel; eps = (11, 22, 33, 12).
template <typename T>
__device__ __forceinline__ bool hencky(const T* e, T* s, const Mat<T>& m) {
  const T t3 = (e[0] + e[1] + e[2]) * (T)(1.0 / 3.0);
  const T d0 = e[0] - t3, d1 = e[1] - t3, d2 = e[2] - t3, d3 = e[3];
  const T nd = sqrt(d0 * d0 + d1 * d1 + d2 * d2 + (T)2 * d3 * d3);
  const bool plastic = (T)2 * m.mu * nd > m.sy;
  const T sc = plastic ? m.sy / nd : (T)2 * m.mu;
  const T pr = (T)3 * m.K * t3;
  s[0] = pr + sc * d0; s[1] = pr + sc * d1; s[2] = pr + sc * d2; s[3] = sc * d3;
  return plastic;
}

// Pointwise step: solve S(eps) + C0:eps = S(eps_old) + C0:e for one pixel.
// e = (e11, e22, e12) with e33 = 0.  Outputs eps_new, sigma and the in-plane
// polarisation tau = sigma - C0:eps_new.
template <typename T>
__device__ __forceinline__ void alm_point(const T* e, const T* eo, bool is_void, const Mat<T>& m, T* en, T* sg,
                                          T* tau) {
  if (is_void) {
    en[0] = e[0]; en[1] = e[1]; en[2] = (T)0; en[3] = e[2];
    sg[0] = sg[1] = sg[2] = sg[3] = (T)0;
    const T tr = e[0] + e[1];
    tau[0] = -(m.lam0 * tr + (T)2 * m.mu0 * e[0]);
    tau[1] = -(m.lam0 * tr + (T)2 * m.mu0 * e[1]);
    tau[2] = -((T)2 * m.mu0 * e[2]);
    return;
  }
  T la[4];
  hencky(eo, la, m);
  const T tre = m.lam0 * (e[0] + e[1]);
  const T R0 = la[0] + tre + (T)2 * m.mu0 * e[0];
  const T R1 = la[1] + tre + (T)2 * m.mu0 * e[1];
  const T R2 = la[2] + tre;
  const T R3 = la[3] + (T)2 * m.mu0 * e[2];
  const T trR3 = (R0 + R1 + R2) * (T)(1.0 / 3.0);
  const T r0 = R0 - trR3, r1 = R1 - trR3, r2 = R2 - trR3, r3 = R3;
  const T rho = sqrt(r0 * r0 + r1 * r1 + r2 * r2 + (T)2 * r3 * r3);
  const T tr_eps = (T)3 * trR3 * m.inv3KK0;
  T s0, s1, s2, s3, d0, d1, d2, d3;
  if (rho <= m.thr_rho) {
    d0 = r0 * m.inv2mu_mu0; d1 = r1 * m.inv2mu_mu0; d2 = r2 * m.inv2mu_mu0; d3 = r3 * m.inv2mu_mu0;
    const T tm = (T)2 * m.mu;
    s0 = tm * d0; s1 = tm * d1; s2 = tm * d2; s3 = tm * d3;
  } else {
    const T c = m.sy / rho;
    s0 = c * r0; s1 = c * r1; s2 = c * r2; s3 = c * r3;
    d0 = (r0 - s0) * m.inv2mu0; d1 = (r1 - s1) * m.inv2mu0; d2 = (r2 - s2) * m.inv2mu0; d3 = (r3 - s3) * m.inv2mu0;
  }
  const T t3 = tr_eps * (T)(1.0 / 3.0);
  en[0] = d0 + t3; en[1] = d1 + t3; en[2] = d2 + t3; en[3] = d3;
  const T pr = m.K * tr_eps;
  sg[0] = pr + s0; sg[1] = pr + s1; sg[2] = pr + s2; sg[3] = s3;
  const T c0t = m.lam0 * tr_eps;
  tau[0] = sg[0] - (c0t + (T)2 * m.mu0 * en[0]);
  tau[1] = sg[1] - (c0t + (T)2 * m.mu0 * en[1]);
  tau[2] = sg[3] - (T)2 * m.mu0 * en[3];
}

// ---------------------------------------------------------------------------
// Block reduction of NV doubles in a fixed order (wave shuffles, then LDS).
template <int NV>
__device__ __forceinline__ void block_reduce_store(double (&v)[NV], double* __restrict__ out) {
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

// Row-pass output: split the complex transform of x + i y into the half
// spectra X (component cx of row qx) and Y (component cy of row qy).
template <typename T, int L, int RMAX>
__device__ __forceinline__ void split_store(const cx<T> (&z)[RMAX], T* lre, T* lim, int t, cx<T>* qx, int cxi,
                                            cx<T>* qy, int cyi) {
  constexpr int TPF = L / RMAX;
  constexpr int H = L / 2 + 1;
  constexpr int NOUT = RMAX / 2 + 1;
  __syncthreads();
#pragma unroll
  for (int s = 0; s < RMAX; ++s) {
    const int idx = lpad(t + TPF * s);
    lre[idx] = z[s].re;
    lim[idx] = z[s].im;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NOUT; ++k) {
    const int mm = t + TPF * k;
    if (mm < H) {
      const int i0 = lpad(mm), i1 = lpad((L - mm) & (L - 1));
      const cx<T> zm = {lre[i0], lim[i0]};
      const cx<T> zr = {lre[i1], -lim[i1]};   // conj Z[L - m]
      const cx<T> d = zm - zr;
      qx[mm * 3 + cxi] = cscale(zm + zr, (T)0.5);
      qy[mm * 3 + cyi] = {d.im * (T)0.5, -d.re * (T)0.5};
    }
  }
}

// ---------------------------------------------------------------------------
// Row pass.  A team of TPF = L / RMAX threads owns rows a = 2p and b = 2p + 1
// and three complex length-L signals: Za = 11a + i 22a, Zb = 11b + i 22b,
// Zc = 12a + i 12b (two real rows per complex transform).
template <typename T, int L, int RMAX, int TEAMS, int MODE>
__global__ void __launch_bounds__(TEAMS*(L / RMAX)) __attribute__((amdgpu_waves_per_eu(2))) k_row(RowArgs<T> a) {
  constexpr int TPF = L / RMAX;
  constexpr int H = L / 2 + 1;
  constexpr int LS = LdsSize<L>::value;
  constexpr int LOAD_GROUP = RMAX >= 4 ? 4 : RMAX;   // unrolled iterations whose loads may be in flight together
  if (a.state && a.state->halted) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int team = threadIdx.x / TPF;
  const int t = threadIdx.x % TPF;
  T* lre = reinterpret_cast<T*>(smem_raw) + team * 2 * LS;
  T* lim = lre + LS;
  const int p = blockIdx.x * TEAMS + team;
  const int ra = 2 * p, rb = 2 * p + 1;
  const long P = a.pitch;
  cx<T>* __restrict__ spec = a.spec;
  const cx<T>* __restrict__ tw = a.tw;
  const Mat<T> m = make_mat<T>(a.prm);
  const long NPX = (long)L * L;

  cx<T> za[RMAX], zb[RMAX], zc[RMAX];
  double acc[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) acc[i] = 0.0;

  if constexpr (MODE == ROW_ITER || MODE == ROW_INV) {
    // Hermitian-extended load of the two row spectra, pattern A.
#pragma unroll
    for (int s = 0; s < RMAX; ++s) {
      const int mm = t + TPF * s;
      const bool direct = mm < H;
      const int mi = direct ? mm : L - mm;
      const cx<T>* qa = spec + ((long)ra * P + mi) * 3;
      const cx<T>* qb = spec + ((long)rb * P + mi) * 3;
      cx<T> a0 = qa[0], a1 = qa[1], a2 = qa[2];
      cx<T> b0 = qb[0], b1 = qb[1], b2 = qb[2];
      if (mi == 0 || mi == L / 2) {
        a0.im = a1.im = a2.im = b0.im = b1.im = b2.im = (T)0;
      }
      if (!direct) {
        a0 = cconj(a0); a1 = cconj(a1); a2 = cconj(a2);
        b0 = cconj(b0); b1 = cconj(b1); b2 = cconj(b2);
      }
      za[s] = {a0.re - a1.im, a0.im + a1.re};
      zb[s] = {b0.re - b1.im, b0.im + b1.re};
      zc[s] = {a2.re - b2.im, a2.im + b2.re};
      if ((s & (LOAD_GROUP - 1)) == LOAD_GROUP - 1) __builtin_amdgcn_sched_barrier(0);
    }
    fft<+1, T, L, RMAX>(za, lre, lim, t, tw);
    fft<+1, T, L, RMAX>(zb, lre, lim, t, tw);
    fft<+1, T, L, RMAX>(zc, lre, lim, t, tw);
  }

  if constexpr (MODE == ROW_INV) {
#pragma unroll
    for (int s = 0; s < RMAX; ++s) {
      const int x1 = t + TPF * s;
      const long ia = (long)ra * L + x1, ib = (long)rb * L + x1;
      a.real_out[ia] = za[s].re; a.real_out[NPX + ia] = za[s].im; a.real_out[2 * NPX + ia] = zc[s].re;
      a.real_out[ib] = zb[s].re; a.real_out[NPX + ib] = zb[s].im; a.real_out[2 * NPX + ib] = zc[s].im;
    }
    return;
  }

  if constexpr (MODE == ROW_FWD) {
#pragma unroll
    for (int s = 0; s < RMAX; ++s) {
      const int x1 = t + TPF * s;
      const long ia = (long)ra * L + x1, ib = (long)rb * L + x1;
      za[s] = {a.real_in[ia], a.real_in[NPX + ia]};
      zb[s] = {a.real_in[ib], a.real_in[NPX + ib]};
      zc[s] = {a.real_in[2 * NPX + ia], a.real_in[2 * NPX + ib]};
    }
  } else {
    // ROW_ITER or ROW_INIT: pointwise step per pixel.  The strain and mask
    // of the next pixel pair are fetched while the current one is solved,
    // and a scheduling fence per pixel pair bounds register pressure.
    T* __restrict__ eps = a.eps;
    const uint8_t* __restrict__ vm = a.mask;
    const T E0 = (T)a.E[0], E1 = (T)a.E[1], E2 = (T)a.E[2];
    T eo_n[2][4];
    uint8_t mk_n[2];
    auto fetch = [&](int s) {
      const int x1 = t + TPF * s;
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        const long ix = (long)(half ? rb : ra) * L + x1;
        mk_n[half] = vm[ix];
        if constexpr (MODE == ROW_ITER) {
#pragma unroll
          for (int c = 0; c < 4; ++c) eo_n[half][c] = eps[c * NPX + ix];
        }
      }
    };
    fetch(0);
#pragma unroll
    for (int s = 0; s < RMAX; ++s) {
      const int x1 = t + TPF * s;
      T eo_c[2][4];
      uint8_t mk_c[2];
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        mk_c[half] = mk_n[half];
#pragma unroll
        for (int c = 0; c < 4; ++c) eo_c[half][c] = eo_n[half][c];
      }
      if (s + 1 < RMAX) fetch(s + 1);
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        const long ix = (long)(half ? rb : ra) * L + x1;
        const bool isv = mk_c[half] != 0;
        T e[3], en[4], sg[4], tau[3];
        if constexpr (MODE == ROW_INIT) {
          e[0] = E0; e[1] = E1; e[2] = E2;
          en[0] = E0; en[1] = E1; en[2] = (T)0; en[3] = E2;
          if (isv) {
            sg[0] = sg[1] = sg[2] = sg[3] = (T)0;
          } else {
            hencky(en, sg, m);
          }
          const T c0t = m.lam0 * (E0 + E1);
          tau[0] = sg[0] - (c0t + (T)2 * m.mu0 * E0);
          tau[1] = sg[1] - (c0t + (T)2 * m.mu0 * E1);
          tau[2] = sg[3] - (T)2 * m.mu0 * E2;
        } else {
          if (half == 0) { e[0] = za[s].re; e[1] = za[s].im; e[2] = zc[s].re; }
          else { e[0] = zb[s].re; e[1] = zb[s].im; e[2] = zc[s].im; }
          alm_point(e, eo_c[half], isv, m, en, sg, tau);
        }
        eps[ix] = en[0]; eps[NPX + ix] = en[1]; eps[2 * NPX + ix] = en[2]; eps[3 * NPX + ix] = en[3];
        acc[0] += (double)sg[0]; acc[1] += (double)sg[1]; acc[2] += (double)sg[2]; acc[3] += (double)sg[3];
        acc[4] += (double)en[0]; acc[5] += (double)en[1]; acc[6] += (double)en[2]; acc[7] += (double)en[3];
        const double c0 = (double)e[0] - (double)en[0], c1 = (double)e[1] - (double)en[1];
        const double c2 = (double)en[2], c3 = (double)e[2] - (double)en[3];
        acc[8] += c0 * c0 + c1 * c1 + c2 * c2 + 2.0 * c3 * c3;
        if (half == 0) { za[s] = {tau[0], tau[1]}; zc[s].re = tau[2]; }
        else { zb[s] = {tau[0], tau[1]}; zc[s].im = tau[2]; }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }

  fft<-1, T, L, RMAX>(za, lre, lim, t, tw);
  fft<-1, T, L, RMAX>(zb, lre, lim, t, tw);
  fft<-1, T, L, RMAX>(zc, lre, lim, t, tw);

  // Split each complex transform into the two real-signal half spectra:
  // X = (Z[m] + conj Z[L-m]) / 2, Y = (Z[m] - conj Z[L-m]) / (2i).
  // Za -> (11, 22) of row a, Zb -> (11, 22) of row b, Zc -> 12 of rows a, b.
  split_store<T, L, RMAX>(za, lre, lim, t, spec + (long)ra * P * 3, 0, spec + (long)ra * P * 3, 1);
  split_store<T, L, RMAX>(zb, lre, lim, t, spec + (long)rb * P * 3, 0, spec + (long)rb * P * 3, 1);
  split_store<T, L, RMAX>(zc, lre, lim, t, spec + (long)ra * P * 3, 2, spec + (long)rb * P * 3, 2);

  if constexpr (MODE == ROW_ITER || MODE == ROW_INIT) {
    // teams of one block reduce together; per-block partials in fixed order
    block_reduce_store<9>(acc, a.partials + (long)blockIdx.x * NPART);
  }
}

// ---------------------------------------------------------------------------
// Column pass.  A team of TPF threads owns one column m1 of the row spectra;
// W adjacent columns per block with the column index fastest across lanes so
// each row access covers W * 3 complex contiguous values.
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
  const T idet = scale / det;
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

__device__ __forceinline__ int xcd_remap(int b, int nb) {
  // Blocks are dispatched round-robin over the 8 XCDs; give each XCD a
  // contiguous range of logical column groups so neighbouring groups, which
  // share cache lines, meet in the same L2.
  const int x = b & 7, q = nb >> 3, r = nb & 7;
  return x * q + (x < r ? x : r) + (b >> 3);
}

template <typename T, int L, int RMAX, int W, int MODE>
__global__ void __launch_bounds__(W*(L / RMAX)) __attribute__((amdgpu_waves_per_eu(2))) k_column(ColArgs<T> a) {
  constexpr int TPF = L / RMAX;
  constexpr int H = L / 2 + 1;
  constexpr int LS = LdsSize<L>::value;
  if (a.state && a.state->halted) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int w = threadIdx.x % W;
  const int t = threadIdx.x / W;
  T* lre = reinterpret_cast<T*>(smem_raw) + w * 2 * LS;
  T* lim = lre + LS;
  const int g = xcd_remap(blockIdx.x, gridDim.x);
  const int m1 = g * W + w;
  const bool valid = m1 < H;
  const long P = a.pitch;
  cx<T>* __restrict__ spec = a.spec;
  const cx<T>* __restrict__ tw = a.tw;

  cx<T> v[3][RMAX];
#pragma unroll
  for (int s = 0; s < RMAX; ++s) {
    const int m2 = t + TPF * s;
    if (valid) {
      const cx<T>* q = spec + ((long)m2 * P + m1) * 3;
      v[0][s] = q[0]; v[1][s] = q[1]; v[2][s] = q[2];
    } else {
      v[0][s] = v[1][s] = v[2][s] = {(T)0, (T)0};
    }
  }
  if constexpr ((MODE & COL_FWD) != 0) {
#pragma unroll
    for (int c = 0; c < 3; ++c) fft<-1, T, L, RMAX>(v[c], lre, lim, t, tw);
  }
  if constexpr ((MODE & COL_GREEN) != 0) {
    const T lam0 = (T)a.lam0, mu0 = (T)a.mu0, scale = (T)a.scale;
    cx<T> k1 = valid ? a.ktab[m1] : cx<T>{(T)0, (T)0};
    if (a.flip1) k1 = {-k1.re, k1.im};   // k(-q) = -conj(k(q))
#pragma unroll
    for (int s = 0; s < RMAX; ++s) {
      const int m2 = t + TPF * s;
      cx<T> k2 = a.ktab[m2];
      if (a.flip2) k2 = {-k2.re, k2.im};
      cx<T> tt[3] = {v[0][s], v[1][s], v[2][s]};
      if (m1 == 0 && m2 == 0) {
        tt[0] = {(T)a.E[0], (T)0};
        tt[1] = {(T)a.E[1], (T)0};
        tt[2] = {(T)a.E[2], (T)0};
        if (a.state) {
          tt[0].re = (T)a.state->E[0]; tt[1].re = (T)a.state->E[1]; tt[2].re = (T)a.state->E[2];
        }
      } else {
        green_apply(tt, k1, k2, lam0, mu0, scale);
      }
      v[0][s] = tt[0]; v[1][s] = tt[1]; v[2][s] = tt[2];
    }
  }
  if constexpr ((MODE & COL_INV) != 0) {
#pragma unroll
    for (int c = 0; c < 3; ++c) fft<+1, T, L, RMAX>(v[c], lre, lim, t, tw);
  }
  if (valid) {
#pragma unroll
    for (int s = 0; s < RMAX; ++s) {
      const int m2 = t + TPF * s;
      cx<T>* q = spec + ((long)m2 * P + m1) * 3;
      q[0] = v[0][s]; q[1] = v[1][s]; q[2] = v[2][s];
    }
  }
}

// ---------------------------------------------------------------------------
// Launch configuration per (precision, L).
template <typename T, int L>
struct Cfg {
  static constexpr int RBASE = (L < 8 || sizeof(T) == 8) ? 4 : 8;
  static constexpr int RMAX = RBASE * 1024 >= L ? RBASE : L / 1024;   // at most 1024 threads per transform
  static constexpr int TPF = L / RMAX;
  static constexpr int ROW_TEAMS_RAW = TPF >= 256 ? 1 : 256 / TPF;
  static constexpr int ROW_TEAMS = ROW_TEAMS_RAW > L / 2 ? L / 2 : ROW_TEAMS_RAW;
  static constexpr int COL_W_RAW = TPF >= 256 ? (sizeof(T) == 8 ? 2 : 4) : (256 / TPF > 16 ? 16 : 256 / TPF);
  static constexpr int COL_W = COL_W_RAW * TPF > 1024 ? 1024 / TPF : COL_W_RAW;
};

template <typename T, int L>
static size_t row_lds() {
  return (size_t)Cfg<T, L>::ROW_TEAMS * 2 * LdsSize<L>::value * sizeof(T);
}
template <typename T, int L>
static size_t col_lds() {
  return (size_t)Cfg<T, L>::COL_W * 2 * LdsSize<L>::value * sizeof(T);
}

template <typename T, int L, int MODE>
static hipError_t launch_row_LM(const RowArgs<T>& a, hipStream_t st) {
  using C = Cfg<T, L>;
  auto kern = k_row<T, L, C::RMAX, C::ROW_TEAMS, MODE>;
  static bool attr = false;
  const size_t lds = row_lds<T, L>();
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr = true;
  }
  const int grid = (L / 2) / C::ROW_TEAMS;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(C::ROW_TEAMS * C::TPF), lds, st, a);
  return hipGetLastError();
}

template <typename T, int L, int MODE>
static hipError_t launch_col_LM(const ColArgs<T>& a, hipStream_t st) {
  using C = Cfg<T, L>;
  auto kern = k_column<T, L, C::RMAX, C::COL_W, MODE>;
  static bool attr = false;
  const size_t lds = col_lds<T, L>();
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr = true;
  }
  const int H = L / 2 + 1;
  const int grid = (H + C::COL_W - 1) / C::COL_W;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(C::COL_W * C::TPF), lds, st, a);
  return hipGetLastError();
}

template <typename T, int L>
static hipError_t launch_row_L(const RowArgs<T>& a, hipStream_t st) {
  switch (a.mode) {
    case ROW_ITER: return launch_row_LM<T, L, ROW_ITER>(a, st);
    case ROW_INIT: return launch_row_LM<T, L, ROW_INIT>(a, st);
    case ROW_FWD: return launch_row_LM<T, L, ROW_FWD>(a, st);
    case ROW_INV: return launch_row_LM<T, L, ROW_INV>(a, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int L>
static hipError_t launch_col_L(const ColArgs<T>& a, hipStream_t st) {
  switch (a.mode) {
    case COL_ALL: return launch_col_LM<T, L, COL_ALL>(a, st);
    case COL_FWD: return launch_col_LM<T, L, COL_FWD>(a, st);
    case COL_INV: return launch_col_LM<T, L, COL_INV>(a, st);
    case COL_GREEN: return launch_col_LM<T, L, COL_GREEN>(a, st);
    default: return hipErrorInvalidValue;
  }
}

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
hipError_t launch_row(int L, const RowArgs<T>& a, hipStream_t st) {
  PM_DISPATCH_L(launch_row_L, T, L, a, st)
}
template <typename T>
hipError_t launch_col(int L, const ColArgs<T>& a, hipStream_t st) {
  PM_DISPATCH_L(launch_col_L, T, L, a, st)
}

template <typename T, int L>
static int row_grid_L() { return (L / 2) / Cfg<T, L>::ROW_TEAMS; }
template <typename T>
int row_grid(int L) {
  switch (L) {
    case 4: return row_grid_L<T, 4>();
    case 8: return row_grid_L<T, 8>();
    case 16: return row_grid_L<T, 16>();
    case 32: return row_grid_L<T, 32>();
    case 64: return row_grid_L<T, 64>();
    case 128: return row_grid_L<T, 128>();
    case 256: return row_grid_L<T, 256>();
    case 512: return row_grid_L<T, 512>();
    case 1024: return row_grid_L<T, 1024>();
    case 2048: return row_grid_L<T, 2048>();
    case 4096: return row_grid_L<T, 4096>();
    case 8192: return row_grid_L<T, 8192>();
    default: return -1;
  }
}

}  // namespace pm
