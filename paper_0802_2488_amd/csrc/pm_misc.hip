// Reductions, convergence logic, residual, outputs and the mask generator.
#include "pm_kernels.hpp"

namespace pm {

// ---------------------------------------------------------------------------
// Reductions and convergence logic (one block of 256 threads).
__device__ __forceinline__ double norm4(const double* a) {
  return sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2] + 2.0 * a[3] * a[3]);
}

__global__ void __launch_bounds__(256) k_reduce(const double* __restrict__ partials, int nblk, DevState* st,
                                                DevParams prm) {
  if (st->halted) return;
  __shared__ double red[256][5];
  double s[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) s[i] = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 256) {
#pragma unroll
    for (int i = 0; i < 5; ++i) s[i] += partials[(long)b * NPART + i];
  }
#pragma unroll
  for (int i = 0; i < 5; ++i) red[threadIdx.x][i] = s[i];
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
#pragma unroll
      for (int i = 0; i < 5; ++i) red[threadIdx.x][i] += red[threadIdx.x + off][i];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double inv = 1.0 / prm.npx;
    double sm[4], dsm[4];
    for (int i = 0; i < 4; ++i) {
      sm[i] = red[0][i] * inv;
      dsm[i] = sm[i] - st->sm[i];
    }
    const int it = st->iter + 1;
    st->iter = it;
    const double ns = fmax(norm4(sm), st->floor_s);
    const double rcmp = sqrt(red[0][4] * inv) / st->normE;
    const double rmac = it >= 2 ? norm4(dsm) / ns : INFINITY;
    for (int i = 0; i < 4; ++i) {
      st->sm_prev[i] = st->sm[i];
      st->sm[i] = sm[i];
    }
    st->res_cmp = rcmp;
    st->res_mac = rmac;
    st->res_eq = INFINITY;
    bool bad = false;
    for (int i = 0; i < 5; ++i) bad |= !isfinite(red[0][i]);
    if (bad) {
      st->status = ST_NAN;
      st->halted = 1;
      st->need_eq = 0;
      return;
    }
    const int need = (it >= 2 && rmac < prm.eta_mac && rcmp < prm.eta_cmp) ? 1 : 0;
    st->need_eq = need;
    if (!need && it >= prm.max_iter) {
      st->status = ST_NOCONV;
      st->halted = 1;
    }
  }
}

// Backward-difference divergence of eq. 1 of the stored stress:
// div_i(x) = sum_j sigma_ij(x) - sigma_ij(x - e^j), direction 1 = x1.
template <typename T>
__global__ void __launch_bounds__(256) k_div(const T* __restrict__ sig, double* __restrict__ partials,
                                             const DevState* st, int L, int force) {
  if (!force && (st->halted || !st->need_eq)) return;
  const long npx = (long)L * L;
  const T* __restrict__ s11 = sig;
  const T* __restrict__ s22 = sig + npx;
  const T* __restrict__ s12 = sig + 3 * npx;
  double acc[1] = {0.0};
  for (long ix = (long)blockIdx.x * blockDim.x + threadIdx.x; ix < npx; ix += (long)gridDim.x * blockDim.x) {
    const int x1 = (int)(ix & (L - 1));
    const int x2 = (int)(ix / L);
    const long i1 = (long)x2 * L + ((x1 + L - 1) & (L - 1));   // x - e^1
    const long i2 = (long)((x2 + L - 1) & (L - 1)) * L + x1;   // x - e^2
    const double d1 = ((double)s11[ix] - (double)s11[i1]) + ((double)s12[ix] - (double)s12[i2]);
    const double d2 = ((double)s12[ix] - (double)s12[i1]) + ((double)s22[ix] - (double)s22[i2]);
    acc[0] += d1 * d1 + d2 * d2;
  }
  block_reduce_store<1>(acc, partials + blockIdx.x);
}

__global__ void __launch_bounds__(256) k_reduce_div(const double* __restrict__ partials, int nblk, DevState* st,
                                                    DevParams prm, int force) {
  if (!force && (st->halted || !st->need_eq)) return;
  __shared__ double red[256];
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 256) s += partials[b];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double ns = fmax(norm4(st->sm), st->floor_s);
    const double req = sqrt(red[0] / prm.npx) / ns;
    st->res_eq = req;
    if (force) return;
    if (!isfinite(red[0])) {
      st->status = ST_NAN;
      st->halted = 1;
    } else if (req < prm.eta_eq) {
      st->status = ST_CONVERGED;
      st->halted = 1;
    } else if (st->iter >= prm.max_iter) {
      st->status = ST_NOCONV;
      st->halted = 1;
    }
  }
}

__global__ void k_begin(DevState* st, double E0, double E1, double E2, double floor_s) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st->E[0] = E0; st->E[1] = E1; st->E[2] = E2;
    st->normE = sqrt(E0 * E0 + E1 * E1 + 2.0 * E2 * E2);
    st->floor_s = floor_s;
    st->iter = 0; st->halted = 0; st->status = ST_RUNNING; st->need_eq = 0;
    st->res_eq = st->res_mac = st->res_cmp = INFINITY;
  }
}

// Final FP64 reduction of the per-block strain sums written by the output pass.
__global__ void __launch_bounds__(256) k_reduce_emit(const double* __restrict__ partials, int nblk, DevState* st,
                                                     double npx) {
  __shared__ double red[256][4];
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nblk; b += 256) {
#pragma unroll
    for (int i = 0; i < 4; ++i) s[i] += partials[(long)b * 4 + i];
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) red[threadIdx.x][i] = s[i];
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
#pragma unroll
      for (int i = 0; i < 4; ++i) red[threadIdx.x][i] += red[threadIdx.x + off][i];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    for (int i = 0; i < 4; ++i) st->em[i] = red[0][i] / npx;
  }
}

// Counter-based Bernoulli mask: SplitMix64 (Steele, Lea, Flood 2014).
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void __launch_bounds__(256) k_mask(uint8_t* __restrict__ out, long npx, double f, uint64_t seed) {
  for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < npx; p += (long)gridDim.x * blockDim.x) {
    const uint64_t z = splitmix64(seed ^ splitmix64((uint64_t)p));
    const double u = (double)(z >> 11) * 0x1.0p-53;
    out[p] = u < f ? 1 : 0;
  }
}


int div_grid(int L) {
  const long npx = (long)L * L;
  long g = (npx + 255) / 256;
  if (g > 4096) g = 4096;
  return (int)g;
}

hipError_t launch_reduce(const double* partials, int nblk, DevState* st, const DevParams& prm, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, s, partials, nblk, st, prm);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_div(const T* sig, double* partials, DevState* st, const DevParams& prm, int L, int force,
                      hipStream_t s) {
  const int g = div_grid(L);
  hipLaunchKernelGGL(k_div<T>, dim3(g), dim3(256), 0, s, sig, partials, st, L, force);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_div, dim3(1), dim3(256), 0, s, partials, g, st, prm, force);
  return hipGetLastError();
}
template hipError_t launch_div<float>(const float*, double*, DevState*, const DevParams&, int, int, hipStream_t);
template hipError_t launch_div<double>(const double*, double*, DevState*, const DevParams&, int, int, hipStream_t);

hipError_t launch_begin(DevState* st, const double* E, double floor_s, hipStream_t s) {
  hipLaunchKernelGGL(k_begin, dim3(1), dim3(64), 0, s, st, E[0], E[1], E[2], floor_s);
  return hipGetLastError();
}

hipError_t launch_reduce_emit(const double* partials, int nblk, DevState* st, double npx, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_emit, dim3(1), dim3(256), 0, s, partials, nblk, st, npx);
  return hipGetLastError();
}

hipError_t launch_mask(uint8_t* out, long npx, double f, uint64_t seed, hipStream_t s) {
  long g = (npx + 255) / 256;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_mask, dim3((int)g), dim3(256), 0, s, out, npx, f, seed);
  return hipGetLastError();
}

}  // namespace pm
