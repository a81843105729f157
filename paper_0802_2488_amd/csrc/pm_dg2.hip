// DG2 combination (Sec. 2, "Discrete Green functions"): the average of the
// strain fields of the four sign variants of the Green tensor, the
// Hencky-Mises stress of that average, the average of the four stresses and
// the plastic mask of the average, with fixed-order FP64 means.
#include "pm_kernels.hpp"

namespace pm {

constexpr int DG2_NSUM = 13;    // eps 4, S(eps) 4, average stress 4, plastic pixels

template <typename T>
struct Ptr4 {
  const T* p[4];
};

template <typename T>
__global__ void __launch_bounds__(256) k_dg2(long npx, DevParams prm, const uint8_t* __restrict__ mask_g,
                                             Ptr4<T> eps4, Ptr4<T> sig4, T* eps_out_g, T* soa_out_g, T* sav_out_g,
                                             uint8_t* pl_out_g, double* __restrict__ partials) {
  const Mat<T> m = make_mat<T>(prm);
  gptr<const uint8_t> mask = glb(mask_g);
  gptr<T> eps_out = glb(eps_out_g);
  gptr<T> soa_out = glb(soa_out_g);
  gptr<T> sav_out = glb(sav_out_g);
  gptr<uint8_t> pl_out = glb(pl_out_g);
  double acc[DG2_NSUM];
#pragma unroll
  for (int i = 0; i < DG2_NSUM; ++i) acc[i] = 0.0;
  const bool has_sig = sig4.p[0] != nullptr;
  for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < npx; p += (long)gridDim.x * blockDim.x) {
    const bool isv = mask[p] != 0;
    T e[4], so[4], sa[4] = {(T)0, (T)0, (T)0, (T)0};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const long ix = c * npx + p;
      e[c] = (((glb(eps4.p[0])[ix] + glb(eps4.p[1])[ix]) + glb(eps4.p[2])[ix]) + glb(eps4.p[3])[ix]) * (T)0.25;
      if (has_sig)
        sa[c] = (((glb(sig4.p[0])[ix] + glb(sig4.p[1])[ix]) + glb(sig4.p[2])[ix]) + glb(sig4.p[3])[ix]) * (T)0.25;
    }
    bool pl = false;
    if (isv) {
      so[0] = so[1] = so[2] = so[3] = (T)0;
    } else {
      pl = hencky(e, so, m);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      if (eps_out_g) eps_out[c * npx + p] = e[c];
      if (soa_out_g) soa_out[c * npx + p] = so[c];
      if (sav_out_g && has_sig) sav_out[c * npx + p] = sa[c];
      acc[c] += (double)e[c];
      acc[4 + c] += (double)so[c];
      acc[8 + c] += (double)sa[c];
    }
    if (pl_out_g) pl_out[p] = pl ? 1 : 0;
    acc[12] += pl ? 1.0 : 0.0;
  }
  block_reduce_store<DG2_NSUM>(acc, glb(partials) + (size_t)blockIdx.x * 16);
}

// Sum the per-block partials in block order; the means go after the partials.
__global__ void __launch_bounds__(256) k_dg2_final(double* __restrict__ partials_g, int nblk, double npx) {
  gptr<double> partials = glb(partials_g);
  __shared__ double red[256][DG2_NSUM];
  double s[DG2_NSUM];
#pragma unroll
  for (int i = 0; i < DG2_NSUM; ++i) s[i] = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 256) {
#pragma unroll
    for (int i = 0; i < DG2_NSUM; ++i) s[i] += partials[(long)b * 16 + i];
  }
#pragma unroll
  for (int i = 0; i < DG2_NSUM; ++i) red[threadIdx.x][i] = s[i];
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
#pragma unroll
      for (int i = 0; i < DG2_NSUM; ++i) red[threadIdx.x][i] += red[threadIdx.x + off][i];
    }
    __syncthreads();
  }
  if (threadIdx.x < DG2_NSUM) partials[(long)nblk * 16 + threadIdx.x] = red[0][threadIdx.x] / npx;
}

int dg2_blocks(int L) {
  const long npx = (long)L * L;
  long g = (npx + 255) / 256;
  if (g > 1024) g = 1024;
  return (int)g;
}

template <typename T>
hipError_t launch_dg2(int L, const DevParams& prm, const uint8_t* mask, const T* const* eps4, const T* const* sig4,
                      T* eps_out, T* soa_out, T* sav_out, uint8_t* pl_out, double* partials, int nblk,
                      hipStream_t s) {
  Ptr4<T> e, g;
  for (int i = 0; i < 4; ++i) {
    e.p[i] = eps4[i];
    g.p[i] = sig4 ? sig4[i] : nullptr;
  }
  const long npx = (long)L * L;
  hipLaunchKernelGGL(k_dg2<T>, dim3(nblk), dim3(256), 0, s, npx, prm, mask, e, g, eps_out, soa_out, sav_out, pl_out,
                     partials);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_dg2_final, dim3(1), dim3(256), 0, s, partials, nblk, (double)npx);
  return hipGetLastError();
}

// Five-point periodic average of each plane (CG2 post-processing).
template <typename T>
__global__ void __launch_bounds__(256) k_avg5(int L, long nval, const T* __restrict__ in_g, T* __restrict__ out_g) {
  gptr<const T> in = glb(in_g);
  gptr<T> out = glb(out_g);
  const long npx = (long)L * L;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < nval; i += (long)gridDim.x * blockDim.x) {
    const long base = (i / npx) * npx;
    const long p = i - base;
    const int x1 = (int)(p % L), x2 = (int)(p / L);
    const long l = base + (long)x2 * L + (x1 == 0 ? L - 1 : x1 - 1);
    const long r = base + (long)x2 * L + (x1 + 1 == L ? 0 : x1 + 1);
    const long u = base + (long)(x2 == 0 ? L - 1 : x2 - 1) * L + x1;
    const long d = base + (long)(x2 + 1 == L ? 0 : x2 + 1) * L + x1;
    out[i] = ((((in[i] + in[r]) + in[l]) + in[u]) + in[d]) / (T)5;
  }
}

template <typename T>
hipError_t launch_avg5(int L, int nplanes, const T* in, T* out, hipStream_t s) {
  const long nval = (long)nplanes * L * L;
  long g = (nval + 255) / 256;
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_avg5<T>, dim3((int)g), dim3(256), 0, s, L, nval, in, out);
  return hipGetLastError();
}
template hipError_t launch_avg5<float>(int, int, const float*, float*, hipStream_t);
template hipError_t launch_avg5<double>(int, int, const double*, double*, hipStream_t);

template hipError_t launch_dg2<float>(int, const DevParams&, const uint8_t*, const float* const*, const float* const*,
                                      float*, float*, float*, uint8_t*, double*, int, hipStream_t);
template hipError_t launch_dg2<double>(int, const DevParams&, const uint8_t*, const double* const*,
                                       const double* const*, double*, double*, double*, uint8_t*, double*, int,
                                       hipStream_t);

}  // namespace pm
