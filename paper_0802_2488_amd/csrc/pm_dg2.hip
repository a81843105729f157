// DG2 combination (Sec. 2, "Discrete Green functions"): the average of the
// strain fields of the four sign variants of the Green tensor, the
// Hencky-Mises stress of that average, the average of the four stresses and
// the plastic mask of the average, with fixed-order FP64 means.
#include <cmath>
#include <mutex>

#include "pm.h"
#include "pm_host.hpp"
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

namespace pm {

// ---------------------------------------------------------------------------
// Measures of a strain map (the comparison of the methods in Fig. 1): the
// equivalent strain eps_eq = sqrt(2/3 e':e') (3-D deviator) on matrix pixels,
// its mean and maximum, the checkerboard index (root mean square of the
// mixed second difference eps_eq(x) - eps_eq(x + e1) - eps_eq(x + e2)
// + eps_eq(x + e1 + e2) over 2 x 2 blocks of matrix pixels, over the mean)
// and the sharpness (root mean square of the first differences between
// matrix neighbours, over the mean).  The mixed difference vanishes for a
// field that varies along one axis only and is 4 b for an oscillation
// b (-1)^(x1 + x2), so it picks out the checkerboard pattern.
constexpr int MAP_NSUM = 6;    // sum eps_eq, matrix pixels, sum d^2, blocks, sum diff^2, pairs
// a block's partials and the final values each take one 8-double record
static_assert(MAP_NSUM + 1 <= 8, "the map partials records hold 8 doubles");

template <typename T>
__device__ __forceinline__ double eps_eq_at(gptr<const T> e, long npx, long p) {
  const double a = (double)e[p], b = (double)e[npx + p], c = (double)e[2 * npx + p], d = (double)e[3 * npx + p];
  const double t3 = (a + b + c) / 3.0;
  const double d0 = a - t3, d1 = b - t3, d2 = c - t3;
  return sqrt(2.0 / 3.0 * (d0 * d0 + d1 * d1 + d2 * d2 + 2.0 * d * d));
}

template <typename T>
__global__ void __launch_bounds__(256) k_map_metrics(int L, const T* __restrict__ eps_g,
                                                     const uint8_t* __restrict__ mask_g,
                                                     double* __restrict__ partials) {
  gptr<const T> e = glb(eps_g);
  gptr<const uint8_t> mask = glb(mask_g);
  const long npx = (long)L * L;
  double acc[MAP_NSUM];
#pragma unroll
  for (int i = 0; i < MAP_NSUM; ++i) acc[i] = 0.0;
  double mx = 0.0;
  for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < npx; p += (long)gridDim.x * blockDim.x) {
    if (mask[p]) continue;
    const int x1 = (int)(p & (L - 1)), x2 = (int)(p / L);
    const long p1 = (long)x2 * L + ((x1 + 1) & (L - 1));               // x + e1
    const long p2 = (long)((x2 + 1) & (L - 1)) * L + x1;               // x + e2
    const long p12 = (long)((x2 + 1) & (L - 1)) * L + ((x1 + 1) & (L - 1));
    const double q = eps_eq_at<T>(e, npx, p);
    acc[0] += q;
    acc[1] += 1.0;
    mx = fmax(mx, q);
    const bool m1 = !mask[p1], m2 = !mask[p2];
    double q1 = 0.0, q2 = 0.0;
    if (m1) {
      q1 = eps_eq_at<T>(e, npx, p1);
      acc[4] += (q1 - q) * (q1 - q);
      acc[5] += 1.0;
    }
    if (m2) {
      q2 = eps_eq_at<T>(e, npx, p2);
      acc[4] += (q2 - q) * (q2 - q);
      acc[5] += 1.0;
    }
    if (m1 && m2 && !mask[p12]) {
      const double d = q - q1 - q2 + eps_eq_at<T>(e, npx, p12);
      acc[2] += d * d;
      acc[3] += 1.0;
    }
  }
  block_reduce_store<MAP_NSUM>(acc, glb(partials) + (size_t)blockIdx.x * 8);
  // block maximum (non-negative values): wave shuffles, then the waves in order
  __shared__ double wmax[4];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) m = fmax(m, wmax[w]);
    glb(partials)[(size_t)blockIdx.x * 8 + MAP_NSUM] = m;
  }
}

__global__ void __launch_bounds__(256) k_map_final(double* __restrict__ partials_g, int nblk) {
  gptr<double> partials = glb(partials_g);
  __shared__ double red[256][MAP_NSUM + 1];
  double s[MAP_NSUM + 1];
#pragma unroll
  for (int i = 0; i <= MAP_NSUM; ++i) s[i] = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 256) {
#pragma unroll
    for (int i = 0; i < MAP_NSUM; ++i) s[i] += partials[(long)b * 8 + i];
    s[MAP_NSUM] = fmax(s[MAP_NSUM], partials[(long)b * 8 + MAP_NSUM]);
  }
#pragma unroll
  for (int i = 0; i <= MAP_NSUM; ++i) red[threadIdx.x][i] = s[i];
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
#pragma unroll
      for (int i = 0; i < MAP_NSUM; ++i) red[threadIdx.x][i] += red[threadIdx.x + off][i];
      red[threadIdx.x][MAP_NSUM] = fmax(red[threadIdx.x][MAP_NSUM], red[threadIdx.x + off][MAP_NSUM]);
    }
    __syncthreads();
  }
  if (threadIdx.x <= MAP_NSUM) partials[(long)nblk * 8 + threadIdx.x] = red[0][threadIdx.x];
}

int map_blocks(int L) {
  const long npx = (long)L * L;
  long g = (npx + 255) / 256;
  if (g > 1024) g = 1024;
  return (int)g;
}

}  // namespace pm

// ---------------------------------------------------------------------------
// The combination without a caller workspace: its partial sums live in a
// file-scope device array of fixed size (one copy per GPU, kept until the
// process ends), reached through the address hipGetSymbolAddress returns on
// each device.  dg2_blocks caps the grid at 1024 blocks of 16 doubles, plus
// the 16 means, so the array covers every L up to PM_MAX_L.
namespace pm {
namespace {

constexpr int kScratchBlocks = 1024;
constexpr size_t kScratchDoubles = (size_t)kScratchBlocks * 16 + 16;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Address of this device's copy of the array, looked up once per device
// with that device current (the caller's current device).
int scratch_on_current_device(double** out) {
  int dev = -1;
  PM_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return pmh::fail(PM_EDEVICE, "device %d beyond the supported %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    PM_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return pmh::fail(PM_EDEVICE, "no address for the DG2 scratch array on device %d", dev);
    g_scratch_ptr[dev] = (double*)ptr;
  }
  *out = g_scratch_ptr[dev];
  return PM_OK;
}

}  // namespace
}  // namespace pm

extern "C" {

size_t pm_dg2_combine_static_max_bytes(void) { return pm::kScratchDoubles * sizeof(double); }

int pm_dg2_combine_static(const pm_params* params, const uint8_t* d_void_mask, const void* const d_eps[4],
                          const void* const d_sigma[4], pm_dg2_out* out, void* stream) {
  using pmh::fail;
  pm_params q;
  int rc = pmh::check_params(params, &q);
  if (rc != PM_OK) return rc;
  if (!d_void_mask || !d_eps || !out) return fail(PM_EINVAL, "NULL argument");
  for (int v = 0; v < 4; ++v) {
    if (!d_eps[v]) return fail(PM_EINVAL, "d_eps[%d] is NULL", v);
    if (d_sigma && !d_sigma[v]) return fail(PM_EINVAL, "d_sigma[%d] is NULL", v);
  }
  const int nblk = pm::dg2_blocks(q.L);
  const size_t need = ((size_t)nblk * 16 + 16) * sizeof(double);
  if (nblk > pm::kScratchBlocks || need > pm_dg2_combine_static_max_bytes())
    return fail(PM_EINVAL, "L = %d needs %zu bytes of scratch, beyond the %zu of the static array", q.L, need,
                pm_dg2_combine_static_max_bytes());
  double* part = nullptr;
  rc = pm::scratch_on_current_device(&part);
  if (rc != PM_OK) return rc;
  const pm::DevParams prm = pmh::dev_params(q);
  hipStream_t st = (hipStream_t)stream;
  // every block writes its own partials and the final kernel writes the
  // means, so nothing needs clearing between calls
  if (q.precision == PM_FP64) {
    PM_HIP(pm::launch_dg2<double>(q.L, prm, d_void_mask, (const double* const*)d_eps,
                                  (const double* const*)d_sigma, (double*)out->eps, (double*)out->sigma_of_avg,
                                  (double*)out->sigma_avg, out->plastic, part, nblk, st));
  } else {
    PM_HIP(pm::launch_dg2<float>(q.L, prm, d_void_mask, (const float* const*)d_eps, (const float* const*)d_sigma,
                                 (float*)out->eps, (float*)out->sigma_of_avg, (float*)out->sigma_avg, out->plastic,
                                 part, nblk, st));
  }
  double means[13];
  PM_HIP(hipMemcpyAsync(means, part + (size_t)nblk * 16, sizeof means, hipMemcpyDeviceToHost, st));
  PM_HIP(hipStreamSynchronize(st));
  for (int c = 0; c < 4; ++c) {
    out->eps_mean[c] = means[c];
    out->sigma_of_avg_mean[c] = means[4 + c];
    out->sigma_avg_mean[c] = means[8 + c];
  }
  out->plastic_fraction = means[12];
  return PM_OK;
}

size_t pm_strain_map_workspace_bytes(int32_t L) {
  if (!pmh::is_pow2(L) || L < 4 || L > PM_MAX_L) return 0;
  return ((size_t)pm::map_blocks(L) * 8 + 8) * sizeof(double);
}

int pm_strain_map_metrics(int32_t L, int32_t precision, const void* d_eps, const uint8_t* d_void_mask,
                          void* d_workspace, size_t workspace_bytes, pm_strain_map_out* out, void* stream) {
  using pmh::fail;
  if (!pmh::is_pow2(L) || L < 4 || L > PM_MAX_L)
    return fail(PM_EINVAL, "L = %d must be a power of two in [4, %d]", L, PM_MAX_L);
  if (precision != PM_FP32 && precision != PM_FP64) return fail(PM_EINVAL, "precision must be PM_FP32 or PM_FP64");
  if (!d_eps || !d_void_mask || !d_workspace || !out) return fail(PM_EINVAL, "NULL argument");
  const int nblk = pm::map_blocks(L);
  const size_t need = ((size_t)nblk * 8 + 8) * sizeof(double);
  if (workspace_bytes < need)
    return fail(PM_EINVAL, "workspace of %zu bytes is smaller than the %zu required", workspace_bytes, need);
  if (((uintptr_t)d_workspace) % 8 != 0) return fail(PM_EINVAL, "workspace must be 8-byte aligned");
  hipStream_t st = (hipStream_t)stream;
  double* part = (double*)d_workspace;
  if (precision == PM_FP64)
    hipLaunchKernelGGL(pm::k_map_metrics<double>, dim3(nblk), dim3(256), 0, st, L, (const double*)d_eps,
                       d_void_mask, part);
  else
    hipLaunchKernelGGL(pm::k_map_metrics<float>, dim3(nblk), dim3(256), 0, st, L, (const float*)d_eps,
                       d_void_mask, part);
  PM_HIP(hipGetLastError());
  hipLaunchKernelGGL(pm::k_map_final, dim3(1), dim3(256), 0, st, part, nblk);
  PM_HIP(hipGetLastError());
  double r[8];
  PM_HIP(hipMemcpyAsync(r, part + (size_t)nblk * 8, sizeof(double) * (pm::MAP_NSUM + 1), hipMemcpyDeviceToHost, st));
  PM_HIP(hipStreamSynchronize(st));
  out->matrix_pixels = (int64_t)r[1];
  out->mean_eq = r[1] > 0 ? r[0] / r[1] : 0.0;
  out->max_eq = r[pm::MAP_NSUM];
  const double m = out->mean_eq > 0 ? out->mean_eq : 1.0;
  out->checkerboard = r[3] > 0 ? std::sqrt(r[2] / r[3]) / m : 0.0;
  out->sharpness = r[5] > 0 ? std::sqrt(r[4] / r[5]) / m : 0.0;
  return PM_OK;
}

}  // extern "C"
