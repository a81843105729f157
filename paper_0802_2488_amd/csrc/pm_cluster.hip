// Void and plastic clusters of a solved grid (Sec. 3): periodic
// nearest-neighbour components of the void phase and of the void-plastic
// phase by union-find on the GPU, then each plastic cluster that touches no
// void joins the cluster of its nearest void.
//
// Union-find invariants: a pixel's link never exceeds its own index, and
// links only decrease (atomic min), so every find walks a strictly
// decreasing chain and every union retry strictly lowers the larger of its
// two roots: all loops end.  A component's root is its smallest pixel
// index, which makes the labels canonical.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pm_fft.hpp"

namespace pm {

__device__ __forceinline__ int ld_link(gptr<int> lab, int x) {
  return __hip_atomic_load((int*)(lab + x), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int cc_find(gptr<int> lab, int x) {
  int y = ld_link(lab, x);
  while (y != x) {
    x = y;
    y = ld_link(lab, x);
  }
  return x;
}

__device__ __forceinline__ void cc_union(gptr<int> lab, int a, int b) {
  while (true) {
    a = cc_find(lab, a);
    b = cc_find(lab, b);
    if (a == b) return;
    if (a > b) {
      const int t = a;
      a = b;
      b = t;
    }
    const int old = atomicMin((int*)(lab + b), a);
    if (old == b) return;   // b was a root and now links to a
    b = old;                // b had been linked meanwhile; join its new parent instead
  }
}

__device__ __forceinline__ bool in_phase(gptr<const uint8_t> vd, gptr<const uint8_t> pl, int mode, long p) {
  return vd[p] != 0 || (mode != 0 && pl[p] != 0);
}

// mode 0: void phase; mode 1: void-plastic phase.
__global__ void __launch_bounds__(256) k_cc_init(long npx, const uint8_t* vd_g, const uint8_t* pl_g, int mode,
                                                 int* lab_g) {
  gptr<const uint8_t> vd = glb(vd_g), pl = glb(pl_g);
  gptr<int> lab = glb(lab_g);
  for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < npx; p += (long)gridDim.x * blockDim.x)
    lab[p] = in_phase(vd, pl, mode, p) ? (int)p : -1;
}

__global__ void __launch_bounds__(256) k_cc_merge(int L, const uint8_t* vd_g, const uint8_t* pl_g, int mode,
                                                  int* lab_g) {
  gptr<const uint8_t> vd = glb(vd_g), pl = glb(pl_g);
  gptr<int> lab = glb(lab_g);
  const long npx = (long)L * L;
  for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < npx; p += (long)gridDim.x * blockDim.x) {
    if (!in_phase(vd, pl, mode, p)) continue;
    const int x1 = (int)(p % L), x2 = (int)(p / L);
    const long right = (long)x2 * L + (x1 + 1 == L ? 0 : x1 + 1);
    const long down = (long)(x2 + 1 == L ? 0 : x2 + 1) * L + x1;
    if (in_phase(vd, pl, mode, right)) cc_union(lab, (int)p, (int)right);
    if (in_phase(vd, pl, mode, down)) cc_union(lab, (int)p, (int)down);
  }
}

__global__ void __launch_bounds__(256) k_cc_compress(long npx, int* lab_g) {
  gptr<int> lab = glb(lab_g);
  for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < npx; p += (long)gridDim.x * blockDim.x) {
    if (lab[p] >= 0) lab[p] = cc_find(lab, (int)p);
  }
}

// counters[slot] += number of roots.
__global__ void __launch_bounds__(256) k_cc_roots(long npx, const int* lab_g, unsigned long long* ctr, int slot) {
  gptr<const int> lab = glb(lab_g);
  unsigned long long n = 0;
  for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < npx; p += (long)gridDim.x * blockDim.x)
    n += lab[p] == (int)p ? 1ull : 0ull;
  if (n) atomicAdd(ctr + slot, n);
}

__global__ void __launch_bounds__(256) k_cc_pixels(long npx, const uint8_t* vd_g, const uint8_t* pl_g,
                                                   unsigned long long* ctr) {
  gptr<const uint8_t> vd = glb(vd_g), pl = glb(pl_g);
  unsigned long long nv = 0, np = 0;
  for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < npx; p += (long)gridDim.x * blockDim.x) {
    const bool v = vd[p] != 0;
    nv += v ? 1ull : 0ull;
    np += (!v && pl[p] != 0) ? 1ull : 0ull;
  }
  if (nv) atomicAdd(ctr + 0, nv);
  if (np) atomicAdd(ctr + 1, np);
}

// flags[root] |= 1 for a void pixel, 2 for a plastic one.
__global__ void __launch_bounds__(256) k_cc_flags(long npx, const uint8_t* vd_g, const int* lab_g, int* flags) {
  gptr<const uint8_t> vd = glb(vd_g);
  gptr<const int> lab = glb(lab_g);
  for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < npx; p += (long)gridDim.x * blockDim.x) {
    const int r = lab[p];
    if (r >= 0) atomicOr(flags + r, vd[p] != 0 ? 1 : 2);
  }
}

// counters: [3] clusters, [4] clusters without plastic pixels, [5] clusters without voids.
__global__ void __launch_bounds__(256) k_cc_rawstats(long npx, const int* lab_g, const int* flags_g,
                                                     unsigned long long* ctr) {
  gptr<const int> lab = glb(lab_g), flags = glb(flags_g);
  unsigned long long n = 0, iso = 0, po = 0;
  for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < npx; p += (long)gridDim.x * blockDim.x) {
    if (lab[p] != (int)p) continue;
    ++n;
    iso += flags[p] == 1 ? 1ull : 0ull;
    po += flags[p] == 2 ? 1ull : 0ull;
  }
  if (n) atomicAdd(ctr + 3, n);
  if (iso) atomicAdd(ctr + 4, iso);
  if (po) atomicAdd(ctr + 5, po);
}

// For boundary pixels of clusters without voids: the nearest void pixel by
// periodic Euclidean distance, as key (d2 << 32) | index, minimised into the
// cluster's root.  Chebyshev rings of growing radius are scanned until no
// farther ring can hold a closer (or equally close) void; the radius never
// exceeds L / 2.
__global__ void __launch_bounds__(256) k_cc_nearest(int L, const uint8_t* vd_g, const int* lab_g, const int* flags_g,
                                                    unsigned long long* key) {
  gptr<const uint8_t> vd = glb(vd_g);
  gptr<const int> lab = glb(lab_g), flags = glb(flags_g);
  const long npx = (long)L * L;
  for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < npx; p += (long)gridDim.x * blockDim.x) {
    const int r = lab[p];
    if (r < 0 || flags[r] != 2) continue;
    const int x1 = (int)(p % L), x2 = (int)(p / L);
    const int xl = x1 == 0 ? L - 1 : x1 - 1, xr = x1 + 1 == L ? 0 : x1 + 1;
    const int yu = x2 == 0 ? L - 1 : x2 - 1, yd = x2 + 1 == L ? 0 : x2 + 1;
    const bool interior = lab[(long)x2 * L + xl] == r && lab[(long)x2 * L + xr] == r && lab[(long)yu * L + x1] == r &&
                          lab[(long)yd * L + x1] == r;
    if (interior) continue;   // a nearest pixel of the cluster lies on its boundary
    unsigned long long best = ~0ull;
    for (int rad = 1; rad <= L / 2; ++rad) {
      if ((best >> 32) < (unsigned long long)rad * rad) break;
      for (int k = -rad; k <= rad; ++k) {
        // the four sides of the ring (corners visited twice; harmless)
        const int dy4[4] = {-rad, rad, k, k};
        const int dx4[4] = {k, k, -rad, rad};
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          int yy = x2 + dy4[s], xx = x1 + dx4[s];
          yy = ((yy % L) + L) % L;
          xx = ((xx % L) + L) % L;
          const long v = (long)yy * L + xx;
          if (vd[v] == 0) continue;
          const unsigned long long d2 = (unsigned long long)(dy4[s] * dy4[s] + dx4[s] * dx4[s]);
          const unsigned long long kk = (d2 << 32) | (unsigned long long)v;
          if (kk < best) best = kk;
        }
      }
    }
    if (best != ~0ull) atomicMin(key + r, best);
  }
}

__global__ void __launch_bounds__(256) k_cc_attach(long npx, int* lab_g, const int* flags_g,
                                                   const unsigned long long* key_g) {
  gptr<int> lab = glb(lab_g);
  gptr<const int> flags = glb(flags_g);
  gptr<const unsigned long long> key = glb(key_g);
  for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < npx; p += (long)gridDim.x * blockDim.x) {
    if (flags[p] != 2) continue;            // only roots carry flags
    const unsigned long long k = key[p];
    if (k == ~0ull) continue;
    cc_union(lab, (int)p, (int)(k & 0xffffffffull));
  }
}

__global__ void __launch_bounds__(256) k_cc_size(long npx, const int* lab_g, int* size) {
  gptr<const int> lab = glb(lab_g);
  for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < npx; p += (long)gridDim.x * blockDim.x) {
    const int r = lab[p];
    if (r >= 0) atomicAdd(size + r, 1);
  }
}

// counters[7] = max over roots of (size << 32) | (2^32 - 1 - root): the
// largest cluster, the smallest root on ties.
__global__ void __launch_bounds__(256) k_cc_largest(long npx, const int* lab_g, const int* size_g,
                                                    unsigned long long* ctr) {
  gptr<const int> lab = glb(lab_g), size = glb(size_g);
  unsigned long long best = 0;
  for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < npx; p += (long)gridDim.x * blockDim.x) {
    if (lab[p] != (int)p) continue;
    const unsigned long long k = ((unsigned long long)size[p] << 32) | (0xffffffffull - (unsigned long long)p);
    if (k > best) best = k;
  }
  if (best) atomicMax(ctr + 7, best);
}

// Columns / rows holding a pixel of cluster `root`.
__global__ void __launch_bounds__(256) k_cc_span(int L, const int* lab_g, int root, int* cols, int* rows) {
  gptr<const int> lab = glb(lab_g);
  gptr<int> c = glb(cols), r = glb(rows);
  const long npx = (long)L * L;
  for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < npx; p += (long)gridDim.x * blockDim.x) {
    if (lab[p] != root) continue;
    c[p % L] = 1;
    r[p / L] = 1;
  }
}

__global__ void __launch_bounds__(256) k_cc_count_ones(int n, const int* a_g, unsigned long long* ctr, int slot) {
  gptr<const int> a = glb(a_g);
  unsigned long long s = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) s += a[i] ? 1ull : 0ull;
  if (s) atomicAdd(ctr + slot, s);
}

__global__ void __launch_bounds__(256) k_fill_u32(long n, unsigned* a_g, unsigned v) {
  gptr<unsigned> a = glb(a_g);
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) a[i] = v;
}

// ---------------------------------------------------------------------------
static int cc_grid(long n) {
  long g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return (int)g;
}

#define PM_LAUNCH(kern, n, ...)                                                            \
  do {                                                                                     \
    hipLaunchKernelGGL(kern, dim3(cc_grid(n)), dim3(256), 0, st, __VA_ARGS__);             \
    hipError_t e_ = hipGetLastError();                                                     \
    if (e_ != hipSuccess) return e_;                                                       \
  } while (0)

hipError_t cc_fill(unsigned* a, long n, unsigned v, hipStream_t st) {
  PM_LAUNCH(k_fill_u32, n, n, a, v);
  return hipSuccess;
}

hipError_t cc_label(int L, const uint8_t* vd, const uint8_t* pl, int mode, int* lab, hipStream_t st) {
  const long npx = (long)L * L;
  PM_LAUNCH(k_cc_init, npx, npx, vd, pl, mode, lab);
  PM_LAUNCH(k_cc_merge, npx, L, vd, pl, mode, lab);
  PM_LAUNCH(k_cc_compress, npx, npx, lab);
  return hipSuccess;
}

hipError_t cc_count_roots(long npx, const int* lab, unsigned long long* ctr, int slot, hipStream_t st) {
  PM_LAUNCH(k_cc_roots, npx, npx, lab, ctr, slot);
  return hipSuccess;
}

hipError_t cc_pixels(long npx, const uint8_t* vd, const uint8_t* pl, unsigned long long* ctr, hipStream_t st) {
  PM_LAUNCH(k_cc_pixels, npx, npx, vd, pl, ctr);
  return hipSuccess;
}

hipError_t cc_raw(long npx, const uint8_t* vd, const int* lab, int* flags, unsigned long long* ctr, hipStream_t st) {
  PM_LAUNCH(k_cc_flags, npx, npx, vd, lab, flags);
  PM_LAUNCH(k_cc_rawstats, npx, npx, lab, flags, ctr);
  return hipSuccess;
}

hipError_t cc_attach(int L, const uint8_t* vd, int* lab, const int* flags, unsigned long long* key, hipStream_t st) {
  const long npx = (long)L * L;
  PM_LAUNCH(k_cc_nearest, npx, L, vd, lab, flags, key);
  PM_LAUNCH(k_cc_attach, npx, npx, lab, flags, key);
  PM_LAUNCH(k_cc_compress, npx, npx, lab);
  return hipSuccess;
}

hipError_t cc_sizes(long npx, const int* lab, int* size, unsigned long long* ctr, hipStream_t st) {
  PM_LAUNCH(k_cc_size, npx, npx, lab, size);
  PM_LAUNCH(k_cc_largest, npx, npx, lab, size, ctr);
  PM_LAUNCH(k_cc_roots, npx, npx, lab, ctr, 6);
  return hipSuccess;
}

hipError_t cc_span(int L, const int* lab, int root, int* cols, int* rows, unsigned long long* ctr, hipStream_t st) {
  const long npx = (long)L * L;
  PM_LAUNCH(k_cc_span, npx, L, lab, root, cols, rows);
  PM_LAUNCH(k_cc_count_ones, L, L, cols, ctr, 8);
  PM_LAUNCH(k_cc_count_ones, L, L, rows, ctr, 9);
  return hipSuccess;
}

#undef PM_LAUNCH

}  // namespace pm

// ---------------------------------------------------------------------------
// C ABI
#include "pm.h"
#include <cmath>

#include "pm_host.hpp"

namespace {

struct CcLayout {
  size_t key, flags, ctr, cols, rows, total;
};

CcLayout cc_layout(int L) {
  CcLayout c{};
  const size_t npx = (size_t)L * L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = pmh::align_up(off + bytes, 256);
    return o;
  };
  c.key = take(npx * 8);     // void-phase labels, then nearest-void keys
  c.flags = take(npx * 4);   // root flags, then cluster sizes
  c.ctr = take(16 * 8);
  c.cols = take((size_t)L * 4);
  c.rows = take((size_t)L * 4);
  c.total = off;
  return c;
}

}  // namespace

extern "C" {

size_t pm_cluster_workspace_bytes(int32_t L) {
  if (!pmh::is_pow2(L) || L < 4 || L > PM_MAX_L) return 0;
  return cc_layout(L).total;
}

int pm_clusters(int32_t L, const uint8_t* d_void_mask, const uint8_t* d_plastic, int32_t* d_labels,
                void* d_workspace, size_t workspace_bytes, pm_cluster_stats* out, void* stream) {
  using pmh::fail;
  if (!pmh::is_pow2(L) || L < 4 || L > PM_MAX_L)
    return fail(PM_EINVAL, "L = %d must be a power of two in [4, %d]", L, PM_MAX_L);
  if (!d_void_mask || !d_plastic || !d_labels || !d_workspace || !out) return fail(PM_EINVAL, "NULL argument");
  const CcLayout c = cc_layout(L);
  if (workspace_bytes < c.total)
    return fail(PM_EINVAL, "workspace of %zu bytes is smaller than the %zu required", workspace_bytes, c.total);
  if (((uintptr_t)d_workspace) % 256 != 0) return fail(PM_EINVAL, "workspace must be 256-byte aligned");
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)d_workspace;
  unsigned long long* key = (unsigned long long*)(ws + c.key);
  int* flags = (int*)(ws + c.flags);
  unsigned long long* ctr = (unsigned long long*)(ws + c.ctr);
  int* cols = (int*)(ws + c.cols);
  int* rows = (int*)(ws + c.rows);
  const long npx = (long)L * L;
  unsigned long long h[16];

  PM_HIP(pm::cc_fill((unsigned*)ctr, 32, 0u, st));
  PM_HIP(pm::cc_pixels(npx, d_void_mask, d_plastic, ctr, st));
  // clusters of the void phase alone
  PM_HIP(pm::cc_label(L, d_void_mask, d_plastic, 0, (int*)key, st));
  PM_HIP(pm::cc_count_roots(npx, (const int*)key, ctr, 2, st));
  // void-plastic clusters, nearest-neighbour rule
  PM_HIP(pm::cc_label(L, d_void_mask, d_plastic, 1, d_labels, st));
  PM_HIP(pm::cc_fill((unsigned*)flags, npx, 0u, st));
  PM_HIP(pm::cc_raw(npx, d_void_mask, d_labels, flags, ctr, st));
  PM_HIP(hipMemcpyAsync(h, ctr, sizeof h, hipMemcpyDeviceToHost, st));
  PM_HIP(hipStreamSynchronize(st));
  // plastic clusters without a void join the cluster of their nearest void
  if (h[0] > 0 && h[5] > 0) {
    PM_HIP(pm::cc_fill((unsigned*)key, 2 * npx, 0xffffffffu, st));
    PM_HIP(pm::cc_attach(L, d_void_mask, d_labels, flags, key, st));
  }
  PM_HIP(pm::cc_fill((unsigned*)flags, npx, 0u, st));
  PM_HIP(pm::cc_sizes(npx, d_labels, flags, ctr, st));
  PM_HIP(hipMemcpyAsync(h, ctr, sizeof h, hipMemcpyDeviceToHost, st));
  PM_HIP(hipStreamSynchronize(st));
  int largest_root = -1;
  int64_t largest = 0;
  if (h[7] != 0) {
    largest = (int64_t)(h[7] >> 32);
    largest_root = (int)(0xffffffffull - (h[7] & 0xffffffffull));
    PM_HIP(pm::cc_fill((unsigned*)cols, L, 0u, st));
    PM_HIP(pm::cc_fill((unsigned*)rows, L, 0u, st));
    PM_HIP(pm::cc_span(L, d_labels, largest_root, cols, rows, ctr, st));
    PM_HIP(hipMemcpyAsync(h, ctr, sizeof h, hipMemcpyDeviceToHost, st));
    PM_HIP(hipStreamSynchronize(st));
  }
  out->n_void = (int64_t)h[0];
  out->n_plastic = (int64_t)h[1];
  out->n_void_clusters = (int64_t)h[2];
  out->n_clusters_raw = (int64_t)h[3];
  out->n_isolated_void_clusters = (int64_t)h[4];
  out->n_plastic_only_clusters = (int64_t)h[5];
  out->n_clusters = (int64_t)h[6];
  out->largest = largest;
  out->largest_label = largest_root;
  out->spans_x1 = (largest_root >= 0 && h[8] == (unsigned long long)L) ? 1 : 0;
  out->spans_x2 = (largest_root >= 0 && h[9] == (unsigned long long)L) ? 1 : 0;
  return PM_OK;
}

// Derivatives of the quadratic through three consecutive samples: with
// h1 = x1 - x0 and h2 = x2 - x1 the weights of (y0, y1, y2) are, for the
// slope at x0, x1, x2 and for the (constant) second derivative,
//   x0: (-(2 h1 + h2) / (h1 (h1 + h2)),  (h1 + h2) / (h1 h2), -h1 / (h2 (h1 + h2)))
//   x1: (-h2 / (h1 (h1 + h2)),  (h2 - h1) / (h1 h2),  h1 / (h2 (h1 + h2)))
//   x2: ( h2 / (h1 (h1 + h2)), -(h1 + h2) / (h1 h2),  (h1 + 2 h2) / (h2 (h1 + h2)))
//   y'': 2 (1 / (h1 (h1 + h2)), -1 / (h1 h2), 1 / (h2 (h1 + h2))).
int pm_cluster_indicators(const pm_cluster_stats* stats, int32_t L, double void_fraction,
                          pm_cluster_indicators_out* out) {
  using pmh::fail;
  if (!stats || !out) return fail(PM_EINVAL, "stats and out must be host pointers");
  if (!pmh::is_pow2(L) || L < 4 || L > PM_MAX_L)
    return fail(PM_EINVAL, "L = %d must be a power of two in [4, %d]", L, PM_MAX_L);
  const int64_t npx = (int64_t)L * L;
  const int64_t counts[] = {stats->n_void, stats->n_plastic, stats->n_void_clusters,
                            stats->n_isolated_void_clusters, stats->n_clusters, stats->largest};
  for (int64_t c : counts)
    if (c < 0 || c > npx) return fail(PM_EINVAL, "cluster count %lld outside [0, L^2]", (long long)c);
  if (stats->n_void + stats->n_plastic > npx)
    return fail(PM_EINVAL, "void and plastic pixels exceed L^2");
  const double area = (double)npx;
  const double f = void_fraction < 0.0 ? (double)stats->n_void / area : void_fraction;
  if (!(f < 1.0)) return fail(PM_EINVAL, "void fraction %g must be below 1", f);
  // Sec. 3: the void-plastic phase is the voids together with the plastic
  // zones; cluster counts are taken relative to the void clusters, which are
  // all the clusters of that phase at zero load.
  const double voids = stats->n_void_clusters > 0 ? (double)stats->n_void_clusters : 1.0;
  out->v_p = (double)(stats->n_void + stats->n_plastic) / area;
  out->f_p = out->v_p / (1.0 - f);
  out->v_max = (double)stats->largest / area;
  out->i = (double)stats->n_isolated_void_clusters / voids;
  out->n = (double)stats->n_clusters / voids;
  return PM_OK;
}

int pm_path_derivatives(int32_t n_steps, const double* x, const double* y, double* dy, double* d2y) {
  using pmh::fail;
  if (n_steps < 3) return fail(PM_EINVAL, "n_steps = %d: at least 3 samples are needed", n_steps);
  if (!x || !y) return fail(PM_EINVAL, "x and y must be host arrays");
  for (int k = 0; k < n_steps; ++k)
    if (!std::isfinite(x[k]) || (k > 0 && !(x[k] > x[k - 1])))
      return fail(PM_EINVAL, "x must be finite and strictly increasing (index %d)", k);
  for (int k = 0; k < n_steps; ++k) {
    // stencil k-1, k, k+1 inside; the first or last three samples at the ends
    const int c = k == 0 ? 1 : (k == n_steps - 1 ? n_steps - 2 : k);
    const double y0 = y[c - 1], y1 = y[c], y2 = y[c + 1];
    const double h1 = x[c] - x[c - 1], h2 = x[c + 1] - x[c], hs = h1 + h2;
    if (dy) {
      if (k == c)
        dy[k] = -h2 / (h1 * hs) * y0 + (h2 - h1) / (h1 * h2) * y1 + h1 / (h2 * hs) * y2;
      else if (k < c)
        dy[k] = -(2.0 * h1 + h2) / (h1 * hs) * y0 + hs / (h1 * h2) * y1 - h1 / (h2 * hs) * y2;
      else
        dy[k] = h2 / (h1 * hs) * y0 - hs / (h1 * h2) * y1 + (h1 + 2.0 * h2) / (h2 * hs) * y2;
    }
    if (d2y) d2y[k] = 2.0 * (y0 / (h1 * hs) - y1 / (h1 * h2) + y2 / (h2 * hs));
  }
  return PM_OK;
}

}  // extern "C"
