// Reductions, convergence logic, equilibrium residual, output sums and the
// mask generator.  One block per slot for the final reductions.
#include <atomic>

#include "pm_kernels.hpp"

namespace pm {

template <typename P>
__device__ __forceinline__ double norm4(P a) {
  return sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2] + 2.0 * a[3] * a[3]);
}

// Start a load step at E (also used when the device advances the ramp).
template <typename P>
__device__ __forceinline__ void begin_step(P st, double E0, double E1, double E2, double mu) {
  st->E[0] = E0; st->E[1] = E1; st->E[2] = E2;
  st->normE = sqrt(E0 * E0 + E1 * E1 + 2.0 * E2 * E2);
  st->floor_s = 1e-12 * mu * st->normE;
  st->iter = 0; st->halted = 0; st->status = ST_RUNNING; st->need_eq = 0;
  st->res_eq = st->res_mac = st->res_cmp = INFINITY;
  st->div_ticket = 0;
}

// A load step ended with `status`.  The slot halts.  Without a device ramp
// the host reads the state; with one, the step's record is written and
// marked pending: the output pass adds <eps> to it and the advance kernel
// starts the next step from the current state.
template <typename T, typename P>
__device__ __forceinline__ void end_step(P st, const Slot<T>& S, int status) {
  st->status = status;
  st->halted = 1;
  if (S.rec == nullptr || S.E_path == nullptr) return;
  StepRecord r;
  for (int i = 0; i < 4; ++i) {
    r.sm[i] = st->sm[i];
    r.em[i] = 0.0;
  }
  r.res_eq = st->res_eq; r.res_mac = st->res_mac; r.res_cmp = st->res_cmp;
  r.plastic = st->plastic;
  r.iters = st->iter; r.status = status;
  S.rec[st->step] = r;
  st->pending = 1;
}

// Sum the row-pass partials of one slot (fixed order), update <sigma>, the
// change indicator eta_2 and the constraint indicator; decide whether the
// equilibrium indicator must be evaluated this iteration.
template <typename T>
__global__ void __launch_bounds__(256) k_reduce(const Slot<T>* __restrict__ slots, int nblk) {
  const Slot<T>& S = slots[blockIdx.x];
  gptr<DevState> st = glb(S.st);
  if (st->halted) return;
  __shared__ double red[256][NSUM];
  double s[NSUM];
#pragma unroll
  for (int i = 0; i < NSUM; ++i) s[i] = 0.0;
  gptr<const double> part = glb(S.part);
  // a fixed order for any nblk: thread t adds blocks t, t + 256, ...; the
  // unrolled loop keeps several loads in flight
#pragma unroll 8
  for (int b = threadIdx.x; b < nblk; b += 256) {
#pragma unroll
    for (int i = 0; i < NSUM; ++i) s[i] += part[(long)b * NPART + i];
  }
#pragma unroll
  for (int i = 0; i < NSUM; ++i) red[threadIdx.x][i] = s[i];
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
#pragma unroll
      for (int i = 0; i < NSUM; ++i) red[threadIdx.x][i] += red[threadIdx.x + off][i];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const DevParams& prm = S.prm;
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
    st->plastic = red[0][5] * inv;
    bool bad = false;
    for (int i = 0; i < NSUM; ++i) bad |= !isfinite(red[0][i]);
    if (bad) {
      st->need_eq = 0;
      end_step(st, S, ST_NAN);
      return;
    }
    // 1: all other tests pass, so test equilibrium; 2: the last iteration
    // allowed, evaluate the equilibrium indicator only for the record.
    int need = (it >= 2 && rmac < prm.eta_mac && rcmp < prm.eta_cmp) ? 1 : 0;
    if (!need && it >= prm.max_iter) need = 2;
    st->need_eq = need;
  }
}

template <typename T>
__device__ __forceinline__ void finish_div(const Slot<T>& S, double (&acc)[1], int lb, int dbps, double norm,
                                           int force);

// Backward-difference divergence of eq. 1 of the stored stress:
// div_i(x) = sum_j sigma_ij(x) - sigma_ij(x - e^j), direction 1 = x1 (with
// x + e^j in place of x - e^j along a direction whose momentum the Green
// tensor takes at -q_j, the sign variants of DG2), and
// from it the equilibrium indicator eta_1, which ends the step on
// convergence or at max_iter.  Each block stores its partial sum; the last
// block of a slot to finish (a ticket in the slot state, taken after a
// device-scope fence that publishes the partial) adds the partials in index
// order and decides.  Blocks return at once unless the indicator is needed,
// so the fences only run in the iterations that evaluate it.  force: only
// record the indicator.
template <typename T>
__global__ void __launch_bounds__(256) k_div(const Slot<T>* __restrict__ slots, int L, int dbps, int force) {
  const Slot<T>& S = slots[blockIdx.x / dbps];
  const int lb = blockIdx.x % dbps;
  gptr<DevState> st = glb(S.st);
  if (!force && (st->halted || !st->need_eq)) return;
  const long npx = (long)L * L;
  // stress state: (11, 22, 33, 12) per pixel
  using v4 = T __attribute__((ext_vector_type(4)));
  gptr<const v4> __restrict__ sg = (gptr<const v4>)glb(S.sig);
  double acc[1] = {0.0};
  // neighbour of each direction: x - e^j, or x + e^j for a Green tensor
  // evaluated at -q_j (its momenta make the equilibrium a difference
  // towards x + e^j)
  const int o1 = S.flip1 ? 1 : L - 1, o2 = S.flip2 ? 1 : L - 1;
  for (long ix = (long)lb * blockDim.x + threadIdx.x; ix < npx; ix += (long)dbps * blockDim.x) {
    const int x1 = (int)(ix & (L - 1));
    const int x2 = (int)(ix / L);
    const long i1 = (long)x2 * L + ((x1 + o1) & (L - 1));   // x -/+ e^1
    const long i2 = (long)((x2 + o2) & (L - 1)) * L + x1;   // x -/+ e^2
    const v4 a = sg[ix], b1 = sg[i1], b2 = sg[i2];
    const double d1 = ((double)a.x - (double)b1.x) + ((double)a.w - (double)b2.w);
    const double d2 = ((double)a.w - (double)b1.w) + ((double)a.y - (double)b2.y);
    acc[0] += d1 * d1 + d2 * d2;
  }
  finish_div(S, acc, lb, dbps, 1.0 / S.prm.npx, force);
}

// Common end of the residual passes: every block stores its partial of
// sum |div sigma|^2; the last block of the slot to finish (a ticket in the
// slot state, taken after a device-scope fence that publishes the partial)
// adds the partials in index order, forms eta_1 = sqrt(sum * norm) / |<sigma>|
// and decides.  force: only record the indicator.
template <typename T>
__device__ __forceinline__ void finish_div(const Slot<T>& S, double (&acc)[1], int lb, int dbps, double norm,
                                           int force) {
  gptr<DevState> st = glb(S.st);
  gptr<double> part2 = glb(S.part2);
  block_reduce_store<1>(acc, part2 + lb);   // thread 0 stores the block's partial
  __shared__ int last;
  if (threadIdx.x == 0) {
    __threadfence();
    last = atomicAdd(&S.st->div_ticket, 1u) == (unsigned)dbps - 1;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  __shared__ double red[256];
  double s = 0.0;
  for (int b = threadIdx.x; b < dbps; b += 256) s += part2[b];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    st->div_ticket = 0;
    const double ns = fmax(norm4(st->sm), st->floor_s);
    const double req = sqrt(red[0] * norm) / ns;
    st->res_eq = req;
    if (force) return;
    if (!isfinite(red[0])) end_step(st, S, ST_NAN);
    else if (st->need_eq == 1 && req < S.prm.eta_eq) end_step(st, S, ST_CONVERGED);
    else if (st->iter >= S.prm.max_iter) end_step(st, S, ST_NOCONV);
  }
}

// The equilibrium indicator of the CG1 scheme: the continuum divergence
// i xi_j sigma_ij(q) of the stress, evaluated on its 2-D transform (the row
// and column forward passes have put it in `spec`, tiled and packed like
// the iteration's spectrum), xi the continuum frequencies of the bins;
// modes with a Nyquist component, on which the continuum Green operator
// imposes nothing, are left out.  Over the full spectrum, bins m1 = 1 ..
// L/2 - 1 stand for their conjugate partners too (weight 2); the packed
// column 0 holds Z = X0 + i XN, with X0(m2) = (Z(m2) + conj Z(-m2)) / 2 the
// transform of bin m1 = 0.  Parseval: <|div|^2> = sum / L^4.
template <typename T>
__global__ void __launch_bounds__(256) k_div_continuum(const Slot<T>* __restrict__ slots, int L, int WT, int dbps,
                                                       const cx<T>* __restrict__ spec_g) {
  const Slot<T>& S = slots[blockIdx.x / dbps];
  const int lb = blockIdx.x % dbps;
  gptr<DevState> st = glb(S.st);
  if (st->halted || !st->need_eq) return;
  gptr<const cx<T>> spec = glb(spec_g);
  const long nq = (long)L * (L / 2);
  const double w = 6.283185307179586476925286766559 / (double)L;
  double acc[1] = {0.0};
  for (long p = (long)lb * blockDim.x + threadIdx.x; p < nq; p += (long)dbps * blockDim.x) {
    const long tile = p / ((long)L * WT);
    const int r = (int)(p - tile * (long)L * WT);
    const int m2 = r / WT;
    const int m1 = (int)tile * WT + r % WT;
    if (m2 == L / 2) continue;
    double s[3][2];
    if (m1 > 0) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const cx<T> z = ldc(spec + p * 3 + c);
        s[c][0] = (double)z.re;
        s[c][1] = (double)z.im;
      }
    } else {
      const int mr = (L - m2) & (L - 1);
      const long pr = tile * (long)L * WT + (long)mr * WT;   // same tile, same column 0
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const cx<T> z = ldc(spec + p * 3 + c), zr = ldc(spec + pr * 3 + c);
        s[c][0] = 0.5 * ((double)z.re + (double)zr.re);
        s[c][1] = 0.5 * ((double)z.im - (double)zr.im);
      }
    }
    const double x1 = w * (double)m1;
    const double x2 = w * (double)(m2 < L / 2 ? m2 : m2 - L);
    const double weight = m1 > 0 ? 2.0 : 1.0;
    double v2s = 0.0;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const double a = x1 * s[0][k] + x2 * s[2][k];   // xi_1 sigma_11 + xi_2 sigma_12
      const double b = x1 * s[2][k] + x2 * s[1][k];   // xi_1 sigma_12 + xi_2 sigma_22
      v2s += a * a + b * b;
    }
    acc[0] += weight * v2s;
  }
  const double Ld = (double)L;
  finish_div(S, acc, lb, dbps, 1.0 / (Ld * Ld * Ld * Ld), 0);
}

// <eps> from the output pass's per-block sums; with gate GATE_PENDING only
// for slots whose step record waits for it, and into that record too.
template <typename T>
__global__ void __launch_bounds__(256) k_reduce_emit(const Slot<T>* __restrict__ slots, int nblk, int gate) {
  const Slot<T>& S = slots[blockIdx.x];
  if (gate == GATE_PENDING && !S.st->pending) return;
  __shared__ double red[256][4];
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nblk; b += 256) {
#pragma unroll
    for (int i = 0; i < 4; ++i) s[i] += S.part2[(long)b * 4 + i];
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
    DevState* st = S.st;
    for (int i = 0; i < 4; ++i) st->em[i] = red[0][i] / S.prm.npx;
    if (gate == GATE_PENDING && S.rec != nullptr) {
      for (int i = 0; i < 4; ++i) S.rec[st->step].em[i] = st->em[i];
    }
  }
}

// Move every slot with a pending record to the next load step of its ramp
// (the current state is the warm start), or mark it finished.
template <typename T>
__global__ void k_advance(const Slot<T>* __restrict__ slots, int nslots) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nslots) return;
  const Slot<T>& S = slots[i];
  DevState* st = S.st;
  if (!st->pending) return;
  st->pending = 0;
  const int next = st->step + 1;
  if (st->status == ST_NAN || next >= st->nsteps) {
    st->finished = 1;
    return;
  }
  if (st->hold) {
    st->held = 1;   // the host reads the step's fields, then resumes the slot
    return;
  }
  st->step = next;
  begin_step(st, S.E_path[3 * next], S.E_path[3 * next + 1], S.E_path[3 * next + 2], S.prm.mu);
}

__global__ void k_begin(DevState* st, double E0, double E1, double E2, double mu, int32_t step, int32_t nsteps,
                        int32_t hold) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    begin_step(st, E0, E1, E2, mu);
    st->step = step;
    st->nsteps = nsteps;
    st->finished = 0;
    st->pending = 0;
    st->hold = hold;
    st->held = 0;
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

// ---------------------------------------------------------------------------
// Tuning table: entry [precision][log2 L] holds row | col << 1.
namespace {
std::atomic<int> g_tune[2][14];
std::atomic<uint64_t> g_tune_gen{1};
int log2_of(int L) {
  int k = 0;
  while ((1 << k) < L) ++k;
  return k;
}
}  // namespace

Tuning get_tuning(int precision, int L) {
  const int k = log2_of(L);
  if (k < 2 || k > 13 || (precision != 0 && precision != 1)) return {0, 0};
  const int v = g_tune[precision][k].load(std::memory_order_relaxed);
  return {v & 1, (v >> 1) & 1};
}

int set_tuning(int precision, int L, Tuning t) {
  const int k = log2_of(L);
  if (k < 2 || k > 13 || (precision != 0 && precision != 1) || (t.row & ~1) || (t.col & ~1)) return -1;
  g_tune[precision][k].store(t.row | (t.col << 1), std::memory_order_relaxed);
  g_tune_gen.fetch_add(1, std::memory_order_relaxed);
  return 0;
}

uint64_t tuning_generation() { return g_tune_gen.load(std::memory_order_relaxed); }

int div_blocks(int L) {
  const long npx = (long)L * L;
  long g = (npx + 255) / 256;
  if (g > 256) g = 256;   // one block per CU; the pass is rarely needed and exits at once otherwise
  return (int)g;
}

template <typename T>
hipError_t launch_reduce(const Slot<T>* slots, int nslots, int nblk, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce<T>, dim3(nslots), dim3(256), 0, s, slots, nblk);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_div(const Slot<T>* slots, int nslots, int L, int force, hipStream_t s) {
  const int g = div_blocks(L);
  hipLaunchKernelGGL(k_div<T>, dim3(nslots * g), dim3(256), 0, s, slots, L, g, force);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_div_continuum(const Slot<T>* slots, int nslots, int L, const cx<T>* spec, hipStream_t s) {
  const int g = div_blocks(L);
  hipLaunchKernelGGL(k_div_continuum<T>, dim3(nslots * g), dim3(256), 0, s, slots, L, tile_width<T>(L), g, spec);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_reduce_emit(const Slot<T>* slots, int nslots, int nblk, int gate, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_emit<T>, dim3(nslots), dim3(256), 0, s, slots, nblk, gate);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_advance(const Slot<T>* slots, int nslots, hipStream_t s) {
  hipLaunchKernelGGL(k_advance<T>, dim3((nslots + 63) / 64), dim3(64), 0, s, slots, nslots);
  return hipGetLastError();
}

#define PM_INST(T)                                                                     \
  template hipError_t launch_reduce<T>(const Slot<T>*, int, int, hipStream_t);        \
  template hipError_t launch_div<T>(const Slot<T>*, int, int, int, hipStream_t);      \
  template hipError_t launch_div_continuum<T>(const Slot<T>*, int, int, const cx<T>*, hipStream_t); \
  template hipError_t launch_reduce_emit<T>(const Slot<T>*, int, int, int, hipStream_t); \
  template hipError_t launch_advance<T>(const Slot<T>*, int, hipStream_t);
PM_INST(float)
PM_INST(double)
#undef PM_INST

hipError_t launch_begin(DevState* st, const double* E, double mu, int32_t step, int32_t nsteps, int32_t hold,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_begin, dim3(1), dim3(64), 0, s, st, E[0], E[1], E[2], mu, step, nsteps, hold);
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
