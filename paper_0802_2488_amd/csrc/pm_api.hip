// C-ABI layer: parameter checks, workspace layout, tables, and the host loop
// of one load step.  All arithmetic of the method runs in the kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "pm.h"
#include "pm_host.hpp"
#include "pm_internal.h"

using pm::DevParams;
using pm::DevState;
using pmh::fail;
using pmh::Layout;

static_assert(sizeof(pm::Slot<float>) == sizeof(pm::Slot<double>), "slot layout must not depend on T");
static_assert(sizeof(pm::StepRecord) == sizeof(pm_step_record), "device and public step records differ");

namespace pmh {

namespace {
thread_local std::string g_err;
}

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

const char* last_error() { return g_err.c_str(); }

int check_params(const pm_params* p, pm_params* q) {
  if (!p) return fail(PM_EINVAL, "params is NULL");
  *q = *p;
  if (!is_pow2(q->L) || q->L < 4 || q->L > PM_MAX_L)
    return fail(PM_EINVAL, "L = %d must be a power of two in [4, %d]", q->L, PM_MAX_L);
  if (!(q->mu > 0) || !(3 * q->lambda + 2 * q->mu > 0) || !(q->Y > 0) || !std::isfinite(q->lambda) ||
      !std::isfinite(q->mu) || !std::isfinite(q->Y))
    return fail(PM_EINVAL, "need mu > 0, 3 lambda + 2 mu > 0, Y > 0 (got mu=%g lambda=%g Y=%g)", q->mu, q->lambda,
                q->Y);
  if (q->mu0 == 0.0) q->mu0 = 2.0 * q->mu;
  if (q->lambda0 == 0.0) q->lambda0 = 2.0 * q->lambda;
  if (!(q->mu0 > 0) || !(q->lambda0 + q->mu0 > 0) || !std::isfinite(q->lambda0))
    return fail(PM_EINVAL, "reference medium needs mu0 > 0 and lambda0 + mu0 > 0");
  if (!(q->eta_eq >= 0) || !(q->eta_mac >= 0) || !(q->eta_cmp >= 0))
    return fail(PM_EINVAL, "tolerances must be >= 0");
  if (q->max_iter < 1) return fail(PM_EINVAL, "max_iter must be >= 1");
  if (q->check_every < 0) return fail(PM_EINVAL, "check_every must be >= 0");
  if (q->precision != PM_FP32 && q->precision != PM_FP64) return fail(PM_EINVAL, "precision must be PM_FP32 or PM_FP64");
  if (q->green_variant < 0 || q->green_variant > 5) return fail(PM_EINVAL, "green_variant must be 0..5");
  return PM_OK;
}

DevParams dev_params(const pm_params& q) {
  DevParams d{};
  d.mu = q.mu; d.lam = q.lambda; d.Y = q.Y; d.mu0 = q.mu0; d.lam0 = q.lambda0;
  d.K = q.lambda + 2.0 * q.mu / 3.0;
  d.K0 = q.lambda0 + 2.0 * q.mu0 / 3.0;
  d.sy = std::sqrt(2.0 / 3.0) * q.Y;
  d.npx = (double)q.L * (double)q.L;
  d.eta_eq = q.eta_eq; d.eta_mac = q.eta_mac; d.eta_cmp = q.eta_cmp;
  d.max_iter = q.max_iter;
  d.L = q.L;
  return d;
}

Layout make_layout(const pm_params& q, bool tables, bool state) {
  Layout lo{};
  const size_t L = (size_t)q.L;
  const size_t fs = q.precision == PM_FP64 ? 8 : 4;
  // row-pass blocks of the larger of the two kernel variants
  lo.nrow = q.precision == PM_FP64 ? std::max(pm::row_blocks<double>(q.L, 0), pm::row_blocks<double>(q.L, 1))
                                   : std::max(pm::row_blocks<float>(q.L, 0), pm::row_blocks<float>(q.L, 1));
  lo.ndiv = std::max(pm::div_blocks(q.L), 4 * lo.nrow);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  };
  lo.sig = take(4 * L * L * fs);
  lo.spec = take(L * (L / 2) * 3 * 2 * fs);
  lo.xbuf = take(3 * L * 2 * fs);
  lo.tw = tables ? take(L * 2 * fs) : 0;
  lo.ktab = tables ? take(L * 2 * fs) : 0;
  lo.part = take((size_t)lo.nrow * pm::NPART * sizeof(double));
  lo.part2 = take((size_t)lo.ndiv * sizeof(double));
  lo.state = state ? take(sizeof(DevState)) : 0;
  lo.slot = state ? take(sizeof(pm::Slot<double>)) : 0;
  lo.spec2 = q.green_variant == 5 ? take(L * (L / 2) * 3 * 2 * fs) : 0;
  lo.total = off;
  return lo;
}

uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace pmh

struct pm_solver {
  pm_params p;
  Layout lo;
  hipStream_t stream;
  int device;
  char* ws;
  void* sig;       // state: stress of the last iterate, 4 components per pixel
  void* spec;
  DevState* st;
  void* slot;      // device table of one pm::Slot<T>
  DevState* hst;   // pinned host copies (two slots)
  hipEvent_t ev[2];
  bool started;
  int chunk;
  // opt-in per-kernel timing of every timing_every-th iteration
  bool timing = false;
  int timing_every = 1;
  std::vector<hipEvent_t> tev;   // 4 events per iteration of a chunk, for both chunk slots
  pm_kernel_timing tacc;
};

namespace {

template <typename T>
const pm::Slot<T>* dslot(const pm_solver* s) {
  return (const pm::Slot<T>*)s->slot;
}

// Tables and the one-entry slot table, uploaded once at create.
template <typename T>
int upload_tables(pm_solver* s, const uint8_t* mask) {
  const int L = s->p.L;
  std::vector<pm::cx<T>> tw, kt;
  pmh::make_tables<T>(L, tw, kt);
  char* tw_d = s->ws + s->lo.tw;
  char* kt_d = s->ws + s->lo.ktab;
  const pm::Slot<T> S = pmh::make_slot<T>(s->p, s->ws, s->lo, mask, tw_d, kt_d, s->st);
  PM_HIP(hipMemcpyAsync(tw_d, tw.data(), L * sizeof(pm::cx<T>), hipMemcpyHostToDevice, s->stream));
  PM_HIP(hipMemcpyAsync(kt_d, kt.data(), L * sizeof(pm::cx<T>), hipMemcpyHostToDevice, s->stream));
  PM_HIP(hipMemcpyAsync(s->slot, &S, sizeof S, hipMemcpyHostToDevice, s->stream));
  PM_HIP(hipStreamSynchronize(s->stream));
  return PM_OK;
}

int green_kind(const pm_params& q) {
  return q.green_variant == 4 ? pm::GK_DG1 : q.green_variant == 5 ? pm::GK_CG1 : pm::GK_SIGN;
}

template <typename T>
int iterate_once(pm_solver* s, int slot_in_chunk, int chunk_slot = 0) {
  const int L = s->p.L;
  pm::Extra<T> x = pmh::extra<T>(1, pm::GATE_RUNNING, 1.0 / ((double)L * (double)L), nullptr);
  x.stream_state = pmh::stream_state((size_t)L * L * 4 * sizeof(T));
  const pm::Slot<T>* S = dslot<T>(s);
  hipEvent_t* ev = s->timing && slot_in_chunk % s->timing_every == 0
                      ? &s->tev[4 * ((size_t)chunk_slot * s->chunk + slot_in_chunk)]
                      : nullptr;
  if (ev) PM_HIP(hipEventRecord(ev[0], s->stream));
  const pm::Tuning tv = pm::get_tuning(s->p.precision, L);
  PM_HIP(pm::launch_col<T>(L, pm::col_mode(pm::COL_ALL, green_kind(s->p)), tv.col, S, 1, x, s->stream));
  if (ev) PM_HIP(hipEventRecord(ev[1], s->stream));
  PM_HIP(pm::launch_row<T>(L, pm::ROW_ITER, tv.row, S, 1, x, s->stream));
  if (ev) PM_HIP(hipEventRecord(ev[2], s->stream));
  PM_HIP(pm::launch_reduce<T>(S, 1, pm::row_blocks<T>(L, tv.row), s->stream));
  if (green_kind(s->p) == pm::GK_CG1) {
    // CG1 is judged on the continuum divergence: the stress is transformed
    // into a second spectrum (only in iterations that evaluate the
    // indicator; the kernels return at once otherwise)
    pm::Extra<T> xs = pmh::extra<T>(0, pm::GATE_NEED_EQ, 1.0, nullptr);
    xs.spec_alt = (pm::cx<T>*)(s->ws + s->lo.spec2);
    PM_HIP(pm::launch_row<T>(L, pm::ROW_SIGFWD, 0, S, 1, xs, s->stream));
    PM_HIP(pm::launch_col<T>(L, pm::COL_FWD, 0, S, 1, xs, s->stream));
    PM_HIP(pm::launch_div_continuum<T>(S, 1, L, xs.spec_alt, s->stream));
  } else {
    PM_HIP(pm::launch_div<T>(S, 1, L, 0, s->stream));
  }
  if (ev) PM_HIP(hipEventRecord(ev[3], s->stream));
  return PM_OK;
}

// Add the event times of the timed iterations among the first `executed` of
// a finished chunk (iterations after the device halted did no work).
int collect_timing(pm_solver* s, int chunk_slot, int executed) {
  for (int i = 0; i < executed; i += s->timing_every) {
    const hipEvent_t* e = &s->tev[4 * ((size_t)chunk_slot * s->chunk + i)];
    float a = 0.f, b = 0.f, c = 0.f;
    PM_HIP(hipEventElapsedTime(&a, e[0], e[1]));
    PM_HIP(hipEventElapsedTime(&b, e[1], e[2]));
    PM_HIP(hipEventElapsedTime(&c, e[2], e[3]));
    s->tacc.col_ms += a;
    s->tacc.row_ms += b;
    s->tacc.other_ms += c;
    s->tacc.col_launches += 1;
    s->tacc.row_launches += 1;
    s->tacc.iterations += 1;
  }
  return PM_OK;
}

// Per-step outputs (strain recovered from the stored stress and tau) and the
// FP64 mean strain into the device state.
template <typename T>
int emit(pm_solver* s, pm_step_out* out) {
  pm::Extra<T> x = pmh::extra<T>(0, pm::GATE_ALL, 1.0, nullptr);
  if (out) {
    x.sig_out = (T*)out->sigma;
    x.eps_out = (T*)out->eps;
    x.plastic_out = out->plastic;
  }
  PM_HIP(pm::launch_row<T>(s->p.L, pm::ROW_EMIT, 0, dslot<T>(s), 1, x, s->stream));
  PM_HIP(pm::launch_reduce_emit<T>(dslot<T>(s), 1, pm::row_blocks<T>(s->p.L, 0), pm::GATE_ALL, s->stream));
  return PM_OK;
}

template <typename T>
int init_state(pm_solver* s, const double* E) {
  const pm::Extra<T> x = pmh::extra<T>(0, pm::GATE_ALL, 1.0, E);
  PM_HIP(pm::launch_row<T>(s->p.L, pm::ROW_INIT, 0, dslot<T>(s), 1, x, s->stream));
  return PM_OK;
}

template <typename T>
int step_impl(pm_solver* s, const double* E, pm_step_out* out) {
  const double nE = std::sqrt(E[0] * E[0] + E[1] * E[1] + 2.0 * E[2] * E[2]);
  if (!std::isfinite(nE)) return fail(PM_EINVAL, "E is not finite");
  if (nE == 0.0) {
    // Zero load: the zero field is the solution; reset the state to it.
    const double z[3] = {0.0, 0.0, 0.0};
    int rc = init_state<T>(s, z);
    if (rc != PM_OK) return rc;
    s->started = true;
    if (out && (out->sigma || out->eps || out->plastic)) {
      rc = emit<T>(s, out);
      if (rc != PM_OK) return rc;
    }
    PM_HIP(hipStreamSynchronize(s->stream));
    if (out) {
      for (int i = 0; i < 4; ++i) out->sigma_mean[i] = out->eps_mean[i] = 0.0;
      out->res_eq = out->res_mac = out->res_cmp = 0.0;
      out->iters = 0;
      out->converged = 1;
      out->status = PM_OK;
    }
    return PM_OK;
  }
  if (!s->started) {
    int rc = init_state<T>(s, E);
    if (rc != PM_OK) return rc;
    s->started = true;
  }
  PM_HIP(pm::launch_begin(s->st, E, s->p.mu, 0, 1, 0, s->stream));
  const int max_iter = s->p.max_iter;
  // Pipelined: the next chunk is queued before the previous chunk's state is
  // read.  With timing on, a chunk's events are read once its state is back;
  // the state's iteration count says how many of its iterations did work.
  int issued = 0, slot = 0, pend = -1, fin = -1;
  int chunk_n[2] = {0, 0};
  int done_iter = 0;   // iteration count at the end of the last chunk read back
  auto finish_chunk = [&](int c) -> int {
    if (s->timing) {
      int rc = collect_timing(s, c, std::min(chunk_n[c], s->hst[c].iter - done_iter));
      if (rc != PM_OK) return rc;
    }
    done_iter = s->hst[c].iter;
    return PM_OK;
  };
  while (fin < 0) {
    if (issued < max_iter) {
      const int n = std::min(s->chunk, max_iter - issued);
      for (int i = 0; i < n; ++i) {
        int rc = iterate_once<T>(s, i, slot);
        if (rc != PM_OK) return rc;
      }
      chunk_n[slot] = n;
      issued += n;
      PM_HIP(hipMemcpyAsync(&s->hst[slot], s->st, sizeof(DevState), hipMemcpyDeviceToHost, s->stream));
      PM_HIP(hipEventRecord(s->ev[slot], s->stream));
      const int prev = pend;
      pend = slot;
      slot ^= 1;
      if (prev >= 0) {
        PM_HIP(hipEventSynchronize(s->ev[prev]));
        int rc = finish_chunk(prev);
        if (rc != PM_OK) return rc;
        if (s->hst[prev].halted) fin = prev;
      }
    } else {
      PM_HIP(hipEventSynchronize(s->ev[pend]));
      int rc = finish_chunk(pend);
      if (rc != PM_OK) return rc;
      fin = pend;
    }
  }
  if (!s->hst[fin].halted) return fail(PM_EDEVICE, "device did not halt after max_iter iterations");
  // outputs and <eps> (always), then the final state
  {
    int rc = emit<T>(s, out);
    if (rc != PM_OK) return rc;
  }
  PM_HIP(hipMemcpyAsync(&s->hst[0], s->st, sizeof(DevState), hipMemcpyDeviceToHost, s->stream));
  PM_HIP(hipStreamSynchronize(s->stream));
  const DevState hs = s->hst[0];
  int rc = PM_OK;
  if (hs.status == pm::ST_NOCONV) rc = PM_ENOCONV;
  if (hs.status == pm::ST_NAN) rc = PM_ENAN;
  if (out) {
    for (int i = 0; i < 4; ++i) {
      out->sigma_mean[i] = hs.sm[i];
      out->eps_mean[i] = hs.em[i];
    }
    out->res_eq = hs.res_eq;
    out->res_mac = hs.res_mac;
    out->res_cmp = hs.res_cmp;
    out->iters = hs.iter;
    out->converged = hs.status == pm::ST_CONVERGED ? 1 : 0;
    out->status = rc;
  }
  if (rc == PM_ENOCONV) fail(rc, "load step stopped at max_iter = %d", max_iter);
  if (rc == PM_ENAN) fail(rc, "non-finite value in the reductions at iteration %d", hs.iter);
  return rc;
}

template <typename T>
int debug_forward(pm_solver* s, const void* d_real) {
  pm::Extra<T> x = pmh::extra<T>(0, pm::GATE_ALL, 1.0, nullptr);
  x.real_in = (const T*)d_real;
  PM_HIP(pm::launch_row<T>(s->p.L, pm::ROW_FWD, 0, dslot<T>(s), 1, x, s->stream));
  PM_HIP(pm::launch_col<T>(s->p.L, pm::COL_FWD, 0, dslot<T>(s), 1, x, s->stream));
  PM_HIP(hipStreamSynchronize(s->stream));
  return PM_OK;
}
template <typename T>
int debug_inverse(pm_solver* s, void* d_real) {
  pm::Extra<T> x = pmh::extra<T>(0, pm::GATE_ALL, 1.0, nullptr);
  x.real_out = (T*)d_real;
  PM_HIP(pm::launch_col<T>(s->p.L, pm::COL_INV, 0, dslot<T>(s), 1, x, s->stream));
  PM_HIP(pm::launch_row<T>(s->p.L, pm::ROW_INV, 0, dslot<T>(s), 1, x, s->stream));
  PM_HIP(hipStreamSynchronize(s->stream));
  return PM_OK;
}
template <typename T>
int debug_green(pm_solver* s, const double* E) {
  const pm::Extra<T> x = pmh::extra<T>(0, pm::GATE_ALL, 1.0, E);
  PM_HIP(pm::launch_col<T>(s->p.L, pm::col_mode(pm::COL_GREEN, green_kind(s->p)), 0, dslot<T>(s), 1, x,
                           s->stream));
  PM_HIP(hipStreamSynchronize(s->stream));
  return PM_OK;
}

}  // namespace

extern "C" {

const char* pm_status_string(int status) {
  switch (status) {
    case PM_OK: return "ok";
    case PM_EINVAL: return "invalid argument";
    case PM_EDEVICE: return "HIP device error";
    case PM_ENOCONV: return "not converged within max_iter";
    case PM_ENAN: return "non-finite value";
    case PM_EBUSY: return "busy: cannot admit now";
    default: return "unknown status";
  }
}

const char* pm_last_error(void) { return pmh::last_error(); }

int32_t pm_spectrum_tile(int32_t L, int32_t precision) {
  if (!pmh::is_pow2(L) || L < 4 || L > PM_MAX_L)
    return fail(PM_EINVAL, "L = %d must be a power of two in [4, %d]", L, PM_MAX_L);
  if (precision == PM_FP32) return pm::tile_width<float>(L);
  if (precision == PM_FP64) return pm::tile_width<double>(L);
  return fail(PM_EINVAL, "precision must be PM_FP32 or PM_FP64");
}

size_t pm_workspace_bytes(const pm_params* params) {
  pm_params q;
  if (pmh::check_params(params, &q) != PM_OK) return 0;
  return pmh::make_layout(q, true, true).total;
}

int pm_solver_create(pm_solver** out, const pm_params* params, const uint8_t* d_void_mask, void* d_workspace,
                     size_t workspace_bytes, void* stream) {
  if (!out) return fail(PM_EINVAL, "out is NULL");
  *out = nullptr;
  pm_params q;
  int rc = pmh::check_params(params, &q);
  if (rc != PM_OK) return rc;
  if (!d_void_mask || !d_workspace) return fail(PM_EINVAL, "mask and workspace must be device pointers");
  if (((uintptr_t)d_workspace) % 256 != 0) return fail(PM_EINVAL, "workspace must be 256-byte aligned");
  const Layout lo = pmh::make_layout(q, true, true);
  if (workspace_bytes < lo.total)
    return fail(PM_EINVAL, "workspace of %zu bytes is smaller than the %zu required", workspace_bytes, lo.total);
  pm_solver* s = new (std::nothrow) pm_solver();
  if (!s) return fail(PM_EDEVICE, "host allocation failed");
  s->p = q;
  s->lo = lo;
  s->stream = (hipStream_t)stream;
  s->ws = (char*)d_workspace;
  s->sig = s->ws + lo.sig;
  s->spec = s->ws + lo.spec;
  s->st = (DevState*)(s->ws + lo.state);
  s->slot = s->ws + lo.slot;
  s->started = false;
  const long L2 = (long)q.L * q.L;
  s->chunk = q.check_every > 0 ? q.check_every
                               : (int)std::max(8L, std::min(128L, (long)(1L << 27) / L2));
  auto cleanup = [&](int code) {
    if (s->hst) (void)hipHostFree(s->hst);
    for (int i = 0; i < 2; ++i)
      if (s->ev[i]) (void)hipEventDestroy(s->ev[i]);
    delete s;
    return code;
  };
  if (hipGetDevice(&s->device) != hipSuccess) return cleanup(fail(PM_EDEVICE, "hipGetDevice failed"));
  if (hipHostMalloc((void**)&s->hst, 2 * sizeof(DevState), hipHostMallocDefault) != hipSuccess)
    return cleanup(fail(PM_EDEVICE, "pinned host allocation failed"));
  memset(s->hst, 0, 2 * sizeof(DevState));
  for (int i = 0; i < 2; ++i)
    if (hipEventCreateWithFlags(&s->ev[i], hipEventDisableTiming) != hipSuccess)
      return cleanup(fail(PM_EDEVICE, "hipEventCreate failed"));
  if (hipMemsetAsync(s->st, 0, sizeof(DevState), s->stream) != hipSuccess)
    return cleanup(fail(PM_EDEVICE, "hipMemsetAsync failed"));
  rc = q.precision == PM_FP64 ? upload_tables<double>(s, d_void_mask) : upload_tables<float>(s, d_void_mask);
  if (rc != PM_OK) return cleanup(rc);
  *out = s;
  return PM_OK;
}

int pm_solver_step(pm_solver* s, const double E[3], pm_step_out* out) {
  if (!s || !E) return fail(PM_EINVAL, "solver and E must not be NULL");
  if (hipSetDevice(s->device) != hipSuccess) return fail(PM_EDEVICE, "hipSetDevice failed");
  return s->p.precision == PM_FP64 ? step_impl<double>(s, E, out) : step_impl<float>(s, E, out);
}

int pm_solver_set_max_iter(pm_solver* s, int32_t max_iter) {
  if (!s) return fail(PM_EINVAL, "NULL solver");
  if (max_iter < 1) return fail(PM_EINVAL, "max_iter = %d must be >= 1", max_iter);
  // the kernels read the limit from the slot descriptor on the device
  const size_t off = s->p.precision == PM_FP64
                         ? offsetof(pm::Slot<double>, prm) + offsetof(pm::DevParams, max_iter)
                         : offsetof(pm::Slot<float>, prm) + offsetof(pm::DevParams, max_iter);
  PM_HIP(hipMemcpyAsync((char*)s->slot + off, &max_iter, sizeof max_iter, hipMemcpyHostToDevice, s->stream));
  PM_HIP(hipStreamSynchronize(s->stream));
  s->p.max_iter = max_iter;
  return PM_OK;
}

int pm_solver_destroy(pm_solver* s) {
  if (!s) return PM_OK;
  (void)hipStreamSynchronize(s->stream);
  for (auto& e : s->tev)
    if (e) (void)hipEventDestroy(e);
  if (s->hst) (void)hipHostFree(s->hst);
  for (int i = 0; i < 2; ++i)
    if (s->ev[i]) (void)hipEventDestroy(s->ev[i]);
  delete s;
  return PM_OK;
}

int pm_solver_timing(pm_solver* s, int32_t enable, pm_kernel_timing* out) {
  if (!s) return fail(PM_EINVAL, "solver is NULL");
  if (enable < 0) return fail(PM_EINVAL, "enable must be >= 0");
  if (enable) {
    if (s->tev.empty()) {
      s->tev.resize(2 * 4 * (size_t)s->chunk, nullptr);
      for (auto& e : s->tev) PM_HIP(hipEventCreate(&e));
    }
    s->tacc = pm_kernel_timing{};
    s->timing = true;
    s->timing_every = enable;
  } else {
    s->timing = false;
  }
  if (out) *out = s->tacc;
  return PM_OK;
}

int pm_solver_buffers(pm_solver* s, void** d_eps, void** d_spectrum) {
  if (!s) return fail(PM_EINVAL, "solver is NULL");
  if (d_eps) *d_eps = s->sig;
  if (d_spectrum) *d_spectrum = s->spec;
  return PM_OK;
}


int pm_debug_forward(pm_solver* s, const void* d_real) {
  if (!s || !d_real) return fail(PM_EINVAL, "NULL argument");
  return s->p.precision == PM_FP64 ? debug_forward<double>(s, d_real) : debug_forward<float>(s, d_real);
}
int pm_debug_inverse(pm_solver* s, void* d_real) {
  if (!s || !d_real) return fail(PM_EINVAL, "NULL argument");
  return s->p.precision == PM_FP64 ? debug_inverse<double>(s, d_real) : debug_inverse<float>(s, d_real);
}
int pm_debug_green(pm_solver* s, const double E[3]) {
  if (!s || !E) return fail(PM_EINVAL, "NULL argument");
  return s->p.precision == PM_FP64 ? debug_green<double>(s, E) : debug_green<float>(s, E);
}

int pm_bernoulli_mask(uint8_t* dst, int32_t L, double f, uint64_t seed, int32_t on_device, void* stream) {
  if (!dst) return fail(PM_EINVAL, "dst is NULL");
  if (L < 1 || L > 65536) return fail(PM_EINVAL, "L = %d out of range", L);
  if (!(f >= 0.0 && f <= 1.0)) return fail(PM_EINVAL, "f = %g must be in [0, 1]", f);
  const long npx = (long)L * L;
  if (on_device) {
    PM_HIP(pm::launch_mask(dst, npx, f, seed, (hipStream_t)stream));
    PM_HIP(hipStreamSynchronize((hipStream_t)stream));
    return PM_OK;
  }
  for (long p = 0; p < npx; ++p) {
    const uint64_t z = pmh::splitmix64(seed ^ pmh::splitmix64((uint64_t)p));
    dst[p] = ((double)(z >> 11) * 0x1.0p-53) < f ? 1 : 0;
  }
  return PM_OK;
}

size_t pm_dg2_workspace_bytes(const pm_params* params) {
  pm_params q;
  if (pmh::check_params(params, &q) != PM_OK) return 0;
  return ((size_t)pm::dg2_blocks(q.L) * 16 + 16) * sizeof(double);
}

int pm_dg2_combine(const pm_params* params, const uint8_t* d_void_mask, const void* const d_eps[4],
                   const void* const d_sigma[4], void* d_workspace, size_t workspace_bytes, pm_dg2_out* out,
                   void* stream) {
  pm_params q;
  int rc = pmh::check_params(params, &q);
  if (rc != PM_OK) return rc;
  if (!d_void_mask || !d_eps || !d_workspace || !out) return fail(PM_EINVAL, "NULL argument");
  for (int v = 0; v < 4; ++v) {
    if (!d_eps[v]) return fail(PM_EINVAL, "d_eps[%d] is NULL", v);
    if (d_sigma && !d_sigma[v]) return fail(PM_EINVAL, "d_sigma[%d] is NULL", v);
  }
  const int nblk = pm::dg2_blocks(q.L);
  const size_t need = ((size_t)nblk * 16 + 16) * sizeof(double);
  if (workspace_bytes < need) return fail(PM_EINVAL, "workspace of %zu bytes is smaller than the %zu required",
                                          workspace_bytes, need);
  if (((uintptr_t)d_workspace) % 8 != 0) return fail(PM_EINVAL, "workspace must be 8-byte aligned");
  const pm::DevParams prm = pmh::dev_params(q);
  hipStream_t st = (hipStream_t)stream;
  double* part = (double*)d_workspace;
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

int pm_five_point_average(int32_t L, int32_t precision, int32_t nplanes, const void* d_in, void* d_out,
                          void* stream) {
  if (!pmh::is_pow2(L) || L < 4 || L > PM_MAX_L)
    return fail(PM_EINVAL, "L = %d must be a power of two in [4, %d]", L, PM_MAX_L);
  if (precision != PM_FP32 && precision != PM_FP64) return fail(PM_EINVAL, "precision must be PM_FP32 or PM_FP64");
  if (nplanes < 1 || nplanes > 64) return fail(PM_EINVAL, "nplanes = %d must be in [1, 64]", nplanes);
  if (!d_in || !d_out) return fail(PM_EINVAL, "NULL argument");
  if (precision == PM_FP64)
    PM_HIP(pm::launch_avg5<double>(L, nplanes, (const double*)d_in, (double*)d_out, (hipStream_t)stream));
  else
    PM_HIP(pm::launch_avg5<float>(L, nplanes, (const float*)d_in, (float*)d_out, (hipStream_t)stream));
  return PM_OK;
}

namespace {
pm_params tune_params(int32_t L, int32_t precision) {
  pm_params q{};
  q.L = L;
  q.mu = 1.0;
  q.lambda = 2.0;
  q.Y = 1.0;
  q.max_iter = 1 << 30;   // never reached: the timing run must not halt
  q.precision = precision;
  return q;
}
}  // namespace

size_t pm_autotune_workspace_bytes(int32_t L, int32_t precision) {
  const pm_params q = tune_params(L, precision);
  const size_t ws = pm_workspace_bytes(&q);
  if (ws == 0) return 0;
  return pmh::align_up(ws, 256) + (size_t)L * L;
}

int pm_set_tuning(int32_t L, int32_t precision, int32_t row_variant, int32_t col_variant) {
  if (!pmh::is_pow2(L) || L < 4 || L > PM_MAX_L) return fail(PM_EINVAL, "L = %d out of range", L);
  if (precision != PM_FP32 && precision != PM_FP64) return fail(PM_EINVAL, "precision must be PM_FP32 or PM_FP64");
  if (pm::set_tuning(precision, L, {row_variant, col_variant}) != 0)
    return fail(PM_EINVAL, "variants must be 0 or 1 (got %d, %d)", row_variant, col_variant);
  return PM_OK;
}

int pm_get_tuning(int32_t L, int32_t precision, int32_t* row_variant, int32_t* col_variant) {
  if (!pmh::is_pow2(L) || L < 4 || L > PM_MAX_L) return fail(PM_EINVAL, "L = %d out of range", L);
  if (precision != PM_FP32 && precision != PM_FP64) return fail(PM_EINVAL, "precision must be PM_FP32 or PM_FP64");
  const pm::Tuning t = pm::get_tuning(precision, L);
  if (row_variant) *row_variant = t.row;
  if (col_variant) *col_variant = t.col;
  return PM_OK;
}

int pm_autotune(int32_t L, int32_t precision, int32_t iters, void* d_workspace, size_t workspace_bytes,
                void* stream, pm_tune_result* out) {
  if (!out || !d_workspace) return fail(PM_EINVAL, "NULL argument");
  if (iters < 1 || iters > 100000) return fail(PM_EINVAL, "iters = %d must be in [1, 100000]", iters);
  const size_t need = pm_autotune_workspace_bytes(L, precision);
  if (need == 0) return fail(PM_EINVAL, "invalid L = %d or precision = %d", L, precision);
  if (workspace_bytes < need) return fail(PM_EINVAL, "workspace of %zu bytes is smaller than the %zu required",
                                          workspace_bytes, need);
  const pm_params q = tune_params(L, precision);
  const size_t ws = pmh::align_up(pm_workspace_bytes(&q), 256);
  hipStream_t st = (hipStream_t)stream;
  uint8_t* mask = (uint8_t*)d_workspace + ws;
  PM_HIP(pm::launch_mask(mask, (long)L * L, 0.2, 0x5eedull, st));
  pm_solver* s = nullptr;
  int rc = pm_solver_create(&s, &q, mask, d_workspace, ws, stream);
  if (rc != PM_OK) return rc;
  const pm::Tuning before = pm::get_tuning(precision, L);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto finish = [&](int code) {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    pm_solver_destroy(s);
    if (code != PM_OK) pm::set_tuning(precision, L, before);
    return code;
  };
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return finish(fail(PM_EDEVICE, "hipEventCreate failed"));
  const double E[3] = {0.01, 0.01, 0.005};
  rc = precision == PM_FP64 ? init_state<double>(s, E) : init_state<float>(s, E);
  if (rc != PM_OK) return finish(rc);
  if (pm::launch_begin(s->st, E, q.mu, 0, 1, 0, st) != hipSuccess) return finish(fail(PM_EDEVICE, "launch failed"));
  double best = 1e300;
  pm::Tuning pick = {0, 0};
  for (int r = 0; r < 2; ++r) {
    for (int c = 0; c < 2; ++c) {
      pm::set_tuning(precision, L, {r, c});
      for (int i = 0; i < iters + 2; ++i) {
        if (i == 2 && hipEventRecord(e0, st) != hipSuccess) return finish(fail(PM_EDEVICE, "hipEventRecord failed"));
        rc = precision == PM_FP64 ? iterate_once<double>(s, 0) : iterate_once<float>(s, 0);
        if (rc != PM_OK) return finish(rc);
      }
      if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
        return finish(fail(PM_EDEVICE, "event failed"));
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return finish(fail(PM_EDEVICE, "hipEventElapsedTime failed"));
      out->ms_per_iteration[r][c] = (double)ms / iters;
      if (out->ms_per_iteration[r][c] < best) {
        best = out->ms_per_iteration[r][c];
        pick = {r, c};
      }
    }
  }
  pm::set_tuning(precision, L, pick);
  out->row_variant = pick.row;
  out->col_variant = pick.col;
  return finish(PM_OK);
}

}  // extern "C"
