// Batch / serving engine: many realizations solved together, each advancing
// along its own load ramp on the device.  Slots of one (precision, L) group
// share every launch; the device table lists the running slots grouped by
// (precision, L) and is rebuilt on the host whenever membership changes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <vector>

#include "pm.h"
#include "pm_host.hpp"
#include "pm_internal.h"

using pm::DevState;
using pmh::fail;
using pmh::Layout;

namespace {

constexpr int NLOG = 12;                  // L = 4 .. 8192
constexpr int NGROUP = 2 * NLOG;          // (precision, log2 L)
constexpr size_t SLOT_DESC = sizeof(pm::Slot<double>);
// Streams the (precision, L) groups of a tick run on: groups do not depend on
// one another, so one group's column pass (arithmetic bound) can run beside
// another's row pass (memory bound).  Three keep one of the process's four
// hardware queues for the engine's own stream.
constexpr int NGS = 3;

int log2i(int L) {
  int k = 0;
  while ((1 << k) < L) ++k;
  return k;
}
int group_of(int precision, int L) { return (precision == PM_FP64 ? NLOG : 0) + log2i(L) - 2; }
int group_L(int g) { return 1 << (g % NLOG + 2); }
bool group_fp64(int g) { return g >= NLOG; }
size_t cx_bytes(int g) { return group_fp64(g) ? 16 : 8; }

// Offsets in the pool's fixed part.
struct Fixed {
  size_t states, table, tables[NGROUP], total;
};

Fixed fixed_layout(int max_slots) {
  Fixed f{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = pmh::align_up(off + bytes, 256);
    return o;
  };
  f.states = take((size_t)max_slots * sizeof(DevState));
  f.table = take((size_t)max_slots * SLOT_DESC);
  for (int g = 0; g < NGROUP; ++g) f.tables[g] = take(2 * (size_t)group_L(g) * cx_bytes(g));   // tw, then ktab
  f.total = off;
  return f;
}

// A slot's own range: the solver buffers (no tables, no state), then the
// ramp, the step records and the slot's own one-entry descriptor table.
struct SlotLayout {
  Layout lo;
  size_t E, rec, desc, total;
};

SlotLayout slot_layout(const pm_params& q, int nsteps) {
  SlotLayout sl{};
  sl.lo = pmh::make_layout(q, false, false);
  size_t off = sl.lo.total;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = pmh::align_up(off + bytes, 256);
    return o;
  };
  sl.E = take((size_t)nsteps * 3 * sizeof(double));
  sl.rec = take((size_t)nsteps * sizeof(pm::StepRecord));
  sl.desc = take(SLOT_DESC);
  sl.total = off;
  return sl;
}

// First-fit allocator over [begin, end) of the pool, 256-byte granules.
class RangeAlloc {
 public:
  void reset(size_t begin, size_t end) {
    free_.clear();
    if (end > begin) free_[begin] = end - begin;
  }
  bool take(size_t bytes, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t at = it->first + bytes;
        free_.erase(it);
        if (rest) free_[at] = rest;
        return true;
      }
    }
    return false;
  }
  void give(size_t off, size_t bytes) {
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t largest() const {
    size_t m = 0;
    for (auto& kv : free_) m = std::max(m, kv.second);
    return m;
  }

 private:
  std::map<size_t, size_t> free_;
};

struct HostSlot {
  bool used = false;
  bool finished = false;     // as of the last readback
  bool in_table = false;
  pm_params q{};
  int group = 0;
  int nsteps = 0;
  int hold = 0;              // PM_ADMIT_HOLD
  size_t off = 0;
  SlotLayout sl{};
  std::vector<double> E;               // host copy of the ramp (source of the upload)
  alignas(16) unsigned char desc[SLOT_DESC];   // host copy of the descriptor
  DevState st{};                       // last readback
};

}  // namespace

struct pm_batch {
  char* pool;
  size_t pool_bytes;
  int max_slots;
  hipStream_t user;          // the caller's stream
  hipStream_t stream;        // the engine's own stream (default priority), capturable
  hipStream_t gstream[NGS];  // group streams (default priority), forked from and joined to `stream`
  hipEvent_t fork_ev, join_ev[NGS];
  hipEvent_t ev_user;        // orders the engine's work after the caller's
  int device;
  Fixed fx;
  RangeAlloc heap;
  std::vector<HostSlot> slots;
  bool tables_ready[NGROUP];
  // device table: running slots grouped by (precision, L)
  bool dirty;
  int grp_begin[NGROUP], grp_count[NGROUP];
  size_t table_state_bytes;  // stress states of the slots in the table (all groups)
  unsigned char* stage;      // pinned copy of the table being uploaded
  DevState* hstates;         // pinned readback of the slot states
  hipEvent_t stage_done;
  int hi;                    // 1 + highest slot id in use
  // a tick's launches are captured into a graph once the table has run eagerly
  bool use_graph;
  uint64_t table_version;    // bumped by every table upload
  uint64_t eager_version;    // table version of the last eager tick
  uint64_t graph_version;    // table version, iteration count and tuning the graph holds
  int graph_iters;
  uint64_t graph_tuning;
  uint64_t eager_tuning;
  hipGraphExec_t gexec;
};

namespace {

DevState* dev_state(pm_batch* b, int i) { return (DevState*)(b->pool + b->fx.states) + i; }

template <typename T>
const pm::Slot<T>* dev_table(pm_batch* b, int g) {
  return (const pm::Slot<T>*)(b->pool + b->fx.table) + b->grp_begin[g];
}

template <typename T>
const pm::Slot<T>* own_desc(pm_batch* b, int i) {
  return (const pm::Slot<T>*)(b->pool + b->slots[i].off + b->slots[i].sl.desc);
}

int upload_group_tables(pm_batch* b, int g) {
  if (b->tables_ready[g]) return PM_OK;
  const int L = group_L(g);
  char* base = b->pool + b->fx.tables[g];
  if (group_fp64(g)) {
    std::vector<pm::cx<double>> tw, kt;
    pmh::make_tables<double>(L, tw, kt);
    PM_HIP(hipMemcpyAsync(base, tw.data(), L * sizeof(tw[0]), hipMemcpyHostToDevice, b->stream));
    PM_HIP(hipMemcpyAsync(base + L * sizeof(tw[0]), kt.data(), L * sizeof(kt[0]), hipMemcpyHostToDevice, b->stream));
    PM_HIP(hipStreamSynchronize(b->stream));
  } else {
    std::vector<pm::cx<float>> tw, kt;
    pmh::make_tables<float>(L, tw, kt);
    PM_HIP(hipMemcpyAsync(base, tw.data(), L * sizeof(tw[0]), hipMemcpyHostToDevice, b->stream));
    PM_HIP(hipMemcpyAsync(base + L * sizeof(tw[0]), kt.data(), L * sizeof(kt[0]), hipMemcpyHostToDevice, b->stream));
    PM_HIP(hipStreamSynchronize(b->stream));
  }
  b->tables_ready[g] = true;
  return PM_OK;
}

// Rebuild the device table from the slots that are used and not finished.
int rebuild_table(pm_batch* b) {
  if (!b->dirty) return PM_OK;
  PM_HIP(hipEventSynchronize(b->stage_done));   // the previous upload has left the stage
  int n = 0;
  size_t state_bytes = 0;
  for (int i = 0; i < b->max_slots; ++i) b->slots[i].in_table = false;
  for (int g = 0; g < NGROUP; ++g) {
    b->grp_begin[g] = n;
    for (int i = 0; i < b->hi; ++i) {
      HostSlot& h = b->slots[i];
      if (!h.used || h.finished || h.group != g) continue;
      h.in_table = true;
      memcpy(b->stage + (size_t)n * SLOT_DESC, h.desc, SLOT_DESC);
      state_bytes += (size_t)h.q.L * h.q.L * 4 * (h.q.precision == PM_FP64 ? 8 : 4);
      ++n;
    }
    b->grp_count[g] = n - b->grp_begin[g];
  }
  b->table_state_bytes = state_bytes;
  if (n > 0)
    PM_HIP(hipMemcpyAsync(b->pool + b->fx.table, b->stage, (size_t)n * SLOT_DESC, hipMemcpyHostToDevice, b->stream));
  PM_HIP(hipEventRecord(b->stage_done, b->stream));
  b->dirty = false;
  ++b->table_version;
  return PM_OK;
}

// A part of a group's table: slots [first, first + n) of group g.
struct Part {
  int g, first, n;
};

template <typename T>
int iterate_group(pm_batch* b, const Part& pt, hipStream_t st) {
  const int g = pt.g, L = group_L(g), n = pt.n;
  const pm::Slot<T>* tab = dev_table<T>(b, g) + pt.first;
  pm::Extra<T> x = pmh::extra<T>(1, pm::GATE_RUNNING, 1.0 / ((double)L * (double)L), nullptr);
  // the states of every group share the caches, so the policy follows their total
  x.stream_state = pmh::stream_state(b->table_state_bytes);
  const pm::Tuning tv = pm::get_tuning(group_fp64(g) ? PM_FP64 : PM_FP32, L);
  PM_HIP(pm::launch_col<T>(L, pm::COL_ALL, tv.col, tab, n, x, st));
  PM_HIP(pm::launch_row<T>(L, pm::ROW_ITER, tv.row, tab, n, x, st));
  PM_HIP(pm::launch_reduce<T>(tab, n, pm::row_blocks<T>(L, tv.row), st));
  PM_HIP(pm::launch_div<T>(tab, n, L, 0, st));
  return PM_OK;
}

// Output pass and record for slots whose step ended, then the next step.
template <typename T>
int finish_group(pm_batch* b, const Part& pt, hipStream_t st) {
  const int g = pt.g, L = group_L(g), n = pt.n;
  const pm::Slot<T>* tab = dev_table<T>(b, g) + pt.first;
  const pm::Extra<T> x = pmh::extra<T>(0, pm::GATE_PENDING, 1.0, nullptr);
  PM_HIP(pm::launch_row<T>(L, pm::ROW_EMIT, 0, tab, n, x, st));
  PM_HIP(pm::launch_reduce_emit<T>(tab, n, pm::row_blocks<T>(L, 0), pm::GATE_PENDING, st));
  PM_HIP(pm::launch_advance<T>(tab, n, st));
  return PM_OK;
}

// Order the engine's stream after the work already queued on the caller's.
int sync_in(pm_batch* b) {
  PM_HIP(hipEventRecord(b->ev_user, b->user));
  PM_HIP(hipStreamWaitEvent(b->stream, b->ev_user, 0));
  return PM_OK;
}

// All launches of one tick: iters iterations of every group, then the end of
// the load steps that finished.  Each group runs on a group stream forked
// from the engine's stream (groups share no data, and every slot's work
// stays in order on its group's stream); the engine's stream joins them
// all at the end, so the tick is one unit for the caller and for a graph.
int tick_launches(pm_batch* b, int iters) {
  int active[NGROUP], na = 0;
  for (int g = 0; g < NGROUP; ++g)
    if (b->grp_count[g]) active[na++] = g;
  // one part per group: splitting a lone group's table over the streams
  // (the four DG2 variants at L = 1024) measured 15 % slower than one launch
  // covering all of its slots
  Part parts[NGROUP];
  int np = 0;
  for (int a = 0; a < na; ++a) parts[np++] = {active[a], 0, b->grp_count[active[a]]};
  const int ns = std::min(np, NGS);
  if (ns > 0) PM_HIP(hipEventRecord(b->fork_ev, b->stream));
  for (int k = 0; k < ns; ++k) PM_HIP(hipStreamWaitEvent(b->gstream[k], b->fork_ev, 0));
  for (int a = 0; a < np; ++a) {
    const Part& pt = parts[a];
    hipStream_t st = b->gstream[a % NGS];
    for (int it = 0; it < iters; ++it) {
      int rc = group_fp64(pt.g) ? iterate_group<double>(b, pt, st) : iterate_group<float>(b, pt, st);
      if (rc != PM_OK) return rc;
    }
    int rc = group_fp64(pt.g) ? finish_group<double>(b, pt, st) : finish_group<float>(b, pt, st);
    if (rc != PM_OK) return rc;
  }
  for (int k = 0; k < ns; ++k) {
    PM_HIP(hipEventRecord(b->join_ev[k], b->gstream[k]));
    PM_HIP(hipStreamWaitEvent(b->stream, b->join_ev[k], 0));
  }
  return PM_OK;
}

int drop_graph(pm_batch* b) {
  if (b->gexec) {
    PM_HIP(hipGraphExecDestroy(b->gexec));
    b->gexec = nullptr;
  }
  return PM_OK;
}

// Capture the tick's launches on the engine's stream and instantiate them.
int capture_tick(pm_batch* b, int iters) {
  int rc = drop_graph(b);
  if (rc != PM_OK) return rc;
  PM_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  rc = tick_launches(b, iters);
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(b->stream, &graph);
  if (rc != PM_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (e != hipSuccess) return fail(PM_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
  const hipError_t ei = hipGraphInstantiate(&b->gexec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ei != hipSuccess) {
    b->gexec = nullptr;
    return fail(PM_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(ei));
  }
  b->graph_version = b->table_version;
  b->graph_iters = iters;
  b->graph_tuning = pm::tuning_generation();
  return PM_OK;
}

template <typename T>
int admit_impl(pm_batch* b, int i, const uint8_t* mask) {
  HostSlot& h = b->slots[i];
  char* region = b->pool + h.off;
  const char* tabs = b->pool + b->fx.tables[h.group];
  const int L = h.q.L;
  pm::Slot<T> S = pmh::make_slot<T>(h.q, region, h.sl.lo, mask, tabs, tabs + L * sizeof(pm::cx<T>),
                                    dev_state(b, i));
  S.E_path = (const double*)(region + h.sl.E);
  S.rec = (pm::StepRecord*)(region + h.sl.rec);
  memcpy(h.desc, &S, SLOT_DESC);
  PM_HIP(hipMemcpyAsync(region + h.sl.E, h.E.data(), h.E.size() * sizeof(double), hipMemcpyHostToDevice, b->stream));
  PM_HIP(hipMemcpyAsync(region + h.sl.desc, h.desc, SLOT_DESC, hipMemcpyHostToDevice, b->stream));
  PM_HIP(pm::launch_begin(dev_state(b, i), h.E.data(), h.q.mu, 0, h.nsteps, h.hold, b->stream));
  // uniform start at E_1 (the state's E), as the first step of a solver
  const pm::Extra<T> x = pmh::extra<T>(1, pm::GATE_ALL, 1.0, nullptr);
  PM_HIP(pm::launch_row<T>(L, pm::ROW_INIT, 0, own_desc<T>(b, i), 1, x, b->stream));
  // the host copies above come from memory that stays alive with the slot;
  // wait so that a failure is reported here
  PM_HIP(hipStreamSynchronize(b->stream));
  return PM_OK;
}

template <typename T>
int fetch_impl(pm_batch* b, int i, pm_step_out* out) {
  const HostSlot& h = b->slots[i];
  pm::Extra<T> x = pmh::extra<T>(0, pm::GATE_ALL, 1.0, nullptr);
  x.sig_out = (T*)out->sigma;
  x.eps_out = (T*)out->eps;
  x.plastic_out = out->plastic;
  PM_HIP(pm::launch_row<T>(h.q.L, pm::ROW_EMIT, 0, own_desc<T>(b, i), 1, x, b->stream));
  PM_HIP(pm::launch_reduce_emit<T>(own_desc<T>(b, i), 1, pm::row_blocks<T>(h.q.L, 0), pm::GATE_ALL, b->stream));
  PM_HIP(hipMemcpyAsync(&b->hstates[i], dev_state(b, i), sizeof(DevState), hipMemcpyDeviceToHost, b->stream));
  PM_HIP(hipStreamSynchronize(b->stream));
  const DevState& st = b->hstates[i];
  for (int c = 0; c < 4; ++c) {
    out->sigma_mean[c] = st.sm[c];
    out->eps_mean[c] = st.em[c];
  }
  out->res_eq = st.res_eq;
  out->res_mac = st.res_mac;
  out->res_cmp = st.res_cmp;
  out->iters = st.iter;
  out->converged = st.status == pm::ST_CONVERGED ? 1 : 0;
  out->status = st.status == pm::ST_NOCONV ? PM_ENOCONV : st.status == pm::ST_NAN ? PM_ENAN : PM_OK;
  return PM_OK;
}

int check_slot(pm_batch* b, int32_t slot) {
  if (!b) return fail(PM_EINVAL, "batch is NULL");
  if (slot < 0 || slot >= b->max_slots || !b->slots[slot].used) return fail(PM_EINVAL, "slot %d is not in use", slot);
  return PM_OK;
}

int steps_done(const HostSlot& h) {
  if (h.st.finished || h.st.held) return h.st.step + 1;
  return h.st.step;
}

}  // namespace

extern "C" {

size_t pm_batch_overhead_bytes(int32_t max_slots) {
  if (max_slots < 1 || max_slots > 65536) return 0;
  return fixed_layout(max_slots).total;
}

size_t pm_batch_slot_bytes(const pm_params* params, int32_t nsteps) {
  pm_params q;
  if (nsteps < 1 || pmh::check_params(params, &q) != PM_OK) return 0;
  return slot_layout(q, nsteps).total;
}

int pm_batch_create(pm_batch** out, void* d_pool, size_t pool_bytes, int32_t max_slots, void* stream) {
  if (!out) return fail(PM_EINVAL, "out is NULL");
  *out = nullptr;
  if (!d_pool) return fail(PM_EINVAL, "pool is NULL");
  if (((uintptr_t)d_pool) % 256 != 0) return fail(PM_EINVAL, "pool must be 256-byte aligned");
  if (max_slots < 1 || max_slots > 65536) return fail(PM_EINVAL, "max_slots = %d must be in [1, 65536]", max_slots);
  const Fixed fx = fixed_layout(max_slots);
  if (pool_bytes < fx.total)
    return fail(PM_EINVAL, "pool of %zu bytes is smaller than the fixed part (%zu bytes)", pool_bytes, fx.total);
  pm_batch* b = new (std::nothrow) pm_batch();
  if (!b) return fail(PM_EDEVICE, "host allocation failed");
  b->pool = (char*)d_pool;
  b->pool_bytes = pool_bytes;
  b->max_slots = max_slots;
  b->user = (hipStream_t)stream;
  b->fx = fx;
  b->heap.reset(fx.total, pool_bytes / 256 * 256);
  b->slots.resize(max_slots);
  for (int g = 0; g < NGROUP; ++g) {
    b->tables_ready[g] = false;
    b->grp_begin[g] = b->grp_count[g] = 0;
  }
  b->dirty = true;
  b->hi = 0;
  b->use_graph = true;
  b->table_version = 1;
  b->eager_version = 0;
  b->graph_version = 0;
  b->graph_iters = 0;
  b->graph_tuning = 0;
  b->eager_tuning = 0;
  b->gexec = nullptr;
  auto cleanup = [&](int code) {
    if (b->stage) (void)hipHostFree(b->stage);
    if (b->hstates) (void)hipHostFree(b->hstates);
    if (b->stage_done) (void)hipEventDestroy(b->stage_done);
    if (b->ev_user) (void)hipEventDestroy(b->ev_user);
    if (b->fork_ev) (void)hipEventDestroy(b->fork_ev);
    for (int k = 0; k < NGS; ++k) {
      if (b->join_ev[k]) (void)hipEventDestroy(b->join_ev[k]);
      if (b->gstream[k]) (void)hipStreamDestroy(b->gstream[k]);
    }
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return code;
  };
  if (hipGetDevice(&b->device) != hipSuccess) return cleanup(fail(PM_EDEVICE, "hipGetDevice failed"));
  if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess)
    return cleanup(fail(PM_EDEVICE, "hipStreamCreate failed"));
  if (hipEventCreateWithFlags(&b->ev_user, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b->fork_ev, hipEventDisableTiming) != hipSuccess)
    return cleanup(fail(PM_EDEVICE, "hipEventCreate failed"));
  for (int k = 0; k < NGS; ++k) {
    if (hipStreamCreateWithFlags(&b->gstream[k], hipStreamNonBlocking) != hipSuccess)
      return cleanup(fail(PM_EDEVICE, "hipStreamCreate failed"));
    if (hipEventCreateWithFlags(&b->join_ev[k], hipEventDisableTiming) != hipSuccess)
      return cleanup(fail(PM_EDEVICE, "hipEventCreate failed"));
  }
  if (hipHostMalloc((void**)&b->stage, (size_t)max_slots * SLOT_DESC, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&b->hstates, (size_t)max_slots * sizeof(DevState), hipHostMallocDefault) != hipSuccess)
    return cleanup(fail(PM_EDEVICE, "pinned host allocation failed"));
  memset(b->hstates, 0, (size_t)max_slots * sizeof(DevState));
  if (hipEventCreateWithFlags(&b->stage_done, hipEventDisableTiming) != hipSuccess)
    return cleanup(fail(PM_EDEVICE, "hipEventCreate failed"));
  if (hipEventRecord(b->stage_done, b->stream) != hipSuccess) return cleanup(fail(PM_EDEVICE, "hipEventRecord failed"));
  *out = b;
  return PM_OK;
}

int pm_batch_admit(pm_batch* b, const pm_params* params, const uint8_t* d_void_mask, int32_t nsteps,
                   const double* E_path, int32_t flags, int32_t* slot) {
  if (!b || !slot) return fail(PM_EINVAL, "batch and slot must not be NULL");
  *slot = -1;
  if (flags & ~PM_ADMIT_HOLD) return fail(PM_EINVAL, "unknown admission flags 0x%x", flags);
  pm_params q;
  int rc = pmh::check_params(params, &q);
  if (rc != PM_OK) return rc;
  if (!d_void_mask || !E_path) return fail(PM_EINVAL, "mask and E_path must not be NULL");
  if (q.green_variant > 3) return fail(PM_EINVAL, "green_variant %d (DG1 / CG1) runs in the single solver only",
                                       q.green_variant);
  if (nsteps < 1) return fail(PM_EINVAL, "nsteps = %d must be >= 1", nsteps);
  for (int n = 0; n < nsteps; ++n) {
    const double* e = E_path + 3 * n;
    const double nE = std::sqrt(e[0] * e[0] + e[1] * e[1] + 2.0 * e[2] * e[2]);
    if (!std::isfinite(nE) || nE == 0.0) return fail(PM_EINVAL, "E_path step %d must be finite and nonzero", n);
  }
  int i = -1;
  for (int k = 0; k < b->max_slots; ++k)
    if (!b->slots[k].used) {
      i = k;
      break;
    }
  if (i < 0) return fail(PM_EBUSY, "all %d slots are in use", b->max_slots);
  const SlotLayout sl = slot_layout(q, nsteps);
  size_t off = 0;
  if (!b->heap.take(sl.total, &off))
    return fail(PM_EBUSY, "no free pool range of %zu bytes (largest free %zu)", sl.total, b->heap.largest());
  const int g = group_of(q.precision, q.L);
  rc = sync_in(b);
  if (rc != PM_OK) {
    b->heap.give(off, sl.total);
    return rc;
  }
  rc = upload_group_tables(b, g);
  if (rc != PM_OK) {
    b->heap.give(off, sl.total);
    return rc;
  }
  HostSlot& h = b->slots[i];
  h.used = true;
  h.finished = false;
  h.in_table = false;
  h.q = q;
  h.group = g;
  h.nsteps = nsteps;
  h.hold = (flags & PM_ADMIT_HOLD) ? 1 : 0;
  h.off = off;
  h.sl = sl;
  h.E.assign(E_path, E_path + 3 * (size_t)nsteps);
  memset(&h.st, 0, sizeof h.st);
  h.st.nsteps = nsteps;
  rc = q.precision == PM_FP64 ? admit_impl<double>(b, i, d_void_mask) : admit_impl<float>(b, i, d_void_mask);
  if (rc != PM_OK) {
    h.used = false;
    b->heap.give(off, sl.total);
    return rc;
  }
  b->hi = std::max(b->hi, i + 1);
  b->dirty = true;
  *slot = i;
  return PM_OK;
}

int pm_batch_tick(pm_batch* b, int32_t iters, int32_t* running) {
  if (!b) return fail(PM_EINVAL, "batch is NULL");
  if (iters < 1) return fail(PM_EINVAL, "iters = %d must be >= 1", iters);
  if (hipSetDevice(b->device) != hipSuccess) return fail(PM_EDEVICE, "hipSetDevice failed");
  int rc = sync_in(b);
  if (rc != PM_OK) return rc;
  rc = rebuild_table(b);
  if (rc != PM_OK) return rc;
  const uint64_t tgen = pm::tuning_generation();
  if (b->use_graph && b->eager_version == b->table_version && b->eager_tuning == tgen) {
    // the table ran eagerly once with this tuning (kernel attributes set): replay a graph
    if (!b->gexec || b->graph_version != b->table_version || b->graph_iters != iters || b->graph_tuning != tgen) {
      rc = capture_tick(b, iters);
      if (rc != PM_OK) return rc;
    }
    PM_HIP(hipGraphLaunch(b->gexec, b->stream));
  } else {
    rc = tick_launches(b, iters);
    if (rc != PM_OK) return rc;
    b->eager_version = b->table_version;
    b->eager_tuning = tgen;
  }
  if (b->hi > 0)
    PM_HIP(hipMemcpyAsync(b->hstates, b->pool + b->fx.states, (size_t)b->hi * sizeof(DevState),
                          hipMemcpyDeviceToHost, b->stream));
  PM_HIP(hipStreamSynchronize(b->stream));
  int nrun = 0;
  for (int i = 0; i < b->hi; ++i) {
    HostSlot& h = b->slots[i];
    if (!h.used || !h.in_table) {
      if (h.used && !h.finished) ++nrun;
      continue;
    }
    h.st = b->hstates[i];
    if (h.st.finished) {
      h.finished = true;
      b->dirty = true;
    } else {
      ++nrun;
    }
  }
  if (running) *running = nrun;
  return PM_OK;
}

int pm_batch_poll(pm_batch* b, int32_t slot, pm_slot_info* info) {
  int rc = check_slot(b, slot);
  if (rc != PM_OK) return rc;
  if (!info) return fail(PM_EINVAL, "info is NULL");
  const HostSlot& h = b->slots[slot];
  info->L = h.q.L;
  info->precision = h.q.precision;
  info->nsteps = h.nsteps;
  info->steps_done = steps_done(h);
  info->finished = h.finished ? 1 : 0;
  info->last_status = info->steps_done > 0 ? h.st.status : 0;
  info->held = (!h.finished && h.st.held) ? 1 : 0;
  return PM_OK;
}

int pm_batch_resume(pm_batch* b, int32_t slot) {
  int rc = check_slot(b, slot);
  if (rc != PM_OK) return rc;
  HostSlot& h = b->slots[slot];
  if (h.finished || !h.st.held) return fail(PM_EINVAL, "slot %d is not waiting after a load step", slot);
  const int next = h.st.step + 1;
  if (hipSetDevice(b->device) != hipSuccess) return fail(PM_EDEVICE, "hipSetDevice failed");
  rc = sync_in(b);
  if (rc != PM_OK) return rc;
  PM_HIP(pm::launch_begin(dev_state(b, slot), h.E.data() + 3 * (size_t)next, h.q.mu, next, h.nsteps, h.hold,
                          b->stream));
  h.st.held = 0;
  h.st.step = next;
  return PM_OK;
}

int pm_batch_records(pm_batch* b, int32_t slot, int32_t first, int32_t count, pm_step_record* out) {
  int rc = check_slot(b, slot);
  if (rc != PM_OK) return rc;
  const HostSlot& h = b->slots[slot];
  if (count < 0 || first < 0 || first + count > steps_done(h))
    return fail(PM_EINVAL, "records %d..%d requested, %d available", first, first + count - 1, steps_done(h));
  if (count == 0) return PM_OK;
  if (!out) return fail(PM_EINVAL, "out is NULL");
  PM_HIP(hipMemcpyAsync(out, b->pool + h.off + h.sl.rec + (size_t)first * sizeof(pm::StepRecord),
                        (size_t)count * sizeof(pm::StepRecord), hipMemcpyDeviceToHost, b->stream));
  PM_HIP(hipStreamSynchronize(b->stream));
  return PM_OK;
}

int pm_batch_fetch(pm_batch* b, int32_t slot, pm_step_out* out) {
  int rc = check_slot(b, slot);
  if (rc != PM_OK) return rc;
  if (!out) return fail(PM_EINVAL, "out is NULL");
  if (hipSetDevice(b->device) != hipSuccess) return fail(PM_EDEVICE, "hipSetDevice failed");
  rc = sync_in(b);
  if (rc != PM_OK) return rc;
  return b->slots[slot].q.precision == PM_FP64 ? fetch_impl<double>(b, slot, out) : fetch_impl<float>(b, slot, out);
}

int pm_batch_release(pm_batch* b, int32_t slot) {
  int rc = check_slot(b, slot);
  if (rc != PM_OK) return rc;
  // queued work may still read the slot's range
  PM_HIP(hipStreamSynchronize(b->stream));
  HostSlot& h = b->slots[slot];
  b->heap.give(h.off, h.sl.total);
  if (h.in_table) b->dirty = true;
  h = HostSlot();
  // a released slot id stays halted on the device until it is admitted again
  DevState halted{};
  halted.halted = 1;
  halted.finished = 1;
  PM_HIP(hipMemcpyAsync(dev_state(b, slot), &halted, sizeof halted, hipMemcpyHostToDevice, b->stream));
  PM_HIP(hipStreamSynchronize(b->stream));
  while (b->hi > 0 && !b->slots[b->hi - 1].used) --b->hi;
  return PM_OK;
}

int pm_batch_set_graphs(pm_batch* b, int32_t enable) {
  if (!b) return fail(PM_EINVAL, "batch is NULL");
  b->use_graph = enable != 0;
  if (!b->use_graph) return drop_graph(b);
  return PM_OK;
}

int pm_batch_destroy(pm_batch* b) {
  if (!b) return PM_OK;
  (void)hipStreamSynchronize(b->stream);
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->ev_user) (void)hipEventDestroy(b->ev_user);
  if (b->fork_ev) (void)hipEventDestroy(b->fork_ev);
  for (int k = 0; k < NGS; ++k) {
    if (b->gstream[k]) {
      (void)hipStreamSynchronize(b->gstream[k]);
      (void)hipStreamDestroy(b->gstream[k]);
    }
    if (b->join_ev[k]) (void)hipEventDestroy(b->join_ev[k]);
  }
  if (b->stream) (void)hipStreamDestroy(b->stream);
  if (b->stage) (void)hipHostFree(b->stage);
  if (b->hstates) (void)hipHostFree(b->hstates);
  if (b->stage_done) (void)hipEventDestroy(b->stage_done);
  delete b;
  return PM_OK;
}

}  // extern "C"
