// Host-side helpers shared by the single-solver and batch C-ABI layers:
// error reporting, parameter checks, the per-realization workspace layout
// and the slot descriptor the kernels read.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdint>
#include <vector>

#include "pm.h"
#include "pm_internal.h"

namespace pmh {

// Records a formatted message as the thread's last error and returns code.
int fail(int code, const char* fmt, ...);
const char* last_error();

#define PM_HIP(call)                                                                           \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess) return pmh::fail(PM_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

inline bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }
inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Resolve defaults (reference medium 2x matrix) and validate; fills *q.
int check_params(const pm_params* p, pm_params* q);

pm::DevParams dev_params(const pm_params& q);

// Byte offsets of one realization's buffers inside its workspace.
struct Layout {
  size_t sig, spec, xbuf, tw, ktab, part, part2, state, slot, total;
  size_t spec2;   // CG1 only: the stress transform for the continuum equilibrium indicator (else 0)
  int nrow;    // row-pass blocks per slot
  int ndiv;    // doubles in part2
};

// tables = false leaves out the twiddle and momentum tables (a batch shares
// them per grid size); state = false leaves out the DevState and the slot.
Layout make_layout(const pm_params& q, bool tables, bool state);

// Twiddles exp(-2 pi i m / L) and momenta k(m) = 2 sin(q/2) exp(i q/2),
// q = 2 pi m / L, rounded from FP64 to the field precision.
template <typename T>
void make_tables(int L, std::vector<pm::cx<T>>& tw, std::vector<pm::cx<T>>& kt) {
  tw.resize(L);
  kt.resize(L);
  for (int i = 0; i < L; ++i) {
    const double a = 2.0 * M_PI * (double)i / (double)L;
    tw[i].re = (T)std::cos(a);
    tw[i].im = (T)(-std::sin(a));
    const double h = std::sin(0.5 * a);
    kt[i].re = (T)std::sin(a);                // 2 sin(q/2) cos(q/2)
    kt[i].im = (T)(2.0 * h * h);              // 2 sin(q/2) sin(q/2)
  }
}

template <typename T>
pm::Slot<T> make_slot(const pm_params& q, char* ws, const Layout& lo, const uint8_t* mask, const void* tw,
                      const void* kt, pm::DevState* st) {
  pm::Slot<T> S{};
  S.spec = (pm::cx<T>*)(ws + lo.spec);
  S.sig = (T*)(ws + lo.sig);
  S.mask = mask;
  S.part = (double*)(ws + lo.part);
  S.part2 = (double*)(ws + lo.part2);
  S.xbuf = (pm::cx<T>*)(ws + lo.xbuf);
  S.st = st;
  S.tw = (const pm::cx<T>*)tw;
  S.ktab = (const pm::cx<T>*)kt;
  S.E_path = nullptr;
  S.rec = nullptr;
  S.prm = dev_params(q);
  const int v = q.green_variant;   // sign variants 0..3; 4 and 5 take no flips
  S.flip1 = (v == 1 || v == 2) ? 1 : 0;
  S.flip2 = (v == 1 || v == 3) ? 1 : 0;
  return S;
}

template <typename T>
pm::Extra<T> extra(int use_state, int gate, double scale, const double* E) {
  pm::Extra<T> x{};
  x.use_state = use_state;
  x.gate = gate;
  x.scale = scale;
  for (int i = 0; i < 3; ++i) x.E[i] = E ? E[i] : 0.0;
  return x;
}

// Whether the iteration streams the stress state past the caches: when the
// states being iterated together exceed half the 256 MB Infinity Cache they
// cannot stay there from one pass to the next, and the non-temporal hint
// keeps them from evicting the spectrum; smaller states are left cached.
inline int stream_state(size_t state_bytes) { return state_bytes > ((size_t)128 << 20) ? 1 : 0; }

// Host mirror of the device mask generator (SplitMix64 of seed ^ SplitMix64(p)).
uint64_t splitmix64(uint64_t z);

}  // namespace pmh
