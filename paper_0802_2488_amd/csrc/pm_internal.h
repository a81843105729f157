// Internal device/host interface between the C-ABI layer and the kernels.
//
// Every kernel works on a table of "slots": one slot is one realization
// (mask, state, half spectrum, partial sums) solved on the device.  A launch
// covers all slots of one grid size L; block b works on slot b / bps
// (bps = blocks per slot).  A single solver is a table of one slot.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pm_fft.hpp"

namespace pm {

enum RowMode { ROW_ITER = 0, ROW_INIT = 1, ROW_FWD = 2, ROW_INV = 3, ROW_EMIT = 4, ROW_SIGFWD = 5 };
enum ColMode { COL_FWD = 1, COL_GREEN = 2, COL_INV = 4, COL_ALL = 7 };
// Green tensor of the column pass, in bits 8.. of the column mode: the sign
// variants of eq. 3 (slot flips), DG1 (symmetrised) or CG1 (continuum).
enum GreenKind { GK_SIGN = 0, GK_DG1 = 1, GK_CG1 = 2 };
constexpr int col_mode(int mode, int kind) { return mode | (kind << 8); }
enum Status { ST_RUNNING = 0, ST_CONVERGED = 1, ST_NOCONV = 2, ST_NAN = 3 };

constexpr int NPART = 8;    // doubles per block in the row-pass partials
constexpr int NSUM = 6;     // sigma 11, 22, 33, 12; |e - eps|^2; plastic pixels

// Result of one load step, written by the device.  Same layout as the
// public pm_step_record.
struct StepRecord {
  double sm[4];                // <sigma> (11, 22, 33, 12)
  double em[4];                // <eps>
  double res_eq, res_mac, res_cmp;
  double plastic;              // fraction of pixels on the capped branch
  int32_t iters, status;       // status: ST_CONVERGED / ST_NOCONV / ST_NAN
};

// Convergence state of one slot, resident on the device.
struct DevState {
  double E[4];                 // E11, E22, E12 of the current load step
  double sm[4], sm_prev[4];    // <sigma> (11, 22, 33, 12), current and previous iteration
  double em[4];                // <eps> (output pass)
  double res_eq, res_mac, res_cmp;
  double normE, floor_s;       // |E| and the floor of the stress normalisation
  double plastic;              // plastic fraction of the last iteration
  int32_t iter, halted, status;
  int32_t need_eq;             // 1: test equilibrium; 2: evaluate it for the record at max_iter
  int32_t step, nsteps;        // load-ramp position when the device advances steps itself
  int32_t finished;            // all steps of the ramp done
  int32_t pending;             // a step ended; its record waits for the output pass
  int32_t hold;                // wait after every step until the host resumes the slot
  int32_t held;                // waiting (step ended, record complete, next step not begun)
  uint32_t div_ticket;         // blocks of the residual pass done (0 between passes)
};

struct DevParams {
  double mu, lam, Y, mu0, lam0, K, K0;
  double sy;
  double npx;
  double eta_eq, eta_mac, eta_cmp;
  int32_t max_iter, L;
};

// One realization as seen by the kernels.
template <typename T>
struct Slot {
  cx<T>* spec;           // half spectrum (tiled, packed)
  T* sig;                // state: stress of the last iterate (= multiplier), 4 components per pixel
  const uint8_t* mask;   // 1 = void
  double* part;          // per-block partial sums of the row pass (NPART each)
  double* part2;         // residual and output-pass partial sums
  cx<T>* xbuf;           // 3 L values: transform of the packed column 0
  DevState* st;
  const cx<T>* tw;       // twiddles exp(-2 pi i m / L)
  const cx<T>* ktab;     // momenta k(m) = 2 sin(q/2) exp(i q/2)
  const double* E_path;  // device ramp (nsteps x 3) when steps advance on the device, else null
  StepRecord* rec;       // per-step records (nsteps), or null
  DevParams prm;
  int32_t flip1, flip2;  // Green tensor evaluated at -q1 / -q2
  int32_t pad[2];
};

// Which slots of a table a launch works on (GATE_NEED_EQ: running slots
// whose equilibrium indicator is due this iteration).
enum Gate { GATE_ALL = 0, GATE_RUNNING = 1, GATE_PENDING = 2, GATE_NEED_EQ = 3 };

// Extra arguments of the check and output modes.
template <typename T>
struct Extra {
  const T* real_in;      // ROW_FWD: 3 planes
  T* real_out;           // ROW_INV: 3 planes
  T* sig_out;            // ROW_EMIT outputs (may be null)
  T* eps_out;
  uint8_t* plastic_out;
  double E[3];           // ROW_INIT / COL_GREEN when use_state = 0: mean strain
  double scale;          // Green-tensor output scale (1/L^2 in the iteration)
  int32_t use_state;     // 1: E from the slot state
  int32_t gate;          // Gate: skip halted slots, or slots without a pending record
  int32_t stream_state;  // ROW_ITER: stress state loaded and stored with the non-temporal hint
  cx<T>* spec_alt;       // ROW_SIGFWD / column transforms: this spectrum instead of the slot's
};

template <typename T>
__device__ __forceinline__ bool gated_out(const Extra<T>& x, const DevState* st_generic) {
  gptr<const DevState> st = glb(st_generic);
  return (x.gate == GATE_RUNNING && st->halted) || (x.gate == GATE_PENDING && !st->pending) ||
         (x.gate == GATE_NEED_EQ && (st->halted || !st->need_eq));
}

// variant: 0 default, 1 the autotuner's alternative; it applies to ROW_ITER
// and COL_ALL (any Green kind), other modes run variant 0.
template <typename T>
hipError_t launch_row(int L, int mode, int variant, const Slot<T>* slots, int nslots, const Extra<T>& x,
                      hipStream_t st);
template <typename T>
hipError_t launch_col(int L, int mode, int variant, const Slot<T>* slots, int nslots, const Extra<T>& x,
                      hipStream_t st);
template <typename T>
int row_blocks(int L, int variant);   // blocks per slot of the row pass

// Process-wide choice of the iteration-kernel variants per (precision, L);
// the generation changes with every update.
struct Tuning {
  int row, col;
};
Tuning get_tuning(int precision, int L);
int set_tuning(int precision, int L, Tuning t);
uint64_t tuning_generation();
template <typename T>
int tile_width(int L);
int div_blocks(int L);      // blocks per slot of the residual pass
template <typename T>
hipError_t launch_reduce(const Slot<T>* slots, int nslots, int nblk, hipStream_t s);
template <typename T>
hipError_t launch_div(const Slot<T>* slots, int nslots, int L, int force, hipStream_t s);
template <typename T>
hipError_t launch_div_continuum(const Slot<T>* slots, int nslots, int L, const cx<T>* spec, hipStream_t s);
template <typename T>
hipError_t launch_reduce_emit(const Slot<T>* slots, int nslots, int nblk, int gate, hipStream_t s);
template <typename T>
hipError_t launch_advance(const Slot<T>* slots, int nslots, hipStream_t s);
hipError_t launch_begin(DevState* st, const double* E, double mu, int32_t step, int32_t nsteps, int32_t hold,
                        hipStream_t s);
template <typename T>
hipError_t launch_dg2(int L, const DevParams& prm, const uint8_t* mask, const T* const* eps4, const T* const* sig4,
                      T* eps_out, T* soa_out, T* sav_out, uint8_t* pl_out, double* partials, int nblk,
                      hipStream_t s);
int dg2_blocks(int L);
template <typename T>
hipError_t launch_avg5(int L, int nplanes, const T* in, T* out, hipStream_t s);
hipError_t launch_mask(uint8_t* out, long npx, double f, uint64_t seed, hipStream_t s);

}  // namespace pm
