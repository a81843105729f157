// Internal device/host interface between the C-ABI layer and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pm_fft.hpp"

namespace pm {

enum RowMode { ROW_ITER = 0, ROW_INIT = 1, ROW_FWD = 2, ROW_INV = 3, ROW_EMIT = 4 };
enum ColMode { COL_FWD = 1, COL_GREEN = 2, COL_INV = 4, COL_ALL = 7 };
enum Status { ST_RUNNING = 0, ST_CONVERGED = 1, ST_NOCONV = 2, ST_NAN = 3 };

constexpr int NPART = 16;   // doubles per block in the row-pass partials

// Convergence state of one solve, resident on the device.
struct DevState {
  double E[4];                 // E11, E22, E12 of the current load step
  double sm[4], sm_prev[4];    // <sigma> (11, 22, 33, 12), current and previous iteration
  double em[4];                // <eps>
  double res_eq, res_mac, res_cmp;
  double normE, floor_s;       // |E| and the floor of the stress normalisation
  int32_t iter, halted, status, need_eq;
  int32_t pad[4];
};

struct DevParams {
  double mu, lam, Y, mu0, lam0, K, K0;
  double sy;
  double npx;
  double eta_eq, eta_mac, eta_cmp;
  int32_t max_iter, L;
};

template <typename T>
struct RowArgs {
  cx<T>* spec;
  const cx<T>* tw;
  T* sig;          // state: stress of the last iterate (= multiplier), 4 planes
  const uint8_t* mask;
  double* partials;
  DevState* state;
  const T* real_in;
  T* real_out;
  T* sig_out;      // ROW_EMIT outputs (may be null)
  T* eps_out;
  uint8_t* plastic_out;
  int mode;
  double E[3];
  DevParams prm;
};

template <typename T>
struct ColArgs {
  cx<T>* spec;
  const cx<T>* tw;
  const cx<T>* ktab;
  DevState* state;
  cx<T>* xbuf;   // 3 L values: transform of the packed column 0
  int mode;
  int flip1, flip2;
  double lam0, mu0, scale;
  double E[3];
};

template <typename T>
hipError_t launch_row(int L, const RowArgs<T>& a, hipStream_t st);
template <typename T>
hipError_t launch_col(int L, const ColArgs<T>& a, hipStream_t st);
template <typename T>
int row_grid(int L);
template <typename T>
int tile_width(int L);
int div_grid(int L);
hipError_t launch_reduce(const double* partials, int nblk, DevState* st, const DevParams& prm, hipStream_t s);
template <typename T>
hipError_t launch_div(const T* sig, double* partials, DevState* st, const DevParams& prm, int L, int force,
                      hipStream_t s);
hipError_t launch_begin(DevState* st, const double* E, double floor_s, hipStream_t s);
hipError_t launch_reduce_emit(const double* partials, int nblk, DevState* st, double npx, hipStream_t s);
hipError_t launch_mask(uint8_t* out, long npx, double f, uint64_t seed, hipStream_t s);

}  // namespace pm
