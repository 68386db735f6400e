// Internal types shared by the kernels (vp_kernels.hip) and the host ABI (vp_api.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vp.h"

namespace vpk {

constexpr int kBlock = 256;      // threads per workgroup for every particle kernel
constexpr int kHistFields = 10;  // doubles per diagnostic record (layout of vp_diag)

enum Mode { kFP64 = 0, kFP32Comp = 1, kFP32 = 2, kFP32TwoSum = 3 };

// Per-instance scalars living in the instance workspace.
struct InstScal {
  double K, mom, chg;      // fused-pass partial sums, cleared by the solving workgroup
  double Kd, momd, chgd;   // partial sums of the diagnostic kernel
  double W, e1r, e1i;      // summary of the current field
  long long step;          // steps taken by the fused path
  int pending;             // 1 when P, q* sit half a kick behind Q, p*
  unsigned ticket;         // workgroups of this instance done in the current pass
  int nonfinite;           // set when a diagnostic came out NaN or Inf
  int pad;
};

// Device descriptor of one instance (one slot of an engine).
struct InstDev {
  void* Q;
  void* P;
  void* qs;
  void* ps;
  void* psi;
  long long n;
  int ng, log2ng;
  int ntiles, acc_copies;
  int hist_cap, solver;
  double L, inv_h, h, dt;
  double* acc;      // acc_copies * ng global load accumulators (float for kFP32)
  double* E;        // element field, ng
  double* g;        // projected curvature phi_h'', ng
  float* Ef;        // float copies for the kFP32 gather
  float* gf;
  double* Phi;      // nodal potential, ng
  double* bt;       // neutralised load, ng
  double* tw;       // tw[2k] = cos(2 pi k / ng), tw[2k+1] = sin(2 pi k / ng), k < ng/2
  double* inv_lam;  // 1 / eigenvalue of the stiffness matrix per Fourier mode (0 for m = 0)
  InstScal* scal;
  double* hist;     // hist_cap records of kHistFields doubles
};

// A run of consecutive particles of one instance, processed by one workgroup.
struct Tile {
  int inst;         // slot index into the InstDev table
  int count;        // particles in this tile (<= kBlock * ppt)
  long long begin;  // first particle index
  int local;        // tile index within its instance
  int pad;
};

// Byte offsets of the workspace regions of one instance (all 256-byte aligned).
struct WsLayout {
  size_t acc, E, g, Ef, gf, Phi, bt, tw, inv_lam, scal, hist, total;
};
WsLayout workspace_layout(int ng, int hist_cap);

size_t particle_lds_bytes(int mode, int max_ng);

hipError_t launch_fused(int mode, int tpb, const InstDev* d_inst, const Tile* d_tiles, int tile0,
                        int ntiles, int ppt, int max_ng, hipStream_t s);
hipError_t launch_deposit(int mode, int tpb, const InstDev* d_inst, const Tile* d_tiles, int tile0,
                          int ntiles, int ppt, int max_ng, hipStream_t s);
hipError_t launch_gather_push(int mode, int tpb, const InstDev* d_inst, const Tile* d_tiles,
                              int tile0, int ntiles, int ppt, int max_ng, double kick, double drift,
                              hipStream_t s);
hipError_t launch_settle(int mode, int tpb, const InstDev* d_inst, const Tile* d_tiles, int tile0,
                         int ntiles, int ppt, int max_ng, hipStream_t s);
hipError_t launch_diag(int mode, int tpb, const InstDev* d_inst, const Tile* d_tiles, int tile0,
                       int ntiles, int ppt, int max_ng, hipStream_t s);
hipError_t launch_solve(int mode, const InstDev* d_inst, const int* d_slots, int nslots,
                        int max_ng, hipStream_t s);
hipError_t launch_slot_scalars(const InstDev* d_inst, const int* d_slots, int nslots, int op,
                               hipStream_t s);
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s);
hipError_t launch_cell_index(const InstDev* d_inst, int slot, int mode, int* cells, long long n,
                             hipStream_t s);
hipError_t launch_sort(int mode, const InstDev* d_inst, int slot, long long n, int chunk,
                       int* perm, hipStream_t s);

// ops for launch_slot_scalars
enum ScalOp { kScalClearDiag = 0, kScalClearPending = 1, kScalReset = 2 };

}  // namespace vpk
