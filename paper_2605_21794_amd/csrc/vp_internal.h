// Internal types shared by the kernels (vp_kernels.hip) and the host ABI (vp_api.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vp.h"

namespace vpk {

constexpr int kBlock = 256;      // threads per workgroup for every particle kernel
constexpr int kHistFields = 12;  // doubles per diagnostic record (layout of vp_diag)
constexpr int kKinFields = 4;    // per-tile sums: K, momentum, charge, prescribed-potential U
constexpr int kMinTile = 256;    // fewest particles per tile (256 threads x 1 particle)

enum Mode { kFP64 = 0, kFP32Comp = 1, kFP32 = 2, kFP32TwoSum = 3 };

// The fused step runs in one of three phases r = (engine step count) mod 3.  A pass in phase
// r solves the field from accumulator ring entry r (deposited by the previous pass), adds the
// new deposit into entry r+1 and clears entry r+2 (read by the pass before it); the kinetic
// sums and the field summary live in rings of the same period.
constexpr int kRing = 3;

// Consistent-mass projection: the solve forms g_j = sum_t cw[t] b~_{(j - t - off) mod Ng}.
// The inverse of circ(1, 4, 1) decays like (2 - sqrt 3)^|d|, below 1e-18 of its diagonal
// beyond |d| = 32, so Ng <= 64 uses all Ng taps (off 0) and larger meshes 65 (off -32).
constexpr int kConsTapsMax = 65;
constexpr int cons_taps(int ng) { return ng <= 64 ? ng : kConsTapsMax; }
constexpr int cons_off(int ng) { return ng <= 64 ? 0 : -(kConsTapsMax / 2); }

constexpr int kArriveGroups = 16;  // arrival counters per instance
constexpr int kReleaseFlags = 32;  // copies of an instance's release flag
constexpr int kArriveStride = 32;  // unsigned words between counters and flags (128 bytes)
// Polls of a persistent launch's wait before it gives up (the instance is then flagged and the
// launch drains).  A handle may be created with fewer (the VP_PERSIST_SPIN_LIMIT environment
// variable), which tests of the time-out path use; never more.
constexpr unsigned kSpinLimit = 1u << 22;

// Per-instance scalars living in the instance workspace.
struct InstScal {
  double W[kRing], e1r[kRing], e1i[kRing];  // summary of the field solved from ring entry r
  double Kd, momd, chgd, Ud;                // partial sums of the diagnostic kernel
  long long step;                           // integer step of the state (fused path)
  int pend[kRing];                          // 1 when P, q* owe the half-kick with the field of entry r
  int nonfinite;                            // set when a diagnostic came out NaN or Inf
  int frozen;                               // nonfinite as of the start of a persistent launch
  int timeout;                              // a persistent launch's wait gave up (error)
  // The barrier between the steps of a persistent launch, a two-level tree: tile t of the
  // instance counts its arrival on group counter t mod G (G = min(kArriveGroups, tiles));
  // the tile that completes a group counts on `top`, and the tile that completes `top`
  // writes the step's number into every release flag.  A waiting tile polls flag
  // t mod kReleaseFlags with one lane.  Each counter and flag has a 128-byte line of its own,
  // so the polls of the waiting tiles are spread over kReleaseFlags lines and leave the
  // counters to the arrivals.
  alignas(128) unsigned arrive[kArriveGroups * kArriveStride];
  alignas(128) unsigned top[kArriveStride];
  alignas(128) unsigned release[kReleaseFlags * kArriveStride];
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
  int order;        // Lagrange degree of the potential: 1 (P1) or 2 (P2)
  int nacc;         // load-vector nodes: ng (P1), 2 ng (P2: vertices [0, ng), midpoints [ng, 2 ng))
  int ntiles, acc_copies;
  int hist_cap, solver;
  double L, inv_h, h, dt;
  double* acc;      // kRing x VP_MAX_ACC_COPIES x nacc load accumulators (float for kFP32)
  double* E;        // element field, ng
  double* g;        // projected curvature phi_h'', ng
  float* Ef;        // float copies for the kFP32 gather
  float* gf;
  double* Phi;      // nodal potential, nacc
  double* bt;       // neutralised load, nacc
  double* tw;       // tw[2k] = cos(2 pi k / ng), tw[2k+1] = sin(2 pi k / ng), k < ng/2
  double* inv_lam;  // 1 / eigenvalue of the stiffness matrix per Fourier mode (0 for m = 0)
  double* cw;       // consistent projection: kConsTaps weights of -M^-1 (see cons_taps)
  InstScal* scal;
  double* hist;     // hist_cap records of kHistFields doubles
  double* kin;      // kRing x kin_cap x kKinFields per-tile kinetic sums of phase r's pass
  int kin_cap;      // tiles the kinetic-sum ring can hold (ceil(n / 256))
  int proj;         // vp_projection
  int general;      // any of: a nodal projection, no self field, a prescribed potential
  int self_on;      // the particles feel their own field
  int ext_on;       // a prescribed potential acts
  double ext_a, ext_k, ext_ak, ext_akk;  // A, kappa = 2 pi m / L, A kappa, A kappa^2
  void* Mqq;        // second moments of k = 3 particles (nullptr otherwise)
  void* Mqp;
  void* Mpp;
  int k3;           // the particles carry second moments (P2, general options)
  int seg;          // the fused and persistent deposits combine runs of equal elements
                    // within each wavefront first (vp_tuning.wave_reduce)
  unsigned spin_limit;  // polls before a persistent wait gives up (<= kSpinLimit)
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
  size_t acc, E, g, Ef, gf, Phi, bt, tw, inv_lam, cw, scal, hist, kin, total;
};
WsLayout workspace_layout(int ng, int order, int hist_cap, long long n);
int kin_capacity(long long n);

size_t particle_lds_bytes(int mode, int max_ng);
// The `max_ng` of every launch below sizes its LDS: the largest ng of the instances it
// serves, doubled for a P2 instance (whose load vector has 2 ng nodes).

// `lds_fft` is true when some instance of the launch uses the FFT solver (more LDS);
// `dipoles` false when every tile of the launch is of a monopole-only instance; `general`
// true when some instance of the launch has general options (InstDev::general); `p2` true
// when its instances have P2 elements; `moments` true when its instances carry second
// moments (InstDev::k3; then dipoles, general and p2 hold too).
hipError_t launch_fused(int mode, int tpb, const InstDev* d_inst, const Tile* d_tiles, int tile0,
                        int ntiles, int ppt, int max_ng, bool lds_fft, int phase, bool dipoles,
                        bool general, bool p2, bool moments, hipStream_t s);
// The same for one precision mode (vpk::Mode), defined in the unit compiled for that mode.
template <int MODE>
hipError_t launch_fused_mode(int tpb, const InstDev* d_inst, const Tile* d_tiles, int tile0,
                             int ntiles, int ppt, int max_ng, bool lds_fft, int phase, bool dipoles,
                             bool general, bool p2, bool moments, hipStream_t s);
hipError_t launch_deposit(int mode, int tpb, const InstDev* d_inst, const Tile* d_tiles, int tile0,
                          int ntiles, int ppt, int max_ng, int phase, hipStream_t s);
hipError_t launch_gather_push(int mode, int tpb, const InstDev* d_inst, const Tile* d_tiles,
                              int tile0, int ntiles, int ppt, int max_ng, double kick, double drift,
                              hipStream_t s);
hipError_t launch_settle(int mode, int tpb, const InstDev* d_inst, const Tile* d_tiles, int tile0,
                         int ntiles, int ppt, int max_ng, int phase, hipStream_t s);
hipError_t launch_diag(int mode, int tpb, const InstDev* d_inst, const Tile* d_tiles, int tile0,
                       int ntiles, int ppt, int max_ng, int phase, hipStream_t s);
// Persistent form of the fused step: nsteps steps in one cooperative launch, the particles
// of each tile held in registers between steps (ppt per thread, 2, 4 or 8).  Every tile of
// the launch must be resident at once: persist_capacity gives how many workgroups can be.
// `general`: some instance of the launch has general options (InstDev::general); `p2`:
// some instance has P2 elements (never with second moments).
hipError_t launch_persist(int mode, int tpb, int ppt, const InstDev* d_inst, const Tile* d_tiles,
                          int ntiles, int max_ng, bool lds_fft, bool general, bool p2, int phase,
                          int nsteps, hipStream_t s);
int persist_capacity(int mode, int tpb, int ppt, int max_ng, bool lds_fft, bool general,
                     bool p2);
// Solve the listed slots from ring entry `phase` and write the field arrays (materialise).
hipError_t launch_solve(int mode, const InstDev* d_inst, const int* d_slots, int nslots,
                        int max_ng, bool lds_fft, int phase, hipStream_t s);
// Ring maintenance for the listed slots (RingOp).
hipError_t launch_ring(int mode, const InstDev* d_inst, const int* d_slots, int nslots, int op,
                       int phase, hipStream_t s);
hipError_t launch_slot_scalars(const InstDev* d_inst, const int* d_slots, int nslots, int op,
                               int phase, hipStream_t s);
// ---------------------------------------------------------------- initialisation (Algorithm 1)
constexpr int kClusterMinMaxBlocks = 1024;  // partial min / max blocks of the velocity range
constexpr int kRadixChunk = 1024;           // elements per workgroup in the radix sort
inline long long cluster_max_cells(int k) { return 4LL * k + 64; }
inline long long radix_blocks(long long m) { return (m + kRadixChunk - 1) / kRadixChunk; }

// Byte offsets of the regions of the caller's clustering workspace (256-byte aligned).
// `batch` > 0 adds the mini-batch regions (absorbed weights v, the gathered batch, its
// visiting order) for batches of that many markers (batch <= m).
struct ClusterWs {
  size_t cq, cp, assign, cnt, off, perm, keys_a, vals_a, keys_b, vals_b, hist, hoff, cell_of, ccnt,
      coff, ccur, clist, mm, tQ, tP, tqs, tps, tpsi, flag, pos, scan, v, bq, bp, bw, bperm, bad,
      total;
};
ClusterWs cluster_layout(long long m, int k, int batch = 0);
// The library's own workspace of vp_cluster_markers_static on the current device (a file-scope
// device array of VP_CLUSTER_STATIC_BYTES, its address looked up once per device).
hipError_t cluster_static_workspace(void** ptr_out);
// *host_bad = how many of the n device indices idx lie outside [0, m) (synchronises).
hipError_t cluster_count_bad(const int* idx, long long n, long long m, void* ws,
                             const ClusterWs& w, int* host_bad, hipStream_t s);
// Velocity range of the markers (synchronises the stream).
hipError_t cluster_p_range(const double* p, long long m, void* ws, const ClusterWs& w,
                           double* host_minmax, hipStream_t s);
// nbatch mini-batch updates (batches of `batch` marker indices, batch_idx[t * batch ..]),
// then Lloyd iterations, final assignment, moments and compaction; *host_n = decorated
// particles written; absorbed_out (k doubles, or NULL) = the weight each centre absorbed in
// the batches (synchronises the stream).
hipError_t cluster_run(const double* q, const double* p, const double* w, long long m, int k,
                       const int* init_idx, const int* batch_idx, int batch, int nbatch,
                       int iters, double L, double pmin, double pmax, void* ws,
                       const ClusterWs& lay, double* Q, double* P, double* qs, double* ps,
                       double* psi, int* assign_out, double* absorbed_out, int* host_n,
                       hipStream_t s);

// out[2t] = step, out[2t+1] = nonfinite of instance slots[t], t < nslots.
hipError_t launch_slot_status(const InstDev* d_inst, const int* d_slots, int nslots,
                              long long* out, hipStream_t s);
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s);
hipError_t launch_cell_index(const InstDev* d_inst, int slot, int mode, int* cells, long long n,
                             hipStream_t s);
hipError_t launch_sort(int mode, const InstDev* d_inst, int slot, long long n, int chunk,
                       int* perm, hipStream_t s);

// ops for launch_slot_scalars
enum ScalOp { kScalClearDiag = 0, kScalClearPending = 1, kScalPersistStart = 2 };
// ops for launch_ring: fold entry `phase` into its copy 0 and clear the two other entries
// (after the number of accumulator copies changed); or clear entry `phase` (before a deposit)
enum RingOp { kRingFold = 0, kRingClear = 1 };

}  // namespace vpk
