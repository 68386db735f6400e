/*
 * vp.h -- C ABI of the MI355X (gfx950) decorated-particle Vlasov-Poisson library.
 *
 * The library advances decorated particles of the Scovel-Weinstein monopole-dipole model
 * (k = 2) for the normalised 1D1V periodic Vlasov-Poisson system (e = m = eps0 = 1) as
 * discretised in Section 5 of arXiv 2605.21794: P1 (or P2) continuous-Galerkin potential on
 * a uniform periodic mesh of Ng elements over [0, L), load vector of eq. rhs-assembly,
 * stiffness system of eq. lin-sys with the zero-mean gauge, equations of motion of
 * eq. sw-evolution, advanced by the kick-drift-kick splitting of the discrete Hamiltonian
 * of eq. Hh.  Each particle carries (Q, P, q*, p*, psi*): position, velocity, momentum
 * dipole, spatial dipole, weight (the tuple of Section 4).  It also builds decorated
 * particles from marker particles (Algorithm 1: vp_cluster_markers) and runs plain
 * particle-in-cell instances, the p* = q* = 0 special case (vp_config.monopole_only).
 *
 * Conventions shared by every entry point
 *   - All pointers to particle or workspace memory are DEVICE pointers on the current HIP
 *     device; host pointers are named host_*.  No call takes ownership of caller memory:
 *     particle arrays and workspaces are borrowed from vp_create / vp_admit until
 *     vp_destroy / vp_retire and must stay allocated and untouched by other work until then.
 *   - Particle arrays are five separate contiguous arrays (structure of arrays) of n
 *     elements each (eight with second moments, vp_config.moment_order 3), float64 for
 *     VP_FP64 and float32 for the three float32 modes.
 *     Positions must lie in [0, L) on entry; psi* is never written.
 *   - Work is enqueued asynchronously on the stream given at creation (a hipStream_t
 *     passed as void*, NULL for the null stream) unless a function says it synchronises.
 *   - Every function returns a vp_status; on failure nothing is enqueued and
 *     vp_last_error() returns a thread-local message.  A handle is not thread-safe.
 *   - Grid sizes Ng are powers of two in [VP_MIN_NG, VP_MAX_NG].
 */
#ifndef VP_H_
#define VP_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VP_ABI_VERSION 10
#define VP_MIN_NG 8
#define VP_MAX_NG 1024
#define VP_MAX_SORT_CHUNK_F32 4096 /* particles per sorted chunk, float32 state */
#define VP_MAX_SORT_CHUNK_F64 2048 /* particles per sorted chunk, float64 state */
#define VP_MAX_ACC_COPIES 8        /* spread copies of the global load accumulator */
#define VP_MAX_SLOTS 65536

typedef enum vp_status {
  VP_OK = 0,
  VP_ERR_ARG = 1,        /* invalid argument or configuration */
  VP_ERR_HIP = 2,        /* a HIP runtime call failed */
  VP_ERR_NONFINITE = 3,  /* a diagnostic came out NaN or Inf (the values are still returned) */
  VP_ERR_STATE = 4,      /* call not valid in the handle's current state (e.g. empty slot) */
  VP_ERR_RANGE = 5       /* requested history records are no longer (or not yet) stored */
} vp_status;

typedef enum vp_precision {
  VP_FP64 = 0,         /* float64 state; float64 loads accumulated in LDS and globally     */
  VP_FP32_COMP = 1,    /* float32 state; per-particle arithmetic in float64; nodal loads
                          accumulated in float64 (LDS atomics, then global atomics), so the
                          sum carries the low-order bits a float32 two-sum would keep in its
                          error word (float64 LDS atomics are the fast ones on gfx950)    */
  VP_FP32 = 2,         /* float32 state, float32 arithmetic and float32 accumulation
                          (naive reference for the precision study)                        */
  VP_FP32_TWOSUM = 3   /* float32 state; per-particle arithmetic in float64; each nodal load
                          kept in LDS as a float32 (hi, lo) pair updated by a two-sum under a
                          64-bit compare-and-swap; block totals added in float64.  Slower
                          when many lanes of a wavefront hit one node (retries serialise). */
} vp_precision;
/* In every mode the neutralising mean subtraction, the Poisson solve and all
 * diagnostics (K, W, H, charge, momentum) are computed in float64 on the GPU. */

typedef struct vp_config {
  int64_t n;           /* decorated particles, >= 1 */
  int32_t ng;          /* mesh elements (= nodes), power of two in [8, 1024] */
  int32_t precision;   /* vp_precision */
  double L;            /* domain length, > 0 */
  double dt;           /* time step, > 0 */
  int32_t sort_every;  /* vp_step sorts particles by cell every this many steps; 0 = never */
  int32_t sort_chunk;  /* particles per sorted chunk (<= VP_MAX_SORT_CHUNK_*); 0 = max */
  int32_t hist_cap;    /* per-step diagnostic records kept on the device (ring); >= 1 */
  int32_t solver;      /* vp_solver: how vp_poisson / vp_step solve A Phi = b~ */
  int32_t projection;  /* vp_projection: how phi_h'' (the curvature in q*'s kick) is formed */
  int32_t monopole_only; /* 1: p* = q* = 0 for all time (plain P1 particle-in-cell, the paper's
                            comparison method and the k = 1 member of the hierarchy).  Admission
                            fills qs and ps with zeros; the fused step then neither reads nor
                            writes them (20 bytes of particle traffic per update instead of
                            36); the other calls carry the zeros through, and they stay zero.
                            0: decorated particles (default). */
  int32_t no_self_field; /* 1: the particles feel no field of their own (charge e = 0; the
                            paper's test-particle example, eq. swpic_test_particle): the load
                            vector and its field are still computed and returned by
                            vp_diagnostics' grid, but the kicks ignore them and W, E_amp and
                            E1 read 0.  0: self-consistent field (default). */
  int32_t ext_mode;      /* prescribed potential V(q) = ext_amplitude (1 - cos(2 pi ext_mode
                            q / L)) added to the field (eq. sw_prescribed_potential): the kick
                            takes E - V'(Q) and phi'' + V''(Q), and U = sum psi* V(Q) -
                            p* V'(Q) enters H.  ext_mode >= 1 with ext_amplitude != 0 turns it
                            on; 0 (default): none. */
  double ext_amplitude;
  int32_t element_order; /* degree k of the Lagrange space V_h^(k) of eq. galerkin.  1 (or 0, the
                            default): P1, one node per element.  2: continuous P2, a vertex and
                            a midpoint node per element; the load vector is taken against the
                            quadratic basis, the stiffness system is solved with the gauge
                            integral(phi_h) = 0 (eq. galerkin), E = -phi_h' is linear on each
                            element and phi_h'' is read from the basis itself (constant per
                            element, so cfg.projection must be VP_PROJ_ELEM and plays no
                            part).  P2 needs a precision other than VP_FP32. */
  int32_t moment_order;  /* highest moment carried by each particle, the k of the ansatz
                            (eq. sw_f_ansatz) and its quotient algebra s_k (Section
                            "Scovel-Weinstein enhancement of PIC").  0 or 2 (default): the
                            monopole-dipole particle (k = 2).  3: each particle also carries
                            its centred second moments M = (Mqq, Mqp, Mpp) (vp_particles'
                            Mqq, Mqp, Mpp, read and written).  Their Lie-Poisson bracket on
                            the quadratic phase-space polynomials gives the covariance
                            equations of the linearised flow: each kick maps M to A M A^T
                            with A = [[1, 0], [-tau phi'', 1]], each drift with A = [[1, tau],
                            [0, 1]], so det M is kept exactly; the load gains (1/2) Mqq
                            phi_j''(Q), q*'s kick gains -(1/2) Mqq V'''(Q) of a prescribed
                            potential, K gains Mpp / 2 and U gains (1/2) Mqq V''(Q).  k = 3
                            needs element_order 2 (phi_j'' exists on each element), a
                            precision other than VP_FP32, monopole_only 0 and sort_every 0;
                            vp_sort and persistent tuning refuse such a slot. */
} vp_config;

/* The dipole equation d(q*)/dt = p* phi_h''(Q) needs a second derivative that a P1 potential
 * does not have (it vanishes inside every element); Section 5 obtains it through an
 * auxiliary projection whose form the paper leaves open.  Three readings: */
typedef enum vp_projection {
  VP_PROJ_ELEM = 0,        /* lumped L2 projection of the element field E onto P1, then
                              differentiated: element-constant g_e = -(b~_e + b~_{e+1}) / (2h),
                              phi_h''(Q) = g_i on the element i holding Q (default) */
  VP_PROJ_NODAL = 1,       /* L2 projection onto P1 of phi_h'' in the weak sense,
                              (phi_h'', phi_j) = -(phi_h', phi_j') = -b~_j, lumped mass:
                              nodal g_j = -b~_j / h; phi_h''(Q) = (1 - s) g_i + s g_{i+1} */
  VP_PROJ_CONSISTENT = 2   /* the same with the consistent mass matrix M_ij = (phi_i, phi_j) =
                              (h/6) circ(1, 4, 1): M g = -b~, applied through the decaying
                              closed-form inverse of circ(1, 4, 1) (terms below 1e-18 relative
                              omitted); phi_h''(Q) interpolated as for VP_PROJ_NODAL */
} vp_projection;

typedef enum vp_solver {
  VP_SOLVE_SCAN = 0,  /* discrete Gauss law: on the periodic P1 mesh (A Phi)_j = E_j - E_{j-1},
                         so E is a prefix sum of b~ with sum_e E_e = 0 (periodic Phi), and Phi a
                         prefix sum of -h E with sum_j Phi_j = 0; exact, O(Ng), one workgroup */
  VP_SOLVE_FFT = 1    /* diagonalise the circulant A by an in-LDS radix-2 FFT:
                         Phi_m = b~_m / lambda_m, lambda_m = (2/h)(1 - cos(2 pi m / Ng)), Phi_0 = 0 */
} vp_solver;

typedef struct vp_particles {
  void* Q;    /* position in [0, L)                    */
  void* P;    /* velocity (momentum, m = 1)            */
  void* qs;   /* q*: momentum dipole                   */
  void* ps;   /* p*: spatial dipole                    */
  void* psi;  /* psi*: weight, read only               */
  void* Mqq;  /* second moments (vp_config.moment_order 3 only; NULL otherwise): */
  void* Mqp;  /*   the particle's centred covariance in q-q, q-p and p-p, a       */
  void* Mpp;  /*   positive semi-definite 2 x 2 matrix                             */
} vp_particles;

typedef struct vp_diag {
  int64_t step;     /* steps taken by vp_step since creation / admission */
  double t;         /* step * dt */
  double K;         /* sum psi* P^2 / 2 + q* P  (kinetic part of eq. Hh), + Mpp / 2 for
                       particles with second moments */
  double W;         /* (1/2) Phi^T A Phi = (1/2) sum_e h E_e^2 (field part of eq. Hh) */
  double H;         /* K + U + W */
  double charge;    /* sum psi* */
  double momentum;  /* sum psi* P + q* */
  double e_amp;     /* sqrt((1/L) int E^2) (eq. Eamp) = sqrt(2 W / L) */
  double e1_re;     /* (1/Ng) sum_e E_e exp(-2 pi i e / Ng), real part */
  double e1_im;     /*   ... imaginary part */
  double U;         /* prescribed potential's energy sum psi* V(Q) - p* V'(Q) (0 without one);
                       H = K + U + W */
  double stamp;     /* records of vp_history: the device's constant-rate clock (ticks of
                       vp_wall_clock_hz) when the record was written, which for a record
                       written by vp_step is during the launch of the following step, so
                       the difference of consecutive records' stamps is the time one step
                       of the engine took; 0 from vp_diagnostics */
} vp_diag;

/* Launch shape of the particle kernels; chosen by vp_tune or set by the caller. */
typedef struct vp_tuning {
  int32_t threads;      /* threads per workgroup of the particle kernels: 256, 512 or 1024 */
  int32_t ppt;          /* particles per thread per tile: 1, 2, 4, 8, 16, 32 or 64 */
  int32_t acc_copies;   /* copies of each instance's global load accumulator, 1..8 */
  int32_t use_graph;    /* 1: vp_step replays captured HIP graphs; 0: direct launches */
  int32_t graph_steps;  /* steps per captured graph, 1..256 (rounded up to a multiple of 3) */
  int32_t persistent;   /* 1: vp_step runs many steps per cooperative launch with every tile's
                         * particles held in registers between steps (threads 512 or 1024,
                         * ppt 2, 4 or 8; every tile must be resident at once, else
                         * vp_set_tuning returns VP_ERR_ARG); 0: one launch per step */
  int32_t wave_reduce;  /* VP_FP32_TWOSUM only (the other modes ignore it): 1: the deposit
                         * of the fused and persistent steps first combines, within each
                         * wavefront, the loads of neighbouring lanes whose particles lie in
                         * the same element (a segmented sum over each run, then one
                         * compare-and-swap per run and node); it pays when particles that are
                         * neighbours in memory are neighbours in space (sorted by cell,
                         * vp_config.sort_every, or bunched).  0: one update per particle and
                         * node.  Results differ in summation order only. */
} vp_tuning;

typedef struct vp_handle vp_handle;

/* ---------------------------------------------------------------- sizing and lifetime */

/* Bytes of device workspace one instance with this configuration needs (grid
 * accumulators, field arrays, FFT tables, diagnostic history).  Validates *cfg. */
vp_status vp_workspace_bytes(const vp_config* cfg, size_t* bytes_out);

/* Single-instance handle: an engine with one slot, slot 0 admitted with (cfg, parts,
 * workspace).  The instance is the paper's problem statement (Section 5, "Discretization
 * in space and time"): the decorated-particle tuple of Section 4 per particle, a periodic
 * mesh of cfg->ng elements over [0, cfg->L), the time step cfg->dt.  Enqueues the initial
 * deposit and Poisson solve (field at t = 0, eqs. rhs-assembly and lin-sys).
 * workspace: device memory of vp_workspace_bytes(cfg) bytes, 256-byte aligned.
 * stream: hipStream_t as void*.  Errors: VP_ERR_ARG (cfg, null or misaligned pointers),
 * VP_ERR_HIP. */
vp_status vp_create(const vp_config* cfg, vp_particles parts, void* workspace,
                    void* stream, vp_handle** out);

/* Engine with max_slots empty slots, all of one precision (for batches and serving). */
vp_status vp_engine_create(int32_t precision, int32_t max_slots, void* stream,
                           vp_handle** out);

/* Batched handle: engine with n_inst slots admitted from the arrays (one entry each). */
vp_status vp_create_batch(int32_t n_inst, const vp_config* cfgs, const vp_particles* parts,
                          void* const* workspaces, void* stream, vp_handle** out);

/* Put an instance into an empty slot; enqueues its initial deposit and solve.  The
 * precision in cfg must equal the engine's.  Errors: VP_ERR_ARG, VP_ERR_STATE (slot in
 * use or out of range), VP_ERR_HIP. */
vp_status vp_admit(vp_handle* h, int32_t slot, const vp_config* cfg, vp_particles parts,
                   void* workspace);

/* Remove an instance: synchronises the stream, applies its pending half-kick so the
 * particle arrays hold the state at integer time step*dt, and releases the slot.  The
 * caller's buffers are then free to reuse.  Errors: VP_ERR_STATE (empty slot). */
vp_status vp_retire(vp_handle* h, int32_t slot);

/* Synchronises the stream and frees the library's own device tables.  Caller buffers are
 * left untouched (a pending half-kick is NOT applied; call vp_sync_state first). */
vp_status vp_destroy(vp_handle* h);

/* ---------------------------------------------------------------- primitive steps
 * The unfused reference composition of one kick-drift-kick step (Section 5):
 *   vp_gather_push(h, dt/2, dt); vp_deposit(h); vp_poisson(h); vp_gather_push(h, dt/2, 0).
 * Each acts on every occupied slot and leaves the step counter alone. */

/* Load vector b_j = sum_a [psi*_a phi_j(Q_a) - p*_a phi_j'(Q_a)] (eq. rhs-assembly) of the
 * current positions and dipoles.  Replaces each instance's load vector (the one vp_poisson
 * and the next vp_step solve from). */
vp_status vp_deposit(vp_handle* h);

/* Poisson solve (eq. lin-sys) of the current load vector: b~ = b - mean(b) in float64
 * (eq. neutrality), A Phi = b~ with 1^T Phi = 0 (the Gauss-law scan E_e - E_{e-1} = b~_e,
 * sum_e E_e = 0, or an in-LDS FFT, per cfg.solver), element field
 * E_e = -(Phi_{e+1} - Phi_e)/h, projected curvature g (per element or per node, per
 * cfg.projection), W = (1/2) sum h E_e^2.  Writes the field arrays that vp_gather_push and
 * vp_diagnostics read.  One workgroup per instance.
 * P2 elements (cfg.element_order = 2): b~ subtracts the background against each basis
 * function's integral (h/3 at a vertex, 2h/3 at a midpoint).  Eliminating each element's
 * midpoint unknown leaves the P1 system above with the load c_e = b~_e + (b~_{m,e-1} +
 * b~_{m,e})/2, solved as above; its E_e is the field at the midpoint of element e, the
 * field on the element is E_e - h g_e (s - 1/2) at local coordinate s, g_e = phi_h'' =
 * -3 b~_{m,e} / (2h), W = (1/2) sum h E_e^2 + (3h/32) sum b~_{m,e}^2, and the midpoint
 * potential is (3h b~_{m,e} + 8 (Phi_e + Phi_{e+1})) / 16. */
vp_status vp_poisson(vp_handle* h);

/* Exact sub-flows of the splitting with the current field (eq. sw-evolution):
 * kick:  P += kick * E_a,  q* += kick * p* * g_a   (Q, p* frozen), where E_a = E[i] and
 *        g_a = phi_h''(Q) per cfg.projection (both 0 with cfg.no_self_field), plus
 *        -V'(Q) and V''(Q) of a prescribed potential (cfg.ext_mode),
 * drift: Q += drift * P (periodic wrap into [0, L)),  p* -= drift * q*   (P, q* frozen).
 * Requires |drift * P| < L.  After vp_step it first writes the field of the current
 * positions (as vp_poisson); a drift makes the load vector stale until vp_deposit (which
 * vp_step then runs by itself). */
vp_status vp_gather_push(vp_handle* h, double kick, double drift);

/* ---------------------------------------------------------------- fused stepping */

/* Advance every occupied slot by nsteps kick-drift-kick steps of the discrete Hamiltonian
 * system (eq. Hh with the equations of motion of eq. sw-evolution; the leapfrog of
 * Section 5 taken as the splitting into the field and kinetic parts).  One fused kernel launch per
 * step and kind of instance (decorated or monopole-only, P1 or P2, with or without general
 * options; a single launch when all instances are of one kind): every workgroup solves the
 * field of the current positions from the load vector the
 * previous step deposited, then runs its particles through the pending half-kick, the
 * diagnostics at the integer step, the half-kick, the drift and the deposit of the new
 * load vector; optionally replayed from captured HIP graphs.  Equals the primitive
 * composition up to rounding.  Leaves a pending half-kick (P, q* at t + dt/2); every state
 * read-back must go through vp_sync_state, vp_retire or vp_diagnostics (which accounts for
 * it).  With vp_tuning.persistent, up to 1024 steps run in one cooperative launch whose
 * workgroups keep their particles in registers and wait for one another between steps;
 * the arithmetic and the results are those of the fused launches.  Each wait between
 * steps is bounded: after 2^22 polls (fewer when the environment variable
 * VP_PERSIST_SPIN_LIMIT, read when the handle is created, gives a smaller count; for tests
 * of this path) the instance is flagged, its tiles wait no more in that launch, and
 * vp_diagnostics reports VP_ERR_HIP for it from then on (its state is not valid). */
vp_status vp_step(vp_handle* h, int32_t nsteps);
/* (vp_step) An instance whose diagnostics come out NaN or Inf is frozen from the next step
 * on: its state, step counter and history stop where they are, vp_diagnostics and
 * vp_history report VP_ERR_NONFINITE, and the other instances are unaffected. */

/* Capture now every HIP graph that vp_step(h, nsteps) will replay (with graphs on: the
 * graph of vp_tuning.graph_steps steps when nsteps reaches it, and the one-step graph of
 * each ring phase that covers the remaining steps), so that vp_step itself replays only.
 * Runs no step.  Nothing to do for persistent steps or with graphs off.  A later change of
 * tuning or of the occupied slots drops the graphs. */
vp_status vp_prepare_step(vp_handle* h, int32_t nsteps);

/* Apply the pending half-kick of every occupied slot (P, q* back to integer time). */
vp_status vp_sync_state(vp_handle* h);

/* Chunked stable counting sort of one slot's particles by cell index (element
 * i = min(floor(Q * Ng / L), Ng - 1), computed in float64), chunks of cfg.sort_chunk
 * particles, ties kept in original order.  Permutes all five arrays in place.  If
 * dev_perm is non-NULL, writes the permutation (dev_perm[k] = source index of slot k,
 * int32, n entries).  slot < 0 sorts every occupied slot (dev_perm must then be NULL).
 * A slot whose particles carry second moments (moment_order 3) is refused (VP_ERR_ARG). */
vp_status vp_sort(vp_handle* h, int32_t slot, int32_t* dev_perm);

/* Cell index of every particle of one slot into dev_cells (int32, n entries), by the
 * same float64 formula the kernels use. */
vp_status vp_cell_index(vp_handle* h, int32_t slot, int32_t* dev_cells);

/* ---------------------------------------------------------------- diagnostics */

/* Synchronises the stream.  Diagnostics of one slot at its current integer step (a
 * pending half-kick is accounted for without modifying the state).  host_grid, if
 * non-NULL, receives 4*Ng float64 values: b~, Phi, E, g of the particles' own mesh field
 * (also when cfg.no_self_field keeps it from acting).  With P2 elements it receives 6*Ng:
 * b~ of the Ng vertices then of the Ng midpoints, Phi likewise (gauge integral(phi_h) = 0),
 * E_e at each element's midpoint (the element average of the linear field), g_e.
 * Returns VP_ERR_NONFINITE (after filling *host_out) if any value is NaN or Inf. */
vp_status vp_diagnostics(vp_handle* h, int32_t slot, vp_diag* host_out, double* host_grid);

/* Ticks per second of the device clock of vp_diag.stamp (the current device's constant-rate
 * wall clock).  Errors: VP_ERR_ARG (NULL), VP_ERR_HIP. */
vp_status vp_wall_clock_hz(double* hz_out);

/* Synchronises the stream.  Copies the per-step records written by vp_step for steps
 * first_step .. first_step+count-1 (each record is the state at that integer step,
 * before the step was taken).  VP_ERR_RANGE if any is outside the stored ring. */
vp_status vp_history(vp_handle* h, int32_t slot, int64_t first_step, int32_t count,
                     vp_diag* host_out);

/* ---------------------------------------------------------------- tuning and misc */
vp_status vp_set_tuning(vp_handle* h, const vp_tuning* t);
vp_status vp_get_tuning(const vp_handle* h, vp_tuning* t);

/* Time each candidate launch shape on the handle's current slots (the particle arrays
 * are advanced and then restored from a device copy the caller provides: scratch of
 * vp_tune_scratch_bytes), keep the fastest and report it. */
vp_status vp_tune_scratch_bytes(const vp_handle* h, size_t* bytes_out);
vp_status vp_tune(vp_handle* h, void* dev_scratch, int32_t steps_per_trial, vp_tuning* best_out,
                  double* best_us_per_step_out);

/* Number of occupied slots and the total particle count over them. */
vp_status vp_occupancy(const vp_handle* h, int32_t* slots_out, int64_t* particles_out);

/* Synchronises the stream.  For slots 0 .. n-1 of an engine: host_steps[s] = the slot's
 * device step count (the integer step its state has reached; it stops when the instance
 * is frozen), or -1 for an empty slot; host_flags[s] = VP_SLOT_OCCUPIED | VP_SLOT_NONFINITE
 * as they apply.  One small kernel and one copy for all slots, so a serving loop can poll
 * every resident job between chunks of steps.  Host arrays of n elements, owned by the
 * caller; n may exceed the engine's slots (the rest read as empty).  Errors: VP_ERR_ARG
 * for a NULL handle or array or n < 0, VP_ERR_HIP. */
#define VP_SLOT_OCCUPIED 1
#define VP_SLOT_NONFINITE 2
vp_status vp_slot_status(vp_handle* h, int32_t n, int64_t* host_steps, int32_t* host_flags);

/* ---------------------------------------------------------------- initialisation */

/* Decorated particles from marker particles, the paper's Algorithm 1 with the periodic
 * moments of its torus subsection.  k-means of the markers in (q, p): `iters` Lloyd
 * iterations from the k markers init_idx (nearest centre by Euclidean distance in (q, p),
 * ties to the lowest centre; centres move to the weighted mean of their markers, weights
 * wm; an empty cluster keeps its centre), then a final assignment.  Each non-empty cluster
 * S_a, in cluster order, gives one decorated particle:
 *   psi*_a = sum of its weights (eq. psi-star);
 *   (Q_a, P_a) = the member nearest the cluster's weighted mean (first in marker order on
 *                ties);
 *   p*_a = sum wm_A (L / 2 pi) sin(2 pi (Q_a - Qm_A) / L),  q*_a = -sum wm_A (P_a - Pm_A)
 *          (eq. moment-def with the periodic c).
 * All sums run over the members in increasing marker order, so results are reproducible.
 * Inputs (device, float64, 8-byte aligned, not modified): Qm in [0, L), Pm, wm > 0, m of
 * each; init_idx: k marker indices in [0, m) (device int32; checked on the host,
 * VP_ERR_ARG if out of range; normally distinct: a repeated index starts two centres at
 * one place, and the higher-numbered one gets no markers in the first assignment).  1 <= k <= m < 2^31, iters >= 0, L > 0.
 * workspace: vp_cluster_workspace_bytes(m, k) bytes of device memory, 256-byte aligned.
 * Outputs (device, float64, capacity k each): Q, P, qs (q*), ps (p*), psi of the non-empty
 * clusters; assign_out (device int32, m, or NULL): final cluster of each marker;
 * *n_out (host): the number of decorated particles written.  Runs on `stream` (a
 * hipStream_t, or NULL) and synchronises it.  Errors: VP_ERR_ARG, VP_ERR_HIP. */
vp_status vp_cluster_workspace_bytes(int64_t m, int32_t k, size_t* bytes_out);
vp_status vp_cluster_markers(const double* Qm, const double* Pm, const double* wm, int64_t m,
                             int32_t k, const int32_t* init_idx, int32_t iters, double L,
                             void* workspace, void* stream, double* Q, double* P, double* qs,
                             double* ps, double* psi, int32_t* assign_out, int32_t* n_out);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): vp_cluster_markers without the workspace
 * argument.  The workspace is the library's own file-scope device array of
 * VP_CLUSTER_STATIC_BYTES (16 MiB), one per device, held until the process ends; the call
 * allocates nothing.  Same arguments, outputs and results as vp_cluster_markers (bit for
 * bit); the starting indices are checked on the device.  Refused with VP_ERR_ARG when
 * vp_cluster_workspace_bytes(m, k) exceeds VP_CLUSTER_STATIC_BYTES (400k markers into 40k
 * clusters fit).  Every call clears the part of the array it uses first.  Calls that
 * overlap on one device (two streams, two threads) share the array and race: serialise
 * them.  Synchronises `stream`.  Errors: VP_ERR_ARG, VP_ERR_HIP. */
#define VP_CLUSTER_STATIC_BYTES (16u << 20)
vp_status vp_cluster_markers_static(const double* Qm, const double* Pm, const double* wm,
                                    int64_t m, int32_t k, const int32_t* init_idx, int32_t iters,
                                    double L, void* stream, double* Q, double* P, double* qs,
                                    double* ps, double* psi, int32_t* assign_out,
                                    int32_t* n_out);

/* Algorithm 1 with mini-batch k-means in place of Lloyd's iteration, which the paper allows
 * for large runs (Section 4, before Algorithm 1).  The update is the weighted, batched form
 * of Sculley's mini-batch k-means ("Web-scale k-means clustering", 2010).  From the k
 * markers init_idx, nbatch batches are taken in turn; batch t is the `batch` marker indices
 * batch_idx[t*batch .. (t+1)*batch) (device int32, nbatch*batch of them, each in [0, m),
 * repeats allowed and counted once per occurrence; the caller draws them).  Per batch:
 * every batch marker goes to its nearest current centre (as in vp_cluster_markers), then
 * every centre c that received members moves to the weighted mean of all the batch members
 * it has received so far, its old value standing in for the earlier ones:
 *   v_c <- v_c + W_c,   centre_c <- (centre_c * v_c(old) + S_c) / v_c(new),
 * W_c and S_c being the weight and weighted (q, p) sums of its members in this batch, summed
 * in batch order (v starts at 0, so a centre's first update is the plain weighted mean).
 * No reassignment of starved centres and no stopping test.  Then, as vp_cluster_markers
 * after its iterations: a final assignment of every marker and one decorated particle per
 * non-empty cluster.  Arguments as for vp_cluster_markers, plus: 1 <= batch <= m,
 * nbatch >= 1, batch * nbatch < 2^31; workspace of
 * vp_cluster_minibatch_workspace_bytes(m, k, batch) bytes; absorbed_out (device float64,
 * k, or NULL) receives each centre's v.  Every batch index is checked on the device before
 * use (VP_ERR_ARG if any lies outside [0, m)).  Synchronises the stream.  Errors:
 * VP_ERR_ARG, VP_ERR_HIP. */
vp_status vp_cluster_minibatch_workspace_bytes(int64_t m, int32_t k, int32_t batch,
                                               size_t* bytes_out);
vp_status vp_cluster_markers_minibatch(const double* Qm, const double* Pm, const double* wm,
                                       int64_t m, int32_t k, const int32_t* init_idx,
                                       const int32_t* batch_idx, int32_t batch, int32_t nbatch,
                                       double L, void* workspace, void* stream, double* Q,
                                       double* P, double* qs, double* ps, double* psi,
                                       int32_t* assign_out, double* absorbed_out,
                                       int32_t* n_out);

const char* vp_status_string(vp_status s);
const char* vp_last_error(void);
int32_t vp_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* VP_H_ */
