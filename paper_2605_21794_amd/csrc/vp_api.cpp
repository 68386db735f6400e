// Host side of the C ABI declared in vp.h: validation, slot and tile tables, launch order,
// HIP graph capture of the fused step, diagnostics read-back and the launch-shape tuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdlib>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "vp.h"
#include "vp_internal.h"

using vpk::InstDev;
using vpk::Tile;

namespace {

thread_local std::string g_err;

vp_status fail(vp_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define VP_HIP(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess) return fail(VP_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

#define VP_TRY(expr)              \
  do {                            \
    vp_status s_ = (expr);        \
    if (s_ != VP_OK) return s_;   \
  } while (0)

constexpr int kGroups = 9;        // kinds of tiles, one fused launch each (see rebuild_tables)
constexpr int kGroupMoments = 8;  // the kind of instances with second moments

bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }
int ilog2(int x) { int m = 0; while ((1 << m) < x) ++m; return m; }
size_t state_elem_size(int prec) { return prec == VP_FP64 ? sizeof(double) : sizeof(float); }
int max_sort_chunk(int prec) { return prec == VP_FP64 ? VP_MAX_SORT_CHUNK_F64 : VP_MAX_SORT_CHUNK_F32; }

vp_status validate(const vp_config* c) {
  if (!c) return fail(VP_ERR_ARG, "config is NULL");
  if (c->n < 1 || c->n > (int64_t)1 << 40) return fail(VP_ERR_ARG, "n = %lld out of range", (long long)c->n);
  if (!is_pow2(c->ng) || c->ng < VP_MIN_NG || c->ng > VP_MAX_NG)
    return fail(VP_ERR_ARG, "ng = %d must be a power of two in [%d, %d]", c->ng, VP_MIN_NG, VP_MAX_NG);
  if (c->precision < VP_FP64 || c->precision > VP_FP32_TWOSUM) return fail(VP_ERR_ARG, "bad precision %d", c->precision);
  if (!(c->L > 0.0) || !std::isfinite(c->L)) return fail(VP_ERR_ARG, "L must be positive and finite");
  if (!(c->dt > 0.0) || !std::isfinite(c->dt)) return fail(VP_ERR_ARG, "dt must be positive and finite");
  if (c->sort_every < 0) return fail(VP_ERR_ARG, "sort_every < 0");
  if (c->sort_chunk < 0 || c->sort_chunk > max_sort_chunk(c->precision))
    return fail(VP_ERR_ARG, "sort_chunk = %d exceeds %d", c->sort_chunk, max_sort_chunk(c->precision));
  if (c->hist_cap < 1) return fail(VP_ERR_ARG, "hist_cap must be >= 1");
  if (c->solver != VP_SOLVE_SCAN && c->solver != VP_SOLVE_FFT) return fail(VP_ERR_ARG, "bad solver %d", c->solver);
  if (c->projection != VP_PROJ_ELEM && c->projection != VP_PROJ_NODAL &&
      c->projection != VP_PROJ_CONSISTENT)
    return fail(VP_ERR_ARG, "bad projection %d", c->projection);
  if (c->monopole_only != 0 && c->monopole_only != 1)
    return fail(VP_ERR_ARG, "monopole_only must be 0 or 1");
  if (c->no_self_field != 0 && c->no_self_field != 1)
    return fail(VP_ERR_ARG, "no_self_field must be 0 or 1");
  if (c->ext_mode < 0 || !std::isfinite(c->ext_amplitude))
    return fail(VP_ERR_ARG, "ext_mode must be >= 0 and ext_amplitude finite");
  if (c->element_order < 0 || c->element_order > 2)
    return fail(VP_ERR_ARG, "element_order = %d must be 0, 1 or 2", c->element_order);
  if (c->element_order == 2) {
    if (c->precision == VP_FP32)
      return fail(VP_ERR_ARG, "P2 elements need a precision other than VP_FP32");
    if (c->projection != VP_PROJ_ELEM)
      return fail(VP_ERR_ARG, "P2 elements take phi_h'' from the basis: projection must be "
                              "VP_PROJ_ELEM");
  }
  if (c->moment_order != 0 && c->moment_order != 2 && c->moment_order != 3)
    return fail(VP_ERR_ARG, "moment_order = %d must be 0, 2 or 3", c->moment_order);
  if (c->moment_order == 3) {
    if (c->element_order != 2)
      return fail(VP_ERR_ARG, "second moments need P2 elements (element_order 2)");
    if (c->precision == VP_FP32)
      return fail(VP_ERR_ARG, "second moments need a precision other than VP_FP32");
    if (c->monopole_only) return fail(VP_ERR_ARG, "second moments need dipoles (monopole_only 0)");
    if (c->sort_every != 0)
      return fail(VP_ERR_ARG, "particles with second moments are not sorted (sort_every 0)");
  }
  return VP_OK;
}

int order_of(const vp_config& c) { return c.element_order == 2 ? 2 : 1; }
// Particle arrays of a slot: five, eight with second moments.
int state_arrays(const vp_config& c) { return c.moment_order == 3 ? 8 : 5; }

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

struct Slot {
  bool used = false;
  vp_config cfg{};
  vp_particles parts{};
  void* ws = nullptr;
  int tile_begin = 0, ntiles = 0;
  long long step = 0;   // host mirror of the device step counter
  bool pending = false; // host mirror of the pending half-kick
  long long last_sort = -1;
};

}  // namespace

struct vp_handle {
  int precision = VP_FP64;
  int max_slots = 0;
  hipStream_t stream = nullptr;
  std::vector<Slot> slots;
  std::vector<InstDev> h_inst;
  std::vector<Tile> h_tiles;
  std::vector<int> h_occ;
  InstDev* d_inst = nullptr;
  Tile* d_tiles = nullptr;
  size_t tiles_cap = 0;
  int ntiles = 0;
  int ntiles_dip = 0;      // tiles of decorated instances
  // tile ranges by kind: decorated / monopole-only x P1 / P2 x without / with general
  // options, then the instances with second moments
  int group_end[kGroups] = {};
  int* d_occ = nullptr;
  int* d_ids = nullptr;     // d_ids[i] = i, for single-slot launches
  long long* d_status = nullptr;  // 2 per slot: step, nonfinite (vp_slot_status)
  int max_ng = VP_MIN_NG;   // largest ng of the slots, doubled for P2 (sizes the launches' LDS)
  bool any_fft = false;     // some slot uses the FFT solver (fused launches need more LDS)
  vp_tuning tun{1024, 4, 4, 1, 33, 0, 0};
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipGraph_t step_graph[vpk::kRing] = {nullptr, nullptr, nullptr};  // one step at phase p
  hipGraphExec_t step_exec[vpk::kRing] = {nullptr, nullptr, nullptr};
  int graph_len = 0;        // fused launches per graph (a multiple of the ring period)
  int graph_phase = 0;      // ring phase the graph was captured at
  bool graph_ok = false;
  int phase = 0;            // ring phase of the next fused launch (step count mod kRing)
  bool field_stale = false; // fused steps ran since the field arrays were last written
  bool acc_stale = false;   // a drift ran since the ring entry of `phase` was deposited
  unsigned spin_limit = vpk::kSpinLimit;  // polls of a persistent wait (VP_PERSIST_SPIN_LIMIT)
};

namespace {

void drop_graph(vp_handle* h) {
  if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  h->gexec = nullptr;
  h->graph = nullptr;
  for (int p = 0; p < vpk::kRing; ++p) {
    if (h->step_exec[p]) (void)hipGraphExecDestroy(h->step_exec[p]);
    if (h->step_graph[p]) (void)hipGraphDestroy(h->step_graph[p]);
    h->step_exec[p] = nullptr;
    h->step_graph[p] = nullptr;
  }
  h->graph_ok = false;
  h->graph_len = 0;
}

// Rebuild the tile list and occupied-slot list from the slots and upload them (with the
// instance table).  Synchronises the stream (no kernel may still read the old tables).
vp_status rebuild_tables(vp_handle* h) {
  VP_HIP(hipStreamSynchronize(h->stream));
  drop_graph(h);
  const int tile_n = h->tun.threads * h->tun.ppt;
  h->h_tiles.clear();
  h->h_occ.clear();
  h->max_ng = VP_MIN_NG;
  for (int s = 0; s < h->max_slots; ++s)
    if (h->slots[s].used) h->h_occ.push_back(s);
  // tiles grouped by kind, one fused launch per non-empty group and step: decorated then
  // monopole-only instances; within each, P1 then P2 elements, each without then with
  // general options; last the instances with second moments (P2, general, decorated)
  auto group_of = [&](int s) {
    const InstDev& d = h->h_inst[s];
    if (d.k3) return kGroupMoments;
    return (h->slots[s].cfg.monopole_only ? 4 : 0) + (d.order == 2 ? 2 : 0) + (d.general ? 1 : 0);
  };
  std::vector<int> order;
  for (int gi = 0; gi < kGroups; ++gi)
    for (int s : h->h_occ)
      if (group_of(s) == gi) order.push_back(s);
  h->ntiles_dip = 0;
  for (int gi = 0; gi < kGroups; ++gi) h->group_end[gi] = 0;
  for (int s : order) {
    Slot& sl = h->slots[s];
    h->max_ng = std::max(h->max_ng, order_of(sl.cfg) * sl.cfg.ng);  // LDS sizing
    const long long n = sl.cfg.n;
    const int nt = (int)((n + tile_n - 1) / tile_n);
    sl.tile_begin = (int)h->h_tiles.size();
    sl.ntiles = nt;
    for (int t = 0; t < nt; ++t) {
      Tile tl{};
      tl.inst = s;
      tl.begin = (long long)t * tile_n;
      tl.count = (int)std::min<long long>(tile_n, n - tl.begin);
      tl.local = t;
      h->h_tiles.push_back(tl);
    }
    InstDev& d = h->h_inst[s];
    if (nt > d.kin_cap) return fail(VP_ERR_STATE, "slot %d: %d tiles exceed the kinetic-sum ring (%d)", s, nt, d.kin_cap);
    d.ntiles = nt;
    d.acc_copies = std::max(1, std::min(h->tun.acc_copies, nt));
    d.seg = h->tun.wave_reduce;
    d.spin_limit = h->spin_limit;
    if (!sl.cfg.monopole_only) h->ntiles_dip += nt;
    for (int gi = group_of(s); gi < kGroups; ++gi) h->group_end[gi] += nt;
  }
  h->ntiles = (int)h->h_tiles.size();
  h->any_fft = false;
  for (int s : h->h_occ) h->any_fft = h->any_fft || h->slots[s].cfg.solver == VP_SOLVE_FFT;
  if ((size_t)h->ntiles > h->tiles_cap) {
    if (h->d_tiles) VP_HIP(hipFree(h->d_tiles));
    h->d_tiles = nullptr;
    size_t cap = std::max<size_t>(1024, (size_t)h->ntiles * 2);
    VP_HIP(hipMalloc(&h->d_tiles, cap * sizeof(Tile)));
    h->tiles_cap = cap;
  }
  if (h->ntiles > 0)
    VP_HIP(hipMemcpyAsync(h->d_tiles, h->h_tiles.data(), h->ntiles * sizeof(Tile),
                          hipMemcpyHostToDevice, h->stream));
  if (!h->h_occ.empty())
    VP_HIP(hipMemcpyAsync(h->d_occ, h->h_occ.data(), h->h_occ.size() * sizeof(int),
                          hipMemcpyHostToDevice, h->stream));
  VP_HIP(hipMemcpyAsync(h->d_inst, h->h_inst.data(), h->max_slots * sizeof(InstDev),
                        hipMemcpyHostToDevice, h->stream));
  // the number of accumulator copies may have changed: fold the live ring entry into copy 0
  VP_HIP(vpk::launch_ring(h->precision, h->d_inst, h->d_occ, (int)h->h_occ.size(), vpk::kRingFold,
                          h->phase, h->stream));
  VP_HIP(hipStreamSynchronize(h->stream));
  return VP_OK;
}

vp_status check_slot(const vp_handle* h, int slot) {
  if (!h) return fail(VP_ERR_ARG, "handle is NULL");
  if (slot < 0 || slot >= h->max_slots) return fail(VP_ERR_STATE, "slot %d out of range", slot);
  if (!h->slots[slot].used) return fail(VP_ERR_STATE, "slot %d is empty", slot);
  return VP_OK;
}

int next_phase(int p) { return p == vpk::kRing - 1 ? 0 : p + 1; }

// One fused step of every instance in phase ph: one launch per non-empty group of tiles
// (decorated / monopole-only instances x P1 / P2 x without / with general options, and the
// instances with second moments).
hipError_t fused_step(vp_handle* h, int ph) {
  int b = 0;
  for (int gi = 0; gi < kGroups; ++gi) {
    const int e_ = h->group_end[gi];
    if (e_ > b) {
      const bool km = gi == kGroupMoments;
      const hipError_t e = vpk::launch_fused(h->precision, h->tun.threads, h->d_inst, h->d_tiles,
                                             b, e_ - b, h->tun.ppt, h->max_ng, h->any_fft, ph,
                                             gi < 4 || km, (gi & 1) != 0 || km,
                                             (gi & 2) != 0 || km, km, h->stream);
      if (e != hipSuccess) return e;
    }
    b = e_;
  }
  return hipSuccess;
}

vp_status launch_steps_direct(vp_handle* h, int nsteps) {
  for (int i = 0; i < nsteps; ++i) {
    VP_HIP(fused_step(h, h->phase));
    h->phase = next_phase(h->phase);
  }
  return VP_OK;
}

// Fused launches per graph: graph_steps rounded up to a multiple of the ring period, so a
// replay leaves the phase where it found it.
int graph_len_of(const vp_handle* h) {
  return (h->tun.graph_steps + vpk::kRing - 1) / vpk::kRing * vpk::kRing;
}

// Capture `len` fused steps starting at ring phase ph into *g / *ge.
vp_status capture_steps(vp_handle* h, int ph, int len, hipGraph_t* g_out, hipGraphExec_t* ge_out) {
  VP_HIP(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
  hipError_t le = hipSuccess;
  for (int i = 0; i < len && le == hipSuccess; ++i) {
    le = fused_step(h, ph);
    ph = next_phase(ph);
  }
  hipGraph_t g = nullptr;
  hipError_t ee = hipStreamEndCapture(h->stream, &g);
  if (le != hipSuccess || ee != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return fail(VP_ERR_HIP, "graph capture failed: %s / %s", hipGetErrorString(le),
                hipGetErrorString(ee));
  }
  hipGraphExec_t ge = nullptr;
  const hipError_t ie = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
  if (ie != hipSuccess) {
    (void)hipGraphDestroy(g);
    return fail(VP_ERR_HIP, "graph instantiation failed: %s", hipGetErrorString(ie));
  }
  *g_out = g;
  *ge_out = ge;
  return VP_OK;
}

vp_status ensure_graph(vp_handle* h) {
  if (h->graph_ok && h->graph_len == graph_len_of(h)) return VP_OK;
  drop_graph(h);
  const int len = graph_len_of(h);
  VP_TRY(capture_steps(h, h->phase, len, &h->graph, &h->gexec));
  h->graph_len = len;
  h->graph_phase = h->phase;
  h->graph_ok = true;
  return VP_OK;
}

// The one-step graph of phase p (the steps a whole graph does not cover are replayed from
// these, so that vp_step with graphs on runs no direct launch).
vp_status ensure_step_graph(vp_handle* h, int p) {
  if (h->step_exec[p]) return VP_OK;
  return capture_steps(h, p, 1, &h->step_graph[p], &h->step_exec[p]);
}

vp_status launch_steps_graphed(vp_handle* h, int nsteps) {
  for (int i = 0; i < nsteps; ++i) {
    VP_TRY(ensure_step_graph(h, h->phase));
    VP_HIP(hipGraphLaunch(h->step_exec[h->phase], h->stream));
    h->phase = next_phase(h->phase);
  }
  return VP_OK;
}

constexpr int kMaxPersistSteps = 1024;  // steps per cooperative launch (bounds its duration)

// Some occupied slot has general options (the persistent kernel then takes their path).
bool any_general(const vp_handle* h) {
  for (int s : h->h_occ)
    if (h->h_inst[s].general) return true;
  return false;
}

// Some occupied slot has P2 elements (the persistent kernel then takes its P2 instance).
bool any_p2(const vp_handle* h) {
  for (int s : h->h_occ)
    if (h->h_inst[s].order == 2) return true;
  return false;
}

// k steps as cooperative persistent launches (particles in registers between steps).
vp_status advance_persistent(vp_handle* h, int k) {
  while (k > 0) {
    const int c = std::min(k, kMaxPersistSteps);
    VP_HIP(vpk::launch_slot_scalars(h->d_inst, h->d_occ, (int)h->h_occ.size(), vpk::kScalPersistStart,
                                    h->phase, h->stream));
    VP_HIP(vpk::launch_persist(h->precision, h->tun.threads, h->tun.ppt, h->d_inst, h->d_tiles, h->ntiles,
                               h->max_ng, h->any_fft, any_general(h), any_p2(h), h->phase, c,
                               h->stream));
    h->phase = (h->phase + c) % vpk::kRing;
    k -= c;
  }
  return VP_OK;
}

// Run k fused steps of every slot.  With graphs on: replays of the whole graph where it
// fits (after at most kRing-1 one-step replays that bring the phase to the graph's) and
// one-step replays for the rest; direct launches with graphs off.
vp_status advance(vp_handle* h, int k) {
  if (h->tun.persistent) return advance_persistent(h, k);
  const bool graphs = h->tun.use_graph && h->stream != nullptr;
  if (!graphs) return launch_steps_direct(h, k);
  if (k >= graph_len_of(h)) {
    VP_TRY(ensure_graph(h));  // captured at the current phase if there was none
    const int lead = (h->graph_phase - h->phase + vpk::kRing) % vpk::kRing;
    if (k - lead >= h->graph_len) {
      VP_TRY(launch_steps_graphed(h, lead));
      k -= lead;
      const int reps = k / h->graph_len;
      for (int r = 0; r < reps; ++r) VP_HIP(hipGraphLaunch(h->gexec, h->stream));
      k -= reps * h->graph_len;
    }
  }
  return launch_steps_graphed(h, k);
}

// Solve the listed slots from the live ring entry and write their field arrays (and the
// record a fused step still owes).
vp_status materialise(vp_handle* h, const int* d_slots, int nslots) {
  VP_HIP(vpk::launch_solve(h->precision, h->d_inst, d_slots, nslots, h->max_ng, h->any_fft, h->phase,
                           h->stream));
  return VP_OK;
}

vp_status materialise_all(vp_handle* h) {
  VP_TRY(materialise(h, h->d_occ, (int)h->h_occ.size()));
  h->field_stale = false;
  return VP_OK;
}

// Deposit the current positions of every slot into the live ring entry (cleared first).
vp_status deposit_all(vp_handle* h) {
  VP_HIP(vpk::launch_ring(h->precision, h->d_inst, h->d_occ, (int)h->h_occ.size(), vpk::kRingClear,
                          h->phase, h->stream));
  VP_HIP(vpk::launch_deposit(h->precision, h->tun.threads, h->d_inst, h->d_tiles, 0, h->ntiles, h->tun.ppt,
                             h->max_ng, h->phase, h->stream));
  h->acc_stale = false;
  return VP_OK;
}

int sort_chunk_of(const vp_config& c) { return c.sort_chunk > 0 ? c.sort_chunk : max_sort_chunk(c.precision); }

void to_diag(const double* r, vp_diag* o) {
  o->step = (int64_t)r[0];
  o->t = r[1];
  o->K = r[2];
  o->W = r[3];
  o->H = r[4];
  o->charge = r[5];
  o->momentum = r[6];
  o->e_amp = r[7];
  o->e1_re = r[8];
  o->e1_im = r[9];
  o->U = r[10];
  o->stamp = r[11];
}

bool diag_finite(const vp_diag& d) {
  return std::isfinite(d.K) && std::isfinite(d.W) && std::isfinite(d.U) && std::isfinite(d.H) &&
         std::isfinite(d.charge) &&
         std::isfinite(d.momentum) && std::isfinite(d.e_amp) && std::isfinite(d.e1_re) &&
         std::isfinite(d.e1_im);
}

}  // namespace

extern "C" {

int32_t vp_abi_version(void) { return VP_ABI_VERSION; }

const char* vp_status_string(vp_status s) {
  // A caller may pass any int (a ctypes binding, a cast in C): read the argument's bits as
  // an int, so that a value outside the enumeration is not loaded as the enum type.
  int v;
  std::memcpy(&v, &s, sizeof v);
  switch (v) {
    case VP_OK: return "ok";
    case VP_ERR_ARG: return "invalid argument";
    case VP_ERR_HIP: return "HIP runtime error";
    case VP_ERR_NONFINITE: return "non-finite diagnostic";
    case VP_ERR_STATE: return "invalid handle state";
    case VP_ERR_RANGE: return "history record out of range";
  }
  return "unknown status";
}

const char* vp_last_error(void) { return g_err.c_str(); }

vp_status vp_wall_clock_hz(double* hz_out) {
  if (!hz_out) return fail(VP_ERR_ARG, "hz_out is NULL");
  int dev = 0, khz = 0;
  VP_HIP(hipGetDevice(&dev));
  VP_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
  if (khz <= 0) return fail(VP_ERR_HIP, "device reports no wall-clock rate");
  *hz_out = 1e3 * (double)khz;
  return VP_OK;
}

vp_status vp_workspace_bytes(const vp_config* cfg, size_t* bytes_out) {
  VP_TRY(validate(cfg));
  if (!bytes_out) return fail(VP_ERR_ARG, "bytes_out is NULL");
  *bytes_out = vpk::workspace_layout(cfg->ng, order_of(*cfg), cfg->hist_cap, cfg->n).total;
  return VP_OK;
}

vp_status vp_engine_create(int32_t precision, int32_t max_slots, void* stream, vp_handle** out) {
  if (!out) return fail(VP_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (precision < VP_FP64 || precision > VP_FP32_TWOSUM) return fail(VP_ERR_ARG, "bad precision %d", precision);
  if (max_slots < 1 || max_slots > VP_MAX_SLOTS) return fail(VP_ERR_ARG, "max_slots = %d out of range", max_slots);
  vp_handle* h = new vp_handle();
  h->precision = precision;
  h->max_slots = max_slots;
  h->stream = static_cast<hipStream_t>(stream);
  h->slots.resize(max_slots);
  h->h_inst.assign(max_slots, InstDev{});
  // fewer polls for a persistent wait, for tests of its time-out path (never more than the
  // default; anything that does not parse as a smaller count leaves the default)
  if (const char* env = std::getenv("VP_PERSIST_SPIN_LIMIT")) {
    char* end = nullptr;
    const unsigned long v = std::strtoul(env, &end, 10);
    if (end != env && *end == '\0' && v < vpk::kSpinLimit) h->spin_limit = (unsigned)v;
  }
  std::vector<int> ids(max_slots);
  for (int i = 0; i < max_slots; ++i) ids[i] = i;
  hipError_t e = hipMalloc(&h->d_inst, max_slots * sizeof(InstDev));
  if (e == hipSuccess) e = hipMalloc(&h->d_occ, max_slots * sizeof(int));
  if (e == hipSuccess) e = hipMalloc(&h->d_ids, max_slots * sizeof(int));
  if (e == hipSuccess) e = hipMalloc(&h->d_status, 2 * (size_t)max_slots * sizeof(long long));
  if (e == hipSuccess)
    e = hipMemcpyAsync(h->d_ids, ids.data(), max_slots * sizeof(int), hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    vp_destroy(h);
    return fail(VP_ERR_HIP, "engine allocation: %s", hipGetErrorString(e));
  }
  *out = h;
  return VP_OK;
}

vp_status vp_admit(vp_handle* h, int32_t slot, const vp_config* cfg, vp_particles parts,
                   void* workspace) {
  if (!h) return fail(VP_ERR_ARG, "handle is NULL");
  VP_TRY(validate(cfg));
  if (slot < 0 || slot >= h->max_slots) return fail(VP_ERR_STATE, "slot %d out of range", slot);
  if (h->slots[slot].used) return fail(VP_ERR_STATE, "slot %d is in use", slot);
  if (cfg->precision != h->precision)
    return fail(VP_ERR_ARG, "precision %d differs from the engine's %d", cfg->precision, h->precision);
  const size_t es = state_elem_size(cfg->precision);
  const bool k3 = cfg->moment_order == 3;
  void* arrs[8] = {parts.Q, parts.P, parts.qs, parts.ps, parts.psi, parts.Mqq, parts.Mqp, parts.Mpp};
  for (int k = 0; k < (k3 ? 8 : 5); ++k)
    if (!arrs[k] || !aligned(arrs[k], es)) return fail(VP_ERR_ARG, "particle array %d NULL or misaligned", k);
  if (!k3) parts.Mqq = parts.Mqp = parts.Mpp = nullptr;
  if (!workspace || !aligned(workspace, 256)) return fail(VP_ERR_ARG, "workspace NULL or not 256-byte aligned");

  if (h->tun.persistent && cfg->moment_order == 3)
    return fail(VP_ERR_ARG, "particles with second moments are not run by persistent tuning");
  const vpk::WsLayout w = vpk::workspace_layout(cfg->ng, order_of(*cfg), cfg->hist_cap, cfg->n);
  char* ws = static_cast<char*>(workspace);
  InstDev d{};
  d.Q = parts.Q; d.P = parts.P; d.qs = parts.qs; d.ps = parts.ps; d.psi = parts.psi;
  d.n = cfg->n;
  d.ng = cfg->ng;
  d.log2ng = ilog2(cfg->ng);
  d.order = order_of(*cfg);
  d.nacc = d.order * cfg->ng;
  d.hist_cap = cfg->hist_cap;
  d.solver = cfg->solver;
  d.L = cfg->L;
  d.inv_h = (double)cfg->ng / cfg->L;
  d.h = cfg->L / (double)cfg->ng;
  d.dt = cfg->dt;
  d.acc = reinterpret_cast<double*>(ws + w.acc);
  d.E = reinterpret_cast<double*>(ws + w.E);
  d.g = reinterpret_cast<double*>(ws + w.g);
  d.Ef = reinterpret_cast<float*>(ws + w.Ef);
  d.gf = reinterpret_cast<float*>(ws + w.gf);
  d.Phi = reinterpret_cast<double*>(ws + w.Phi);
  d.bt = reinterpret_cast<double*>(ws + w.bt);
  d.tw = reinterpret_cast<double*>(ws + w.tw);
  d.inv_lam = reinterpret_cast<double*>(ws + w.inv_lam);
  d.cw = reinterpret_cast<double*>(ws + w.cw);
  d.proj = cfg->projection;
  d.self_on = cfg->no_self_field ? 0 : 1;
  d.ext_on = (cfg->ext_mode >= 1 && cfg->ext_amplitude != 0.0) ? 1 : 0;
  d.Mqq = parts.Mqq; d.Mqp = parts.Mqp; d.Mpp = parts.Mpp;
  d.k3 = k3 ? 1 : 0;
  // second moments run in the kernels' general path
  d.general = (d.proj != VP_PROJ_ELEM || !d.self_on || d.ext_on || k3) ? 1 : 0;
  d.ext_a = cfg->ext_amplitude;
  d.ext_k = 6.283185307179586 * (double)cfg->ext_mode / cfg->L;  // 2 pi m / L
  d.ext_ak = d.ext_a * d.ext_k;
  d.ext_akk = d.ext_ak * d.ext_k;
  d.scal = reinterpret_cast<vpk::InstScal*>(ws + w.scal);
  d.hist = reinterpret_cast<double*>(ws + w.hist);
  d.kin = reinterpret_cast<double*>(ws + w.kin);
  d.kin_cap = vpk::kin_capacity(cfg->n);

  // FFT twiddles and inverse stiffness eigenvalues lambda_m = (2/h)(1 - cos(2 pi m / Ng)).
  const int ng = cfg->ng;
  std::vector<double> tw(ng), il(ng);
  const double two_pi = 6.283185307179586;
  for (int k = 0; k < ng / 2; ++k) {
    tw[2 * k] = std::cos(two_pi * k / ng);
    tw[2 * k + 1] = std::sin(two_pi * k / ng);
  }
  il[0] = 0.0;
  for (int m = 1; m < ng; ++m) il[m] = 1.0 / ((2.0 / d.h) * (1.0 - std::cos(two_pi * m / ng)));
  // Taps of -M^-1 for the consistent projection, M = (h/6) circ(1, 4, 1).  On the infinite
  // mesh circ(1, 4, 1)^-1 has entries r^|d| / (2 sqrt 3), r = sqrt 3 - 2 (the root of
  // x^2 + 4x + 1 inside the unit circle); summing the periodic images gives entry
  // (r^k + r^(Ng-k)) / ((1 - r^Ng) 2 sqrt 3) at circular offset k.
  std::vector<double> cw(vpk::kConsTapsMax, 0.0);
  {
    const double r = std::sqrt(3.0) - 2.0, a = 1.0 / (2.0 * std::sqrt(3.0));
    const double rn = std::pow(r, ng);
    const int taps = vpk::cons_taps(ng), off = vpk::cons_off(ng);
    for (int t = 0; t < taps; ++t) {
      const int k = ((t + off) % ng + ng) % ng;
      const double c = a * (std::pow(r, k) + std::pow(r, ng - k)) / (1.0 - rn);
      cw[t] = -(6.0 / d.h) * c;
    }
  }

  VP_HIP(hipStreamSynchronize(h->stream));
  VP_HIP(vpk::launch_fill_zero(ws, w.total, h->stream));
  VP_HIP(hipMemcpyAsync(d.tw, tw.data(), ng * sizeof(double), hipMemcpyHostToDevice, h->stream));
  VP_HIP(hipMemcpyAsync(d.inv_lam, il.data(), ng * sizeof(double), hipMemcpyHostToDevice, h->stream));
  VP_HIP(hipMemcpyAsync(d.cw, cw.data(), cw.size() * sizeof(double), hipMemcpyHostToDevice,
                        h->stream));
  if (cfg->monopole_only) {  // p* = q* = 0 from the start
    const size_t bytes = (size_t)cfg->n * state_elem_size(cfg->precision);
    VP_HIP(vpk::launch_fill_zero(parts.qs, bytes, h->stream));
    VP_HIP(vpk::launch_fill_zero(parts.ps, bytes, h->stream));
  }
  VP_HIP(hipStreamSynchronize(h->stream));

  Slot& sl = h->slots[slot];
  sl.used = true;
  sl.cfg = *cfg;
  sl.parts = parts;
  sl.ws = workspace;
  sl.step = 0;
  sl.pending = false;
  sl.last_sort = -1;
  h->h_inst[slot] = d;
  vp_status st = rebuild_tables(h);
  if (st != VP_OK) {
    sl.used = false;
    return st;
  }
  // Load vector and field at t = 0 from the initial state (the ring entries start cleared).
  VP_HIP(vpk::launch_deposit(h->precision, h->tun.threads, h->d_inst, h->d_tiles, sl.tile_begin, sl.ntiles,
                             h->tun.ppt, h->max_ng, h->phase, h->stream));
  VP_TRY(materialise(h, h->d_ids + slot, 1));
  return VP_OK;
}

vp_status vp_create(const vp_config* cfg, vp_particles parts, void* workspace, void* stream,
                    vp_handle** out) {
  VP_TRY(validate(cfg));
  VP_TRY(vp_engine_create(cfg->precision, 1, stream, out));
  vp_status s = vp_admit(*out, 0, cfg, parts, workspace);
  if (s != VP_OK) {
    std::string keep = g_err;
    vp_destroy(*out);
    *out = nullptr;
    g_err = keep;
  }
  return s;
}

vp_status vp_create_batch(int32_t n_inst, const vp_config* cfgs, const vp_particles* parts,
                          void* const* workspaces, void* stream, vp_handle** out) {
  if (n_inst < 1 || !cfgs || !parts || !workspaces || !out) return fail(VP_ERR_ARG, "bad batch arguments");
  VP_TRY(vp_engine_create(cfgs[0].precision, n_inst, stream, out));
  for (int i = 0; i < n_inst; ++i) {
    vp_status s = vp_admit(*out, i, &cfgs[i], parts[i], workspaces[i]);
    if (s != VP_OK) {
      std::string keep = g_err;
      vp_destroy(*out);
      *out = nullptr;
      g_err = "instance " + std::to_string(i) + ": " + keep;
      return s;
    }
  }
  return VP_OK;
}

vp_status vp_retire(vp_handle* h, int32_t slot) {
  VP_TRY(check_slot(h, slot));
  Slot& sl = h->slots[slot];
  if (sl.pending) {
    VP_TRY(materialise(h, h->d_ids + slot, 1));
    VP_HIP(vpk::launch_settle(h->precision, h->tun.threads, h->d_inst, h->d_tiles, sl.tile_begin, sl.ntiles,
                              h->tun.ppt, h->max_ng, h->phase, h->stream));
    VP_HIP(vpk::launch_slot_scalars(h->d_inst, h->d_ids + slot, 1, vpk::kScalClearPending, h->phase,
                                    h->stream));
    sl.pending = false;
  }
  VP_HIP(hipStreamSynchronize(h->stream));
  sl.used = false;
  h->h_inst[slot] = InstDev{};
  return rebuild_tables(h);
}

vp_status vp_destroy(vp_handle* h) {
  if (!h) return VP_OK;
  (void)hipStreamSynchronize(h->stream);
  drop_graph(h);
  if (h->d_inst) (void)hipFree(h->d_inst);
  if (h->d_tiles) (void)hipFree(h->d_tiles);
  if (h->d_occ) (void)hipFree(h->d_occ);
  if (h->d_ids) (void)hipFree(h->d_ids);
  if (h->d_status) (void)hipFree(h->d_status);
  delete h;
  return VP_OK;
}

vp_status vp_deposit(vp_handle* h) {
  if (!h) return fail(VP_ERR_ARG, "handle is NULL");
  if (h->h_occ.empty()) return VP_OK;
  return deposit_all(h);
}

vp_status vp_poisson(vp_handle* h) {
  if (!h) return fail(VP_ERR_ARG, "handle is NULL");
  if (h->h_occ.empty()) return VP_OK;
  return materialise_all(h);
}

vp_status vp_gather_push(vp_handle* h, double kick, double drift) {
  if (!h) return fail(VP_ERR_ARG, "handle is NULL");
  if (!std::isfinite(kick) || !std::isfinite(drift)) return fail(VP_ERR_ARG, "kick and drift must be finite");
  if (h->h_occ.empty()) return VP_OK;
  if (h->field_stale) VP_TRY(materialise_all(h));
  VP_HIP(vpk::launch_gather_push(h->precision, h->tun.threads, h->d_inst, h->d_tiles, 0, h->ntiles, h->tun.ppt,
                                 h->max_ng, kick, drift, h->stream));
  if (drift != 0.0) h->acc_stale = true;
  return VP_OK;
}

vp_status vp_step(vp_handle* h, int32_t nsteps) {
  if (!h) return fail(VP_ERR_ARG, "handle is NULL");
  if (nsteps < 0) return fail(VP_ERR_ARG, "nsteps < 0");
  if (h->h_occ.empty() || nsteps == 0) return VP_OK;
  if (h->acc_stale) VP_TRY(deposit_all(h));
  int done = 0;
  while (done < nsteps) {
    // sort the slots whose step count is a multiple of their sort interval (once per step)
    for (int s : h->h_occ) {
      Slot& sl = h->slots[s];
      if (sl.cfg.sort_every > 0 && sl.step % sl.cfg.sort_every == 0 && sl.last_sort != sl.step) {
        VP_HIP(vpk::launch_sort(h->precision, h->d_inst, s, sl.cfg.n, sort_chunk_of(sl.cfg),
                                nullptr, h->stream));
        sl.last_sort = sl.step;
      }
    }
    int chunk = nsteps - done;
    for (int s : h->h_occ) {
      const Slot& sl = h->slots[s];
      if (sl.cfg.sort_every <= 0) continue;
      const long long r = sl.step % sl.cfg.sort_every;
      chunk = (int)std::min<long long>(chunk, sl.cfg.sort_every - r);
    }
    VP_TRY(advance(h, chunk));
    h->field_stale = true;
    for (int s : h->h_occ) {
      h->slots[s].step += chunk;
      h->slots[s].pending = true;
    }
    done += chunk;
  }
  return VP_OK;
}

vp_status vp_prepare_step(vp_handle* h, int32_t nsteps) {
  if (!h) return fail(VP_ERR_ARG, "handle is NULL");
  if (nsteps < 0) return fail(VP_ERR_ARG, "nsteps < 0");
  if (h->h_occ.empty() || nsteps == 0 || h->tun.persistent) return VP_OK;
  if (!h->tun.use_graph || h->stream == nullptr) return VP_OK;
  if (nsteps >= graph_len_of(h)) VP_TRY(ensure_graph(h));
  for (int p = 0; p < vpk::kRing; ++p) VP_TRY(ensure_step_graph(h, p));
  return VP_OK;
}

vp_status vp_sync_state(vp_handle* h) {
  if (!h) return fail(VP_ERR_ARG, "handle is NULL");
  if (h->h_occ.empty()) return VP_OK;
  VP_TRY(materialise_all(h));
  VP_HIP(vpk::launch_settle(h->precision, h->tun.threads, h->d_inst, h->d_tiles, 0, h->ntiles, h->tun.ppt,
                            h->max_ng, h->phase, h->stream));
  VP_HIP(vpk::launch_slot_scalars(h->d_inst, h->d_occ, (int)h->h_occ.size(), vpk::kScalClearPending,
                                  h->phase, h->stream));
  for (int s : h->h_occ) h->slots[s].pending = false;
  return VP_OK;
}

vp_status vp_sort(vp_handle* h, int32_t slot, int32_t* dev_perm) {
  if (!h) return fail(VP_ERR_ARG, "handle is NULL");
  if (slot < 0) {
    if (dev_perm) return fail(VP_ERR_ARG, "dev_perm must be NULL when sorting every slot");
    for (int s : h->h_occ)
      if (h->h_inst[s].k3) return fail(VP_ERR_ARG, "slot %d carries second moments, which are not sorted", s);
    for (int s : h->h_occ)
      VP_HIP(vpk::launch_sort(h->precision, h->d_inst, s, h->slots[s].cfg.n,
                              sort_chunk_of(h->slots[s].cfg), nullptr, h->stream));
    return VP_OK;
  }
  VP_TRY(check_slot(h, slot));
  const Slot& sl = h->slots[slot];
  if (h->h_inst[slot].k3) return fail(VP_ERR_ARG, "slot %d carries second moments, which are not sorted", slot);
  if (dev_perm && sl.cfg.n > INT32_MAX) return fail(VP_ERR_ARG, "n too large for an int32 permutation");
  VP_HIP(vpk::launch_sort(h->precision, h->d_inst, slot, sl.cfg.n, sort_chunk_of(sl.cfg), dev_perm,
                          h->stream));
  return VP_OK;
}

vp_status vp_cell_index(vp_handle* h, int32_t slot, int32_t* dev_cells) {
  VP_TRY(check_slot(h, slot));
  if (!dev_cells) return fail(VP_ERR_ARG, "dev_cells is NULL");
  VP_HIP(vpk::launch_cell_index(h->d_inst, slot, h->precision, dev_cells, h->slots[slot].cfg.n,
                                h->stream));
  return VP_OK;
}

vp_status vp_diagnostics(vp_handle* h, int32_t slot, vp_diag* host_out, double* host_grid) {
  VP_TRY(check_slot(h, slot));
  if (!host_out) return fail(VP_ERR_ARG, "host_out is NULL");
  const Slot& sl = h->slots[slot];
  const InstDev& d = h->h_inst[slot];
  VP_TRY(materialise(h, h->d_ids + slot, 1));
  VP_HIP(vpk::launch_slot_scalars(h->d_inst, h->d_ids + slot, 1, vpk::kScalClearDiag, h->phase, h->stream));
  VP_HIP(vpk::launch_diag(h->precision, h->tun.threads, h->d_inst, h->d_tiles, sl.tile_begin, sl.ntiles, h->tun.ppt,
                          h->max_ng, h->phase, h->stream));
  vpk::InstScal sc{};
  VP_HIP(hipMemcpyAsync(&sc, d.scal, sizeof sc, hipMemcpyDeviceToHost, h->stream));
  if (host_grid) {  // b~ and Phi have nacc nodes (2 ng for P2), E and g ng elements
    const int ng = sl.cfg.ng, na = d.nacc;
    VP_HIP(hipMemcpyAsync(host_grid, d.bt, na * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    VP_HIP(hipMemcpyAsync(host_grid + na, d.Phi, na * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    VP_HIP(hipMemcpyAsync(host_grid + 2 * na, d.E, ng * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    VP_HIP(hipMemcpyAsync(host_grid + 2 * na + ng, d.g, ng * sizeof(double), hipMemcpyDeviceToHost,
                          h->stream));
  }
  VP_HIP(hipStreamSynchronize(h->stream));
  host_out->step = sc.step;
  host_out->t = (double)sc.step * sl.cfg.dt;
  const int p = h->phase;
  const bool self = !sl.cfg.no_self_field;  // without a field of their own: W, E_amp, E1 are 0
  host_out->K = sc.Kd;
  host_out->U = sc.Ud;
  host_out->W = self ? sc.W[p] : 0.0;
  host_out->H = sc.Kd + sc.Ud + host_out->W;
  host_out->charge = sc.chgd;
  host_out->momentum = sc.momd;
  host_out->e_amp = std::sqrt(2.0 * host_out->W / sl.cfg.L);
  host_out->e1_re = self ? sc.e1r[p] : 0.0;
  host_out->e1_im = self ? sc.e1i[p] : 0.0;
  host_out->stamp = 0.0;
  if (sc.timeout) return fail(VP_ERR_HIP, "slot %d: a persistent step's wait for its tiles timed out", slot);
  if (!diag_finite(*host_out) || sc.nonfinite)
    return fail(VP_ERR_NONFINITE, "slot %d: non-finite diagnostics at step %lld", slot, sc.step);
  return VP_OK;
}

vp_status vp_history(vp_handle* h, int32_t slot, int64_t first_step, int32_t count,
                     vp_diag* host_out) {
  VP_TRY(check_slot(h, slot));
  if (count < 0 || (count > 0 && !host_out)) return fail(VP_ERR_ARG, "bad count or output");
  const Slot& sl = h->slots[slot];
  const InstDev& d = h->h_inst[slot];
  const long long cap = sl.cfg.hist_cap;
  if (sl.pending) VP_TRY(materialise(h, h->d_ids + slot, 1));  // the last step's record
  // the device step counter is authoritative: a frozen (non-finite) instance stops counting
  vpk::InstScal sc{};
  VP_HIP(hipMemcpyAsync(&sc, d.scal, sizeof sc, hipMemcpyDeviceToHost, h->stream));
  VP_HIP(hipStreamSynchronize(h->stream));
  const long long have = std::min<long long>(sc.step, sl.step);
  const long long lo = std::max(0LL, have - cap);
  if (first_step < lo || first_step + count > have)
    return fail(VP_ERR_RANGE, "records %lld..%lld not stored (have %lld..%lld)", (long long)first_step,
                (long long)(first_step + count - 1), lo, have - 1);
  std::vector<double> buf((size_t)count * vpk::kHistFields);
  long long k = 0;
  while (k < count) {
    const long long st = first_step + k;
    const long long pos = st % cap;
    const long long run = std::min<long long>(count - k, cap - pos);
    VP_HIP(hipMemcpy(buf.data() + k * vpk::kHistFields, d.hist + pos * vpk::kHistFields,
                     run * vpk::kHistFields * sizeof(double), hipMemcpyDeviceToHost));
    k += run;
  }
  bool finite = true;
  for (int i = 0; i < count; ++i) {
    to_diag(buf.data() + (size_t)i * vpk::kHistFields, host_out + i);
    finite = finite && diag_finite(host_out[i]);
  }
  if (!finite) return fail(VP_ERR_NONFINITE, "slot %d: non-finite records in the requested range", slot);
  return VP_OK;
}

vp_status vp_set_tuning(vp_handle* h, const vp_tuning* t) {
  if (!h || !t) return fail(VP_ERR_ARG, "NULL argument");
  if (!(t->threads == 256 || t->threads == 512 || t->threads == 1024))
    return fail(VP_ERR_ARG, "threads must be 256, 512 or 1024");
  if (!(t->ppt == 1 || t->ppt == 2 || t->ppt == 4 || t->ppt == 8 || t->ppt == 16 || t->ppt == 32 ||
        t->ppt == 64))
    return fail(VP_ERR_ARG, "ppt must be 1, 2, 4, 8, 16, 32 or 64");
  if (t->acc_copies < 1 || t->acc_copies > VP_MAX_ACC_COPIES) return fail(VP_ERR_ARG, "acc_copies out of range");
  if (t->graph_steps < 1 || t->graph_steps > 256) return fail(VP_ERR_ARG, "graph_steps out of range");
  if (t->wave_reduce != 0 && t->wave_reduce != 1) return fail(VP_ERR_ARG, "wave_reduce must be 0 or 1");
  if (t->persistent) {
    if (!(t->threads == 512 || t->threads == 1024) || !(t->ppt == 2 || t->ppt == 4 || t->ppt == 8))
      return fail(VP_ERR_ARG, "persistent steps need threads 512 or 1024 and ppt 2, 4 or 8");
    for (int s : h->h_occ)
      if (h->h_inst[s].k3)
        return fail(VP_ERR_ARG, "slot %d has particles with second moments, which persistent "
                                "steps do not run", s);
  }
  const vp_tuning old = h->tun;
  h->tun = *t;
  h->tun.use_graph = t->use_graph ? 1 : 0;
  h->tun.persistent = t->persistent ? 1 : 0;
  VP_TRY(rebuild_tables(h));
  if (h->tun.persistent) {
    const int cap = vpk::persist_capacity(h->precision, h->tun.threads, h->tun.ppt, h->max_ng,
                                          h->any_fft, any_general(h), any_p2(h));
    if (h->ntiles > cap) {
      const int need = h->ntiles;
      h->tun = old;
      VP_TRY(rebuild_tables(h));
      return fail(VP_ERR_ARG, "persistent steps need all %d workgroups resident; the device holds %d",
                  need, cap);
    }
  }
  return VP_OK;
}

vp_status vp_get_tuning(const vp_handle* h, vp_tuning* t) {
  if (!h || !t) return fail(VP_ERR_ARG, "NULL argument");
  *t = h->tun;
  return VP_OK;
}

vp_status vp_occupancy(const vp_handle* h, int32_t* slots_out, int64_t* particles_out) {
  if (!h) return fail(VP_ERR_ARG, "handle is NULL");
  int64_t p = 0;
  for (int s : h->h_occ) p += h->slots[s].cfg.n;
  if (slots_out) *slots_out = (int32_t)h->h_occ.size();
  if (particles_out) *particles_out = p;
  return VP_OK;
}

vp_status vp_slot_status(vp_handle* h, int32_t n, int64_t* host_steps, int32_t* host_flags) {
  if (!h || !host_steps || !host_flags || n < 0) return fail(VP_ERR_ARG, "NULL argument or n < 0");
  for (int32_t s = 0; s < n; ++s) {
    host_steps[s] = -1;
    host_flags[s] = 0;
  }
  const int nocc = (int)h->h_occ.size();
  if (nocc == 0) return VP_OK;
  std::vector<long long> buf(2 * (size_t)nocc);
  VP_HIP(vpk::launch_slot_status(h->d_inst, h->d_occ, nocc, h->d_status, h->stream));
  VP_HIP(hipMemcpyAsync(buf.data(), h->d_status, buf.size() * sizeof(long long),
                        hipMemcpyDeviceToHost, h->stream));
  VP_HIP(hipStreamSynchronize(h->stream));
  for (int t = 0; t < nocc; ++t) {
    const int s = h->h_occ[t];
    if (s >= n) continue;
    host_steps[s] = buf[2 * (size_t)t];
    host_flags[s] = VP_SLOT_OCCUPIED | (buf[2 * (size_t)t + 1] ? VP_SLOT_NONFINITE : 0);
  }
  return VP_OK;
}

static vp_status cluster_check(int64_t m, int32_t k) {
  if (m < 1 || m > 0x7fffffffLL) return fail(VP_ERR_ARG, "marker count %lld out of range", (long long)m);
  if (k < 1 || k > m) return fail(VP_ERR_ARG, "cluster count %d must lie in [1, m]", k);
  return VP_OK;
}

vp_status vp_cluster_workspace_bytes(int64_t m, int32_t k, size_t* bytes_out) {
  if (!bytes_out) return fail(VP_ERR_ARG, "NULL argument");
  VP_TRY(cluster_check(m, k));
  *bytes_out = vpk::cluster_layout(m, k).total;
  return VP_OK;
}

// Shared body of the two initialisation entry points (nbatch = 0: Lloyd only).
static vp_status cluster_impl(const double* Qm, const double* Pm, const double* wm, int64_t m,
                              int32_t k, const int32_t* init_idx, const int32_t* batch_idx,
                              int32_t batch, int32_t nbatch, int32_t iters, double L,
                              void* workspace, void* stream, double* Q, double* P, double* qs,
                              double* ps, double* psi, int32_t* assign_out,
                              double* absorbed_out, int32_t* n_out) {
  VP_TRY(cluster_check(m, k));
  if (!Qm || !Pm || !wm || !init_idx || !Q || !P || !qs || !ps || !psi || !n_out)
    return fail(VP_ERR_ARG, "NULL argument");
  const void* dptr[9] = {Qm, Pm, wm, Q, P, qs, ps, psi, init_idx};
  for (int i = 0; i < 9; ++i)
    if (!aligned(dptr[i], i < 8 ? 8 : 4)) return fail(VP_ERR_ARG, "argument %d misaligned", i);
  if (assign_out && !aligned(assign_out, 4)) return fail(VP_ERR_ARG, "assign_out misaligned");
  if (absorbed_out && !aligned(absorbed_out, 8)) return fail(VP_ERR_ARG, "absorbed_out misaligned");
  if (!(iters >= 0)) return fail(VP_ERR_ARG, "iters must be >= 0");
  if (!(L > 0.0) || !std::isfinite(L)) return fail(VP_ERR_ARG, "L must be positive and finite");
  if (!workspace || !aligned(workspace, 256)) return fail(VP_ERR_ARG, "workspace NULL or not 256-byte aligned");
  if (nbatch > 0 && (!batch_idx || !aligned(batch_idx, 4)))
    return fail(VP_ERR_ARG, "batch_idx NULL or misaligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  // every starting marker index must address a marker
  std::vector<int32_t> idx(k);
  VP_HIP(hipMemcpyAsync(idx.data(), init_idx, (size_t)k * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  VP_HIP(hipStreamSynchronize(s));
  for (int32_t a = 0; a < k; ++a)
    if (idx[a] < 0 || idx[a] >= m) return fail(VP_ERR_ARG, "init_idx[%d] = %d outside [0, %lld)", a, idx[a], (long long)m);
  const vpk::ClusterWs lay = vpk::cluster_layout(m, k, nbatch > 0 ? batch : 0);
  if (nbatch > 0) {  // and so must every batch index
    int bad = 0;
    VP_HIP(vpk::cluster_count_bad(batch_idx, (long long)batch * nbatch, m, workspace, lay, &bad, s));
    if (bad) return fail(VP_ERR_ARG, "%d batch indices outside [0, %lld)", bad, (long long)m);
  }
  double mm[2] = {0.0, 0.0};
  VP_HIP(vpk::cluster_p_range(Pm, m, workspace, lay, mm, s));
  if (!std::isfinite(mm[0]) || !std::isfinite(mm[1])) return fail(VP_ERR_ARG, "non-finite marker velocities");
  int n = 0;
  VP_HIP(vpk::cluster_run(Qm, Pm, wm, m, k, init_idx, batch_idx, batch, nbatch, iters, L, mm[0],
                          mm[1], workspace, lay, Q, P, qs, ps, psi, assign_out, absorbed_out, &n,
                          s));
  *n_out = n;
  return VP_OK;
}

vp_status vp_cluster_markers(const double* Qm, const double* Pm, const double* wm, int64_t m,
                             int32_t k, const int32_t* init_idx, int32_t iters, double L,
                             void* workspace, void* stream, double* Q, double* P, double* qs,
                             double* ps, double* psi, int32_t* assign_out, int32_t* n_out) {
  return cluster_impl(Qm, Pm, wm, m, k, init_idx, nullptr, 0, 0, iters, L, workspace, stream, Q,
                      P, qs, ps, psi, assign_out, nullptr, n_out);
}

vp_status vp_cluster_markers_static(const double* Qm, const double* Pm, const double* wm,
                                    int64_t m, int32_t k, const int32_t* init_idx, int32_t iters,
                                    double L, void* stream, double* Q, double* P, double* qs,
                                    double* ps, double* psi, int32_t* assign_out,
                                    int32_t* n_out) {
  VP_TRY(cluster_check(m, k));
  if (!Qm || !Pm || !wm || !init_idx || !Q || !P || !qs || !ps || !psi || !n_out)
    return fail(VP_ERR_ARG, "NULL argument");
  const void* dptr[9] = {Qm, Pm, wm, Q, P, qs, ps, psi, init_idx};
  for (int i = 0; i < 9; ++i)
    if (!aligned(dptr[i], i < 8 ? 8 : 4)) return fail(VP_ERR_ARG, "argument %d misaligned", i);
  if (assign_out && !aligned(assign_out, 4)) return fail(VP_ERR_ARG, "assign_out misaligned");
  if (!(iters >= 0)) return fail(VP_ERR_ARG, "iters must be >= 0");
  if (!(L > 0.0) || !std::isfinite(L)) return fail(VP_ERR_ARG, "L must be positive and finite");
  const vpk::ClusterWs lay = vpk::cluster_layout(m, k);
  if (lay.total > (size_t)VP_CLUSTER_STATIC_BYTES)
    return fail(VP_ERR_ARG,
                "%lld markers into %d clusters need %zu bytes of workspace; the static workspace "
                "holds %zu (vp_cluster_markers takes a workspace of any size)",
                (long long)m, k, lay.total, (size_t)VP_CLUSTER_STATIC_BYTES);
  void* ws = nullptr;
  VP_HIP(vpk::cluster_static_workspace(&ws));
  hipStream_t s = static_cast<hipStream_t>(stream);
  // the array keeps the previous call's contents: this call's part starts cleared
  VP_HIP(vpk::launch_fill_zero(ws, lay.total, s));
  // every starting marker index must address a marker (counted on the device)
  int bad = 0;
  VP_HIP(vpk::cluster_count_bad(init_idx, k, m, ws, lay, &bad, s));
  if (bad) return fail(VP_ERR_ARG, "%d starting indices outside [0, %lld)", bad, (long long)m);
  double mm[2] = {0.0, 0.0};
  VP_HIP(vpk::cluster_p_range(Pm, m, ws, lay, mm, s));
  if (!std::isfinite(mm[0]) || !std::isfinite(mm[1])) return fail(VP_ERR_ARG, "non-finite marker velocities");
  int n = 0;
  VP_HIP(vpk::cluster_run(Qm, Pm, wm, m, k, init_idx, nullptr, 0, 0, iters, L, mm[0], mm[1], ws,
                          lay, Q, P, qs, ps, psi, assign_out, nullptr, &n, s));
  *n_out = n;
  return VP_OK;
}

static vp_status minibatch_check(int64_t m, int32_t k, int32_t batch, int32_t nbatch) {
  VP_TRY(cluster_check(m, k));
  if (batch < 1 || batch > m) return fail(VP_ERR_ARG, "batch = %d must lie in [1, m]", batch);
  if (nbatch < 1) return fail(VP_ERR_ARG, "nbatch must be >= 1");
  if ((long long)batch * nbatch > 0x7fffffffLL)
    return fail(VP_ERR_ARG, "batch * nbatch = %lld exceeds 2^31 - 1", (long long)batch * nbatch);
  return VP_OK;
}

vp_status vp_cluster_minibatch_workspace_bytes(int64_t m, int32_t k, int32_t batch,
                                               size_t* bytes_out) {
  if (!bytes_out) return fail(VP_ERR_ARG, "NULL argument");
  VP_TRY(minibatch_check(m, k, batch, 1));
  *bytes_out = vpk::cluster_layout(m, k, batch).total;
  return VP_OK;
}

vp_status vp_cluster_markers_minibatch(const double* Qm, const double* Pm, const double* wm,
                                       int64_t m, int32_t k, const int32_t* init_idx,
                                       const int32_t* batch_idx, int32_t batch, int32_t nbatch,
                                       double L, void* workspace, void* stream, double* Q,
                                       double* P, double* qs, double* ps, double* psi,
                                       int32_t* assign_out, double* absorbed_out,
                                       int32_t* n_out) {
  VP_TRY(minibatch_check(m, k, batch, nbatch));
  return cluster_impl(Qm, Pm, wm, m, k, init_idx, batch_idx, batch, nbatch, 0, L, workspace,
                      stream, Q, P, qs, ps, psi, assign_out, absorbed_out, n_out);
}

vp_status vp_tune_scratch_bytes(const vp_handle* h, size_t* bytes_out) {
  if (!h || !bytes_out) return fail(VP_ERR_ARG, "NULL argument");
  size_t b = 0;
  for (int s : h->h_occ) {
    const Slot& sl = h->slots[s];
    b += ((size_t)state_arrays(sl.cfg) * sl.cfg.n * state_elem_size(h->precision) + 255) & ~size_t(255);
    b += vpk::workspace_layout(sl.cfg.ng, order_of(sl.cfg), sl.cfg.hist_cap, sl.cfg.n).total;
  }
  *bytes_out = b;
  return VP_OK;
}

namespace {
// Copy the state of every occupied slot (its particle arrays, which a scheduled sort
// permutes, and the workspace) to or from
// the tuner scratch buffer.
vp_status tune_copy(vp_handle* h, char* scratch, bool save) {
  size_t off = 0;
  for (int s : h->h_occ) {
    const Slot& sl = h->slots[s];
    const size_t es = state_elem_size(h->precision);
    void* arrs[8] = {sl.parts.Q,  sl.parts.P,   sl.parts.qs,  sl.parts.ps,
                     sl.parts.psi, sl.parts.Mqq, sl.parts.Mqp, sl.parts.Mpp};
    const int na = state_arrays(sl.cfg);
    for (int k = 0; k < na; ++k) {
      char* sp = scratch + off + (size_t)k * sl.cfg.n * es;
      if (save) VP_HIP(hipMemcpyAsync(sp, arrs[k], sl.cfg.n * es, hipMemcpyDeviceToDevice, h->stream));
      else VP_HIP(hipMemcpyAsync(arrs[k], sp, sl.cfg.n * es, hipMemcpyDeviceToDevice, h->stream));
    }
    off += ((size_t)na * sl.cfg.n * es + 255) & ~size_t(255);
    const size_t wb = vpk::workspace_layout(sl.cfg.ng, order_of(sl.cfg), sl.cfg.hist_cap, sl.cfg.n).total;
    if (save) VP_HIP(hipMemcpyAsync(scratch + off, sl.ws, wb, hipMemcpyDeviceToDevice, h->stream));
    else VP_HIP(hipMemcpyAsync(sl.ws, scratch + off, wb, hipMemcpyDeviceToDevice, h->stream));
    off += wb;
  }
  return VP_OK;
}
}  // namespace

vp_status vp_tune(vp_handle* h, void* dev_scratch, int32_t steps_per_trial, vp_tuning* best_out,
                  double* best_us_per_step_out) {
  if (!h || !dev_scratch) return fail(VP_ERR_ARG, "NULL argument");
  if (steps_per_trial < 1) return fail(VP_ERR_ARG, "steps_per_trial < 1");
  if (h->h_occ.empty()) return fail(VP_ERR_STATE, "no occupied slot to tune on");
  char* scratch = static_cast<char*>(dev_scratch);
  std::vector<Slot> saved = h->slots;
  const vp_tuning orig = h->tun;
  const int saved_phase = h->phase;
  const bool saved_fs = h->field_stale, saved_as = h->acc_stale;
  VP_TRY(tune_copy(h, scratch, true));
  hipEvent_t e0, e1;
  VP_HIP(hipEventCreate(&e0));
  VP_HIP(hipEventCreate(&e1));
  vp_tuning best = orig;
  double best_us = 1e300;
  struct Cand { int threads, ppt, acc, persistent; };
  std::vector<Cand> cands;
  long long nmax = 0;
  for (int s : h->h_occ) nmax = std::max<long long>(nmax, h->slots[s].cfg.n);
  for (int th : {512, 1024})
    for (int pp : {1, 2, 4, 8, 16, 32})
      if (pp <= 8 || (long long)th * pp * 512 <= nmax)  // big tiles only for big instances
        for (int ac : {1, 2, 4, 8}) cands.push_back({th, pp, ac, 0});
  // persistent shapes that keep every tile resident
  for (int th : {512, 1024})
      for (int pp : {2, 4, 8}) {
        const long long tiles_needed = [&] {
          long long t = 0;
          for (int s : h->h_occ) t += (h->slots[s].cfg.n + (long long)th * pp - 1) / ((long long)th * pp);
          return t;
        }();
        if (tiles_needed <= vpk::persist_capacity(h->precision, th, pp, h->max_ng, h->any_fft,
                                                  any_general(h), any_p2(h)))
          for (int ac : {1, 2, 4, 8}) cands.push_back({th, pp, ac, 1});
      }
  vp_status st = VP_OK;
  // one trial: set the shape, one untimed graph build + warm-up pass, the timed steps, then
  // the saved state back.  Returns false when a persistent shape cannot keep every tile
  // resident (skipped); st carries any error.
  auto trial = [&](vp_tuning t) -> bool {
    t.use_graph = (h->stream != nullptr) ? 1 : 0;
    t.graph_steps = std::min(steps_per_trial, 256);
    st = vp_set_tuning(h, &t);
    if (st == VP_ERR_ARG && t.persistent) {  // this shape cannot keep every tile resident
      st = VP_OK;
      return false;
    }
    if (st != VP_OK) return false;
    st = vp_step(h, t.graph_steps);
    if (st != VP_OK) return false;
    if (hipEventRecord(e0, h->stream) != hipSuccess) { st = fail(VP_ERR_HIP, "event record"); return false; }
    st = vp_step(h, steps_per_trial);
    if (st != VP_OK) return false;
    float ms = 0.f;
    if (hipEventRecord(e1, h->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      st = fail(VP_ERR_HIP, "event timing");
      return false;
    }
    const double us = 1000.0 * ms / steps_per_trial;
    if (us < best_us) {
      best_us = us;
      best = t;
    }
    h->slots = saved;
    h->phase = saved_phase;
    h->field_stale = saved_fs;
    h->acc_stale = saved_as;
    st = tune_copy(h, scratch, false);
    return true;
  };
  for (size_t ci = 0; ci < cands.size() && st == VP_OK; ++ci) {
    vp_tuning t = orig;
    t.threads = cands[ci].threads;
    t.ppt = cands[ci].ppt;
    t.acc_copies = cands[ci].acc;
    t.persistent = cands[ci].persistent;
    t.wave_reduce = 0;
    trial(t);
  }
  // the wavefront-combined deposit (compensated float32 pairs only), at the fastest shape
  if (st == VP_OK && best_us < 1e300 && h->precision == VP_FP32_TWOSUM) {
    vp_tuning t = best;
    t.wave_reduce = 1;
    trial(t);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  h->slots = saved;
  h->phase = saved_phase;
  h->field_stale = saved_fs;
  h->acc_stale = saved_as;
  vp_status s2 = tune_copy(h, scratch, false);
  vp_status s3 = vp_set_tuning(h, st == VP_OK ? &best : &orig);
  if (st != VP_OK) return st;
  if (s2 != VP_OK) return s2;
  if (s3 != VP_OK) return s3;
  if (best_out) *best_out = best;
  if (best_us_per_step_out) *best_us_per_step_out = best_us;
  return VP_OK;
}

}  // extern "C"
