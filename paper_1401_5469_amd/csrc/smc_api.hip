// smc_api.hip -- host runtime behind the C ABI declared in include/smc.h:
// validation, workspace layout, uploads, launch sequencing and read-back.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "../../include/smc.h"
#include "smc_internal.h"

// Multi-model launches stage their model table in pinned host memory and
// copy it to a device table; a launch takes a slot whose last launch has
// finished (event per slot), so that launches in flight on several streams
// never make the host wait while a slot is free.
constexpr int kBatchSlots = 8;

struct smc_ctx {
  int device;
  int n_cu;
  int transport_blocks_per_cu[2];  // occupancy of the lane-per-packet kernel (single, multi)
  int long_blocks_per_cu[2][3][2];  // occupancy of the group-per-packet kernel
                                    // [multi][16, 32, 64 lanes][plain, extended]
  smc::BatchEntry* host_table[kBatchSlots];   // pinned
  smc::BatchEntry* dev_table[kBatchSlots];
  unsigned long long* dev_ctr[kBatchSlots];   // launch-wide control blocks (kCtlBytes)
  hipEvent_t slot_done[kBatchSlots];
  bool slot_used[kBatchSlots];
  int next_slot;
  hipEvent_t ev_start, ev_stop;               // timing of the last batch
  bool batch_timed;
  uint8_t* scratch;  // device address of this device's copy of `scratch`
};

struct smc_model {
  smc_ctx* ctx;
  smc::Layout lay;
  smc::DevModel dev;
  uint8_t* base;
  unsigned int* order_hist;  // this model's hand-off order histogram (single-model launches)
  uint64_t ws_bytes;
  uint64_t n_packets_max;
  uint32_t load_flags;
  bool has_T;        // a previous iteration left a T_inner on the device
  bool ran;          // at least one iteration ran
  uint32_t last_flags;
  uint64_t last_work;
  bool last_virtual;  // the last iteration ran v-packets
  hipEvent_t ev_start, ev_stop;  // created on the first timed iteration
  bool timed;                    // the last iteration recorded ev_start/ev_stop
  smc_tune tune;
  int32_t n_levels;     // macro-atom levels (0 in scatter mode)
  bool derived_tables;  // macroatom rows laid out by a plasma object, em_cum from its updates
  bool tables_ready;    // false until the first plasma update has derived them
};

// A plasma object bound to a model (see smc_plasma_load).
struct smc_plasma {
  smc_model* model;
  smc::PlasmaLayout lay;
  smc::DevPlasma dev;
  uint8_t* base;
  int32_t n_nlte;
  bool updated;
};

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int ok() {
  g_err.clear();
  return SMC_OK;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(SMC_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                 \
  do {                                      \
    hipError_t e_ = (expr);                 \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

constexpr uint64_t kAlign = 256;
// flight segments before a history moves to the group kernel unless tuned:
// fewer for one model in a plain mode (its longest histories start sooner),
// more with macro atoms (their group-kernel variant carries more registers
// and runs fewer histories at once), most in multi-model launches of the
// plain modes (where throughput matters more than the latency of one
// history: the coordinate search picks 4096 on the 64-model mix)
constexpr uint32_t kDefaultLongBudget = 256;
constexpr uint32_t kDefaultLongBudgetWide = 1024;
constexpr uint32_t kDefaultLongBudgetMulti = 4096;
// lanes per handed-off history unless tuned: one history per wavefront (its
// segments have the shortest latency) for one model in the plain modes,
// four per wavefront in their multi-model launches (the search's pick on
// the 64-model mix), two per wavefront in the group kernel variant with the
// macro-atom and v-packet code
constexpr int kDefaultLongLanes = 64;
constexpr int kDefaultLongLanesMulti = 16;
constexpr int kDefaultLongLanesExt = 32;
// wavefronts per CU of the group-per-packet kernel unless tuned (fewer when
// its occupancy allows fewer): 16 one-history wavefronts, else 12
constexpr int kDefaultLongWaves = 12;
constexpr int kDefaultSoloWaves = 16;
// launch-wide control block of a multi-model launch: 4 queue counters, then
// the hand-off order histogram and cursors
constexpr size_t kCtlBytes = 4 * sizeof(unsigned long long) + 2 * smc::kOrderBuckets * 4;

// Launch-wide scratch of smc_batch_run_static, which allocates nothing: the
// control block (queue heads, hand-off order histogram and cursors), then the
// device model table.  Every GPU the library runs on holds one copy until the
// process ends; its device address is looked up once per context.
constexpr size_t kScratchBytes = 128 * 1024;
constexpr size_t kScratchTableOffset = (kCtlBytes + 255) / 256 * 256;
constexpr int kScratchModels =
    (int)((kScratchBytes - kScratchTableOffset) / sizeof(smc::BatchEntry));
static_assert(kScratchModels >= SMC_STATIC_MAX_MODELS, "the scratch holds the largest batch");
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

void release_ctx(smc_ctx* c) {
  if (!c) return;
  for (int i = 0; i < kBatchSlots; ++i) {
    if (c->slot_done[i]) (void)hipEventSynchronize(c->slot_done[i]);
    if (c->host_table[i]) (void)hipHostFree(c->host_table[i]);
    if (c->dev_table[i]) (void)hipFree(c->dev_table[i]);
    if (c->dev_ctr[i]) (void)hipFree(c->dev_ctr[i]);
    if (c->slot_done[i]) (void)hipEventDestroy(c->slot_done[i]);
  }
  if (c->ev_start) (void)hipEventDestroy(c->ev_start);
  if (c->ev_stop) (void)hipEventDestroy(c->ev_stop);
  delete c;
}

int lanes_of(const smc_tune& t, bool ext, bool multi) {
  if (t.long_lanes != 0) return (int)t.long_lanes;
  return ext ? kDefaultLongLanesExt : (multi ? kDefaultLongLanesMulti : kDefaultLongLanes);
}
int lanes_index(int lanes) { return lanes == 16 ? 0 : (lanes == 32 ? 1 : 2); }

int default_long_waves(const smc_ctx* c, bool multi, const smc_tune& t, bool ext) {
  const int lanes = lanes_of(t, ext, multi);
  const int occ = c->long_blocks_per_cu[multi][lanes_index(lanes)][ext];
  const int want = (lanes == 64 && !ext) ? kDefaultSoloWaves : kDefaultLongWaves;
  return occ < want ? occ : want;
}

int check_tune(const smc_tune& t) {
  if (t.blocks_per_cu < 0 || t.blocks_per_cu > 64 || t.long_waves_per_cu < 0 ||
      t.long_waves_per_cu > 64)
    return fail(SMC_EINVAL, "blocks_per_cu and long_waves_per_cu must lie in [0, 64]");
  if (t.long_lanes != 0 && t.long_lanes != 16 && t.long_lanes != 32 && t.long_lanes != 64)
    return fail(SMC_EINVAL, "long_lanes must be 0, 16, 32 or 64 (got %u)", t.long_lanes);
  return 0;
}

// hand-off positions run at the highest wave priority: two histories per SIMD
// hand-off positions that run at the highest wave priority: one wavefront's
// histories per SIMD (4 SIMDs per CU), so that no two top-priority
// wavefronts share a SIMD
uint32_t hot_of(const smc_ctx* c, const smc_tune& t, bool ext, bool multi) {
  return 4u * (uint32_t)c->n_cu * (uint32_t)(64 / lanes_of(t, ext, multi));
}

uint32_t budget_of(const smc_tune& t, bool macro, bool multi) {
  if (t.long_budget == 0)
    return macro ? kDefaultLongBudgetWide : (multi ? kDefaultLongBudgetMulti : kDefaultLongBudget);
  return t.long_budget == UINT32_MAX ? 0u : t.long_budget;
}

// launch shape from the tuning (0 = occupancy default), capped by the work
smc::Shape shape_of(const smc_ctx* c, const smc_tune& t, bool multi, uint64_t n_work,
                    bool handoff, bool ext) {
  smc::Shape sh;
  const int block = smc::transport_block_threads();
  uint64_t want = (n_work + block - 1) / block;
  const int per_cu = t.blocks_per_cu > 0 ? t.blocks_per_cu : c->transport_blocks_per_cu[multi];
  const uint64_t cap = (uint64_t)c->n_cu * (uint64_t)per_cu;
  sh.transport_grid = (int)(want > cap ? cap : want);
  uint64_t lgrid = 0;
  if (handoff && n_work > 0) {
    const int lper =
        t.long_waves_per_cu > 0 ? t.long_waves_per_cu : default_long_waves(c, multi, t, ext);
    lgrid = (uint64_t)c->n_cu * (uint64_t)lper;
    if (lgrid > n_work) lgrid = n_work;
  }
  sh.long_grid = (int)lgrid;
  sh.long_lanes = lanes_of(t, ext, multi);
  sh.long_ext = ext;
  return sh;
}

// validate one iteration's parameters against its model; fill the device view
int make_iter(const smc_model* m, const smc_iter_params* p, uint32_t budget, smc::DevIter* it) {
  if (!p) return fail(SMC_EINVAL, "null parameters");
  if (m->derived_tables && !m->tables_ready)
    return fail(SMC_EINVAL,
                "the macro-atom tables are derived from the plasma state: load a plasma object "
                "and run smc_plasma_update before the first iteration");
  if (p->n_packets == 0) return fail(SMC_EINVAL, "n_packets must be >= 1");
  if (p->flags & ~(SMC_F_JBLUE | SMC_F_PACKETS | SMC_F_TIMING))
    return fail(SMC_EINVAL, "unknown flags");
  if ((p->flags & ~m->load_flags & (SMC_F_JBLUE | SMC_F_PACKETS)) != 0)
    return fail(SMC_EINVAL, "iteration flags 0x%x exceed the model's load flags 0x%x", p->flags,
                m->load_flags);
  if (p->packet_ids == nullptr && p->n_ids != 0)
    return fail(SMC_EINVAL, "n_ids given without packet_ids");
  const uint64_t n_work = p->packet_ids ? p->n_ids : p->n_packets;
  if (n_work > m->n_packets_max)
    return fail(SMC_ENOMEM, "%llu packets exceed the model's n_packets_max=%llu",
                (unsigned long long)n_work, (unsigned long long)m->n_packets_max);
  if (!(p->T_inner > 0.0) && !m->has_T)
    return fail(SMC_EINVAL, "T_inner must be > 0 on the first iteration");
  if (!isfinite(p->T_inner)) return fail(SMC_EINVAL, "T_inner must be finite");
  if (p->L_requested > 0.0 && !(p->damping > 0.0 && p->damping <= 1.0))
    return fail(SMC_EINVAL, "damping must lie in (0, 1]");
  if (p->max_segments < 1 || p->max_segments > (1ull << 30))
    return fail(SMC_EINVAL, "max_segments must lie in [1, 2^30]");
  if (p->n_virtual > smc::kMaxVirtual)
    return fail(SMC_EINVAL, "n_virtual=%u exceeds %u", p->n_virtual, smc::kMaxVirtual);
  if (p->reserved != 0) return fail(SMC_EINVAL, "reserved must be 0");
  it->n_packets = p->n_packets;
  it->n_work = n_work;
  it->ids = p->packet_ids;
  it->max_segments = p->max_segments;
  it->iteration = p->iteration;
  it->flags = p->flags;
  it->long_budget = budget;
  it->n_virtual = p->n_virtual;
  it->T_param = p->T_inner;
  it->L_requested = p->L_requested;
  it->damping = p->damping;
  return SMC_OK;
}

uint64_t jblue_entries(const smc_model* m, uint32_t flags) {
  return (m->dev.jblue && (flags & SMC_F_JBLUE)) ? (uint64_t)m->dev.S * (uint64_t)m->dev.L : 0;
}
constexpr int kMaxBins = 8192;
constexpr int kMaxShells = 4096;

uint64_t align_up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// A macroatom model loaded without tables takes them from a plasma object:
// three entries per line (a deactivation and an internal jump down in the
// upper level's row, a jump up in the lower level's row).
bool derived_macroatom(const smc_model_desc* d) {
  return d->line_mode == SMC_MACROATOM && !d->level_ptr && !d->em_line && !d->em_cum;
}

int64_t em_entries(const smc_model_desc* d) {
  return derived_macroatom(d) ? 3 * d->n_lines : d->n_em;
}

uint64_t em_cum_entries(const smc_model_desc* d) {
  return d->line_mode == SMC_MACROATOM ? (uint64_t)d->n_shells * (uint64_t)em_entries(d)
                                       : (uint64_t)d->n_em;
}

// Copies between a host [rows][width] array and a device one of row pitch
// `pitch`, one plain copy per row (one copy in all when the rows are not
// padded): strided copies from or to pageable host memory are avoided.
hipError_t copy_rows(void* dst, size_t dpitch, const void* src, size_t spitch, size_t width,
                     size_t rows, hipMemcpyKind kind, hipStream_t s) {
  if (dpitch == width && spitch == width) return hipMemcpyAsync(dst, src, width * rows, kind, s);
  for (size_t r = 0; r < rows; ++r) {
    const hipError_t e = hipMemcpyAsync((uint8_t*)dst + r * dpitch,
                                        (const uint8_t*)src + r * spitch, width, kind, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// A workspace must be device memory of the context's device from hipMalloc
// (coarse-grained): the tallies are FP64 atomic adds, which host and managed
// memory do not guarantee.
int check_workspace(const void* ptr, int device) {
  hipPointerAttribute_t at;
  memset(&at, 0, sizeof at);
  const hipError_t e = hipPointerGetAttributes(&at, ptr);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(SMC_EINVAL, "the workspace is not memory the HIP runtime knows (%s)",
                hipGetErrorString(e));
  }
  if (at.type != hipMemoryTypeDevice || at.isManaged)
    return fail(SMC_EINVAL, "the workspace must be device memory from hipMalloc, not host or "
                            "managed memory");
  if (at.device != device)
    return fail(SMC_EINVAL, "the workspace is memory of device %d, the context's is %d",
                at.device, device);
  return SMC_OK;
}

int validate(const smc_model_desc* d) {
  if (!d) return fail(SMC_EINVAL, "null model description");
  if (d->n_shells < 1 || d->n_shells > kMaxShells)
    return fail(SMC_EINVAL, "n_shells=%d outside [1, %d]", d->n_shells, kMaxShells);
  if (d->n_lines < 0 || d->n_lines > INT32_MAX)
    return fail(SMC_EINVAL, "n_lines=%lld outside [0, 2^31)", (long long)d->n_lines);
  if (d->n_bins < 1 || d->n_bins > kMaxBins)
    return fail(SMC_EINVAL, "n_bins=%d outside [1, %d]", d->n_bins, kMaxBins);
  if (!d->v_bounds || !d->n_e) return fail(SMC_EINVAL, "null shell arrays");
  if (d->n_lines > 0 && (!d->line_nu || !d->tau_sobolev)) return fail(SMC_EINVAL, "null line arrays");
  if (!(d->t_exp > 0.0) || !isfinite(d->t_exp)) return fail(SMC_EINVAL, "t_exp must be > 0");
  if (!(d->nu_max > d->nu_min) || !isfinite(d->nu_max) || !isfinite(d->nu_min))
    return fail(SMC_EINVAL, "spectrum range must satisfy nu_min < nu_max");
  for (int i = 0; i <= d->n_shells; ++i) {
    if (!(d->v_bounds[i] > 0.0) || !isfinite(d->v_bounds[i]))
      return fail(SMC_EINVAL, "v_bounds[%d] must be finite and > 0", i);
    if (i > 0 && !(d->v_bounds[i] > d->v_bounds[i - 1]))
      return fail(SMC_EINVAL, "v_bounds must be strictly increasing (index %d)", i);
  }
  // first-order Doppler factors: D = 1 - mu v / c stays above 1/2, so lab
  // energies stay below 2 packet units and their fixed-point sums cannot
  // overflow
  if (!(d->v_bounds[d->n_shells] < 0.5 * 2.99792458e10))
    return fail(SMC_EINVAL, "outer velocity must be below c/2");
  // radii within [2^-300, 2^300] cm keep every squared distance the kernels
  // take a root of either zero or a normal number
  if (!(d->v_bounds[0] * d->t_exp >= 0x1p-300) ||
      !(d->v_bounds[d->n_shells] * d->t_exp <= 0x1p300))
    return fail(SMC_EINVAL, "radii v t_exp must lie in [2^-300, 2^300] cm");
  for (int i = 0; i < d->n_shells; ++i)
    if (!(d->n_e[i] >= 0.0) || !(d->n_e[i] <= 1e200))
      return fail(SMC_EINVAL, "n_e[%d] must lie in [0, 1e200]", i);
  for (int64_t k = 0; k < d->n_lines; ++k) {
    if (!(d->line_nu[k] > 0.0) || !isfinite(d->line_nu[k]))
      return fail(SMC_EINVAL, "line_nu[%lld] must be finite and > 0", (long long)k);
    if (k > 0 && !(d->line_nu[k] <= d->line_nu[k - 1]))
      return fail(SMC_EINVAL, "line_nu must be non-increasing (index %lld)", (long long)k);
  }
  const int64_t n_tau = (int64_t)d->n_shells * d->n_lines;
  for (int64_t i = 0; i < n_tau; ++i)
    if (!(d->tau_sobolev[i] >= 0.0) || !isfinite(d->tau_sobolev[i]))
      return fail(SMC_EINVAL, "tau_sobolev[%lld] must be finite and >= 0", (long long)i);
  if (d->line_mode != SMC_SCATTER && d->line_mode != SMC_DOWNBRANCH &&
      d->line_mode != SMC_MACROATOM)
    return fail(SMC_EINVAL, "unknown line_mode %d", d->line_mode);
  if (derived_macroatom(d) && d->n_lines > 0) {
    if (!d->line_upper || d->n_levels < 1)
      return fail(SMC_EINVAL, "a macroatom model with derived tables needs line_upper and "
                              "n_levels >= 1");
    if (d->n_em != 0) return fail(SMC_EINVAL, "n_em must be 0 when the tables are derived");
    for (int64_t k = 0; k < d->n_lines; ++k)
      if (d->line_upper[k] < 0 || d->line_upper[k] >= d->n_levels)
        return fail(SMC_EINVAL, "line_upper[%lld] out of range", (long long)k);
  } else if (d->line_mode != SMC_SCATTER && d->n_lines > 0) {
    const bool macro = d->line_mode == SMC_MACROATOM;
    if (!d->line_upper || !d->level_ptr || !d->em_line || !d->em_cum || d->n_levels < 1)
      return fail(SMC_EINVAL, "macro-atom modes need line_upper, level_ptr, em_line, em_cum");
    if (d->level_ptr[0] != 0 || d->level_ptr[d->n_levels] != d->n_em)
      return fail(SMC_EINVAL, "level_ptr must run from 0 to n_em");
    for (int32_t v = 0; v < d->n_levels; ++v)
      if (d->level_ptr[v + 1] < d->level_ptr[v])
        return fail(SMC_EINVAL, "level_ptr must be non-decreasing (level %d)", v);
    for (int64_t j = 0; j < d->n_em; ++j) {
      const int32_t t = d->em_line[j];
      if (t >= d->n_lines || (t < 0 && !macro))
        return fail(SMC_EINVAL, "em_line[%lld] out of range", (long long)j);
      if (t < 0) {
        const int64_t lv = -(int64_t)t - 1;
        if (lv >= d->n_levels || !(d->level_ptr[lv + 1] > d->level_ptr[lv]))
          return fail(SMC_EINVAL, "em_line[%lld] jumps to level %lld, which has no row",
                      (long long)j, (long long)lv);
      }
    }
    const int64_t n_cum = macro ? (int64_t)d->n_shells * d->n_em : d->n_em;
    for (int64_t j = 0; j < n_cum; ++j)
      if (!(d->em_cum[j] >= 0.0 && d->em_cum[j] <= 1.0))
        return fail(SMC_EINVAL, "em_cum[%lld] must lie in [0, 1]", (long long)j);
    // the kernels select an entry by bisection, which needs sorted rows
    for (int64_t t = 0; t < n_cum; t += d->n_em)
      for (int32_t v = 0; v < d->n_levels; ++v)
        for (int64_t j = d->level_ptr[v] + 1; j < d->level_ptr[v + 1]; ++j)
          if (d->em_cum[t + j] < d->em_cum[t + j - 1])
            return fail(SMC_EINVAL, "em_cum must be non-decreasing within a row (entry %lld)",
                        (long long)(t + j));
    for (int64_t k = 0; k < d->n_lines; ++k) {
      const int32_t u = d->line_upper[k];
      if (u < 0 || u >= d->n_levels)
        return fail(SMC_EINVAL, "line_upper[%lld] out of range", (long long)k);
      if (!(d->level_ptr[u + 1] > d->level_ptr[u]))
        return fail(SMC_EINVAL, "upper level %d of line %lld has no emission row", u,
                    (long long)k);
    }
  }
  return SMC_OK;
}

smc::Layout layout_of(const smc_model_desc* d, uint64_t n_packets_max, uint32_t flags) {
  smc::Layout l;
  memset(&l, 0, sizeof l);
  const uint64_t S = (uint64_t)d->n_shells, L = (uint64_t)d->n_lines;
  const uint64_t NB = (uint64_t)d->n_bins + 2;
  uint64_t off = 0;
  auto take = [&](uint64_t bytes) {
    const uint64_t o = off;
    off = align_up(off + (bytes ? bytes : 1));
    return o;
  };
  l.r_bounds = take((S + 1) * 8);
  l.v_bounds = take((S + 1) * 8);
  l.n_e = take(S * 8);
  l.volume = take(S * 8);
  const uint64_t Lp = (L + 3) / 4 * 4;  // rows padded for aligned 4-line loads
  l.line_nu = take(Lp * 8);
  l.tau = take(S * Lp * 8);
  if (d->line_mode != SMC_SCATTER) {
    l.line_upper = take(L * 4);
    l.level_ptr = take(((uint64_t)d->n_levels + 1) * 8);
    l.em_line = take((uint64_t)em_entries(d) * 4);
    l.em_cum = take(em_cum_entries(d) * 8);
  }
  l.raw = take((2 * S + NB) * 8);
  l.lsum = take(4 * 8);
  l.counters = take(smc::CTR_TOTAL * 8);
  l.longs = take(n_packets_max * sizeof(smc::LongState));
  l.long_order = take(n_packets_max * 8);
  l.long_hist = take(2 * smc::kOrderBuckets * 4);
  l.jblue = (flags & SMC_F_JBLUE) ? take(S * L * 8) : 0;
  l.out_shell = take(6 * S * 8);
  l.out_spec = take(NB * 8);
  l.vraw = take(NB * 8);
  l.vcounts = take(4 * 8);
  l.out_vspec = take((NB + 1) * 8);
  l.scalars = take(8 * 8);
  l.packets = (flags & SMC_F_PACKETS) ? take(n_packets_max * sizeof(smc_packet_out)) : 0;
  l.total = off;
  return l;
}

int sync_copy_out(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (!dst || bytes == 0) return SMC_OK;
  HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
  return SMC_OK;
}

// Validate the parameters of a plasma update and fill the kernels' arguments,
// with the radiation field taken from the model (a caller giving host arrays
// stages them and repoints T_R and W).  after_iteration: an iteration of the
// model precedes the update in stream order (always in a captured sequence),
// so a detailed J_b reads that iteration's J_blue.
int plasma_args(const smc_plasma* p, const smc_plasma_params* pp, bool after_iteration,
                smc::DevPlasma* d) {
  if (!p || !pp) return fail(SMC_EINVAL, "null plasma or parameters");
  if (pp->ionization != SMC_ION_LTE && pp->ionization != SMC_ION_NEBULAR)
    return fail(SMC_EINVAL, "unknown ionization mode %d", pp->ionization);
  if (pp->excitation != SMC_EXC_LTE && pp->excitation != SMC_EXC_DILUTE_LTE)
    return fail(SMC_EINVAL, "unknown excitation mode %d", pp->excitation);
  if (!(pp->delta >= 0.0) || !isfinite(pp->delta))
    return fail(SMC_EINVAL, "delta must be finite and >= 0");
  if ((pp->T_R == nullptr) != (pp->W == nullptr))
    return fail(SMC_EINVAL, "give both T_R and W, or neither");
  if (pp->nlte != 0 && pp->nlte != 1) return fail(SMC_EINVAL, "nlte must be 0 or 1");
  if (pp->jblue_mode != SMC_JB_DILUTE_BLACKBODY && pp->jblue_mode != SMC_JB_DETAILED)
    return fail(SMC_EINVAL, "unknown J_b mode %d", pp->jblue_mode);
  const smc_model* m = p->model;
  const bool detailed = pp->nlte && p->n_nlte > 0 && pp->jblue_mode == SMC_JB_DETAILED;
  const bool macro_detailed = m->derived_tables && pp->jblue_mode == SMC_JB_DETAILED;
  if ((detailed || macro_detailed) && !m->dev.jblue)
    return fail(SMC_EINVAL, "detailed J_b needs a model loaded with SMC_F_JBLUE");
  *d = p->dev;
  d->ionization = pp->ionization;
  d->excitation = pp->excitation;
  d->delta = pp->delta;
  d->n_nlte = pp->nlte ? p->n_nlte : 0;
  d->jb_detailed = detailed && after_iteration ? 1 : 0;  // before any iteration: W B_nu(T_R)
  d->macro = m->derived_tables ? 1 : 0;
  d->macro_detailed = macro_detailed && after_iteration ? 1 : 0;
  d->jblue = m->dev.jblue;
  const size_t S = (size_t)p->dev.S;
  d->T_R = m->dev.out_shell + 2 * S;
  d->W = m->dev.out_shell + 3 * S;
  return SMC_OK;
}

}  // namespace

extern "C" {

const char* smc_last_error(void) { return g_err.c_str(); }

int smc_ctx_create(smc_ctx** out, int hip_device) {
  if (!out) return fail(SMC_EINVAL, "null output pointer");
  *out = nullptr;
  int n = 0;
  HIP_TRY(hipGetDeviceCount(&n), "hipGetDeviceCount");
  if (hip_device < 0 || hip_device >= n)
    return fail(SMC_EINVAL, "device %d outside [0, %d)", hip_device, n);
  HIP_TRY(hipSetDevice(hip_device), "hipSetDevice");
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, hip_device), "hipGetDeviceProperties");
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(SMC_EDEVICE, "libsmc is built for gfx950, device %d is %s", hip_device,
                prop.gcnArchName);
  smc_ctx* c = new (std::nothrow) smc_ctx;
  if (!c) return fail(SMC_ENOMEM, "host allocation failed");
  memset(c, 0, sizeof *c);
  c->device = hip_device;
  c->n_cu = prop.multiProcessorCount;
  for (int multi = 0; multi < 2; ++multi) {
    int occ = 0;
    hipError_t e = smc::transport_occupancy(multi != 0, &occ);
    if (e != hipSuccess) {
      release_ctx(c);
      return hip_fail(e, "occupancy query");
    }
    c->transport_blocks_per_cu[multi] = occ > 0 ? occ : 1;
    for (int li = 0; li < 3; ++li) {
      for (int ext = 0; ext < 2; ++ext) {
        e = smc::long_occupancy(multi != 0, 16 << li, ext != 0, &occ);
        if (e != hipSuccess) {
          release_ctx(c);
          return hip_fail(e, "occupancy query");
        }
        c->long_blocks_per_cu[multi][li][ext] = occ > 0 ? occ : 1;
      }
    }
  }
  {
    // the device's copy of the static scratch (host code may not use the
    // array's name as a device address)
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e == hipSuccess) e = hipEventCreate(&c->ev_start);
    if (e == hipSuccess) e = hipEventCreate(&c->ev_stop);
    if (e != hipSuccess) {
      release_ctx(c);
      return hip_fail(e, "scratch lookup");
    }
    c->scratch = static_cast<uint8_t*>(p);
  }
  for (int i = 0; i < kBatchSlots; ++i) {
    const size_t tb = sizeof(smc::BatchEntry) * smc::kMaxBatchModels;
    hipError_t e = hipHostMalloc((void**)&c->host_table[i], tb, hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc((void**)&c->dev_table[i], tb);
    if (e == hipSuccess) e = hipMalloc((void**)&c->dev_ctr[i], kCtlBytes);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->slot_done[i], hipEventDisableTiming);
    if (e != hipSuccess) {
      release_ctx(c);
      return hip_fail(e, "batch table allocation");
    }
  }
  *out = c;
  return ok();
}

int smc_ctx_destroy(smc_ctx* ctx) {
  release_ctx(ctx);
  return ok();
}

int smc_model_workspace_bytes(const smc_model_desc* desc, uint64_t n_packets_max, uint32_t flags,
                              uint64_t* bytes) {
  if (!bytes) return fail(SMC_EINVAL, "null output pointer");
  int rc = validate(desc);
  if (rc) return rc;
  *bytes = layout_of(desc, n_packets_max, flags).total;
  return ok();
}

int smc_model_load(smc_ctx* ctx, const smc_model_desc* d, uint64_t n_packets_max, uint32_t flags,
                   void* d_workspace, uint64_t ws_bytes, void* stream, smc_model** out) {
  if (!ctx || !out) return fail(SMC_EINVAL, "null context or output pointer");
  *out = nullptr;
  if (flags & ~(SMC_F_JBLUE | SMC_F_PACKETS)) return fail(SMC_EINVAL, "unknown flags 0x%x", flags);
  int rc = validate(d);
  if (rc) return rc;
  if (!d_workspace || ((uintptr_t)d_workspace % kAlign) != 0)
    return fail(SMC_EINVAL, "workspace must be a non-null, 256-byte aligned device pointer");
  smc::Layout lay = layout_of(d, n_packets_max, flags);
  if (ws_bytes < lay.total)
    return fail(SMC_ENOMEM, "workspace of %llu bytes is smaller than the %llu needed",
                (unsigned long long)ws_bytes, (unsigned long long)lay.total);
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  if ((rc = check_workspace(d_workspace, ctx->device))) return rc;
  hipStream_t s = (hipStream_t)stream;
  uint8_t* base = (uint8_t*)d_workspace;
  const uint64_t S = (uint64_t)d->n_shells, L = (uint64_t)d->n_lines;

  HIP_TRY(hipMemcpyAsync(base + lay.v_bounds, d->v_bounds, (S + 1) * 8, hipMemcpyHostToDevice, s),
          "upload v_bounds");
  HIP_TRY(hipMemcpyAsync(base + lay.n_e, d->n_e, S * 8, hipMemcpyHostToDevice, s), "upload n_e");
  if (L > 0) {
    // the rows are padded to whole 4-line loads; the copies and the clears
    // of the padding touch disjoint bytes, so no ordering between a fill and
    // a copy engine is relied on
    const uint64_t Lp = (L + 3) / 4 * 4;
    HIP_TRY(hipMemcpyAsync(base + lay.line_nu, d->line_nu, L * 8, hipMemcpyHostToDevice, s),
            "upload line_nu");
    HIP_TRY(copy_rows(base + lay.tau, Lp * 8, d->tau_sobolev, L * 8, L * 8, S,
                      hipMemcpyHostToDevice, s),
            "upload tau_sobolev");
    if (Lp > L) {
      HIP_TRY(hipMemsetAsync(base + lay.line_nu + L * 8, 0, (Lp - L) * 8, s), "pad line_nu");
      HIP_TRY(hipMemset2DAsync(base + lay.tau + L * 8, Lp * 8, 0, (Lp - L) * 8, S, s),
              "pad tau_sobolev");
    }
  }
  const bool derived = derived_macroatom(d) && L > 0;
  if (d->line_mode != SMC_SCATTER && L > 0)
    HIP_TRY(hipMemcpyAsync(base + lay.line_upper, d->line_upper, L * 4, hipMemcpyHostToDevice, s),
            "upload line_upper");
  if (d->line_mode != SMC_SCATTER && L > 0 && !derived) {
    HIP_TRY(hipMemcpyAsync(base + lay.level_ptr, d->level_ptr, ((uint64_t)d->n_levels + 1) * 8,
                           hipMemcpyHostToDevice, s),
            "upload level_ptr");
    HIP_TRY(hipMemcpyAsync(base + lay.em_line, d->em_line, (uint64_t)d->n_em * 4,
                           hipMemcpyHostToDevice, s),
            "upload em_line");
    HIP_TRY(hipMemcpyAsync(base + lay.em_cum, d->em_cum, em_cum_entries(d) * 8,
                           hipMemcpyHostToDevice, s),
            "upload em_cum");
  }

  smc_model* m = new (std::nothrow) smc_model;
  if (!m) return fail(SMC_ENOMEM, "host allocation failed");
  memset(m, 0, sizeof *m);
  m->ctx = ctx;
  m->lay = lay;
  m->base = base;
  m->ws_bytes = ws_bytes;
  m->n_packets_max = n_packets_max;
  m->load_flags = flags;
  smc::DevModel& dm = m->dev;
  dm.S = d->n_shells;
  dm.L = (int32_t)d->n_lines;
  dm.Lp = (int32_t)((d->n_lines + 3) / 4 * 4);
  dm.n_bins = d->n_bins;
  dm.mode = d->line_mode;
  dm.n_em = d->line_mode != SMC_SCATTER ? em_entries(d) : 0;
  m->n_levels = d->line_mode != SMC_SCATTER ? d->n_levels : 0;
  m->derived_tables = derived;
  dm.t_exp = d->t_exp;
  dm.ct = 2.99792458e10 * d->t_exp;
  dm.nu_min = d->nu_min;
  dm.nu_max = d->nu_max;
  dm.seed = d->seed;
  dm.r_bounds = (const double*)(base + lay.r_bounds);
  dm.n_e = (const double*)(base + lay.n_e);
  dm.volume = (const double*)(base + lay.volume);
  dm.line_nu = (const double*)(base + lay.line_nu);
  dm.tau = (const double*)(base + lay.tau);
  if (d->line_mode != SMC_SCATTER) {
    dm.line_upper = (const int32_t*)(base + lay.line_upper);
    dm.level_ptr = (const int64_t*)(base + lay.level_ptr);
    dm.em_line = (const int32_t*)(base + lay.em_line);
    dm.em_cum = (const double*)(base + lay.em_cum);
  }
  dm.raw = (double*)(base + lay.raw);
  dm.lsum = (unsigned long long*)(base + lay.lsum);
  dm.counters = (unsigned long long*)(base + lay.counters);
  dm.jblue = (flags & SMC_F_JBLUE) ? (double*)(base + lay.jblue) : nullptr;
  dm.out_shell = (double*)(base + lay.out_shell);
  dm.out_spec = (double*)(base + lay.out_spec);
  dm.vraw = (double*)(base + lay.vraw);
  dm.vcounts = (unsigned long long*)(base + lay.vcounts);
  dm.out_vspec = (double*)(base + lay.out_vspec);
  dm.scalars = (double*)(base + lay.scalars);
  dm.packets = (flags & SMC_F_PACKETS) ? (void*)(base + lay.packets) : nullptr;
  dm.longs = (smc::LongState*)(base + lay.longs);
  dm.long_order = (uint64_t*)(base + lay.long_order);
  m->order_hist = (unsigned int*)(base + lay.long_hist);
  dm.long_cap = n_packets_max;

  hipError_t e = smc::launch_geometry(dm, (const double*)(base + lay.v_bounds), s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    delete m;
    return hip_fail(e, "model set-up");
  }
  *out = m;
  return ok();
}

int smc_model_free(smc_model* model) {
  if (model) {
    if (model->ev_start) (void)hipEventDestroy(model->ev_start);
    if (model->ev_stop) (void)hipEventDestroy(model->ev_stop);
  }
  delete model;
  return ok();
}

int smc_run_iteration(smc_model* m, const smc_iter_params* p, void* stream) {
  if (!m || !p) return fail(SMC_EINVAL, "null model or parameters");
  smc::LaunchArgs a;
  memset(&a, 0, sizeof a);
  int rc = make_iter(m, p, budget_of(m->tune, m->dev.mode == SMC_MACROATOM, false),
                     &a.single.it);
  if (rc) return rc;
  HIP_TRY(hipSetDevice(m->ctx->device), "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  const bool timed = (p->flags & SMC_F_TIMING) != 0;
  if (timed && !m->ev_start) {
    HIP_TRY(hipEventCreate(&m->ev_start), "hipEventCreate");
    HIP_TRY(hipEventCreate(&m->ev_stop), "hipEventCreate");
  }
  a.single.m = m->dev;
  a.single.work_begin = 0;
  a.single.long_begin = 0;
  a.table = nullptr;
  a.n_models = 1;
  a.total_work = a.single.it.n_work;
  a.ctr = m->dev.counters + smc::CTR_QUEUE;
  a.order_hist = m->order_hist;
  a.max_lines = (uint32_t)m->dev.L;
  const bool ext = a.single.it.n_virtual > 0 || m->dev.mode == SMC_MACROATOM;
  a.hot = hot_of(m->ctx, m->tune, ext, false);
  const smc::Shape sh =
      shape_of(m->ctx, m->tune, false, a.total_work,
               a.single.it.long_budget > 0 || a.single.it.n_virtual > 0, ext);
  HIP_TRY(smc::launch_iteration(a, false, sh, jblue_entries(m, p->flags),
                                timed ? m->ev_start : nullptr, timed ? m->ev_stop : nullptr, s),
          "iteration launch");
  m->timed = timed;
  m->has_T = true;
  m->ran = true;
  m->last_flags = p->flags;
  m->last_work = a.single.it.n_work;
  m->last_virtual = p->n_virtual > 0;
  return ok();
}

}  // extern "C"

namespace {

// One iteration of each model in one set of launches.  The launch-wide
// control block and device model table are `dev_ctr` and `dev_table` when
// given (the static scratch), else the context's next slot; the table is
// staged in that slot's pinned host buffer either way.
int batch_launch(smc_ctx* ctx, smc_model* const* models, const smc_iter_params* params,
                 int n_models, const smc_tune* tune, uint32_t flags, void* stream,
                 smc::BatchEntry* dev_table, unsigned long long* dev_ctr) {
  if (!ctx || !models || !params) return fail(SMC_EINVAL, "null context, models or parameters");
  if (n_models < 1 || n_models > smc::kMaxBatchModels)
    return fail(SMC_EINVAL, "n_models=%d outside [1, %d]", n_models, smc::kMaxBatchModels);
  if (flags & ~SMC_F_TIMING) return fail(SMC_EINVAL, "unknown batch flags 0x%x", flags);
  smc_tune t;
  memset(&t, 0, sizeof t);
  if (tune) t = *tune;
  if (int rc = check_tune(t)) return rc;
  bool any_macro = false;
  for (int k = 0; k < n_models; ++k)
    if (models[k] && models[k]->dev.mode == SMC_MACROATOM) any_macro = true;
  const uint32_t budget = budget_of(t, any_macro, n_models > 1);
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  // a slot whose last launch has finished, searched from the next in turn;
  // with every slot in flight, wait for that next one
  int slot = ctx->next_slot;
  for (int i = 0; i < kBatchSlots; ++i) {
    const int c = (ctx->next_slot + i) % kBatchSlots;
    if (!ctx->slot_used[c]) {
      slot = c;
      break;
    }
    const hipError_t q = hipEventQuery(ctx->slot_done[c]);
    if (q == hipSuccess) {
      slot = c;
      break;
    }
    if (q != hipErrorNotReady) return hip_fail(q, "slot query");
  }
  if (ctx->slot_used[slot]) HIP_TRY(hipEventSynchronize(ctx->slot_done[slot]), "slot wait");
  smc::BatchEntry* tab = ctx->host_table[slot];
  uint64_t work = 0, max_jb = 0;
  uint32_t max_lines = 0;
  bool any_virtual = false, any_ext = false;
  for (int k = 0; k < n_models; ++k) {
    smc_model* m = models[k];
    if (!m) return fail(SMC_EINVAL, "model %d is null", k);
    if (m->ctx != ctx) return fail(SMC_EINVAL, "model %d belongs to another context", k);
    for (int j = 0; j < k; ++j)
      if (models[j] == m) return fail(SMC_EINVAL, "model %d appears twice in the batch", k);
    int rc = make_iter(m, &params[k], budget, &tab[k].it);
    if (rc) {
      char msg[512];
      snprintf(msg, sizeof msg, "model %d: %s", k, g_err.c_str());
      return fail(rc, "%s", msg);
    }
    tab[k].m = m->dev;
    tab[k].work_begin = work;
    tab[k].long_begin = 0;
    work += tab[k].it.n_work;
    if ((uint32_t)m->dev.L > max_lines) max_lines = (uint32_t)m->dev.L;
    if (tab[k].it.n_virtual > 0) any_virtual = true;
    if (tab[k].it.n_virtual > 0 || m->dev.mode == SMC_MACROATOM) any_ext = true;
    const uint64_t jb = jblue_entries(m, params[k].flags);
    if (jb > max_jb) max_jb = jb;
  }
  if (!dev_table) dev_table = ctx->dev_table[slot];
  if (!dev_ctr) dev_ctr = ctx->dev_ctr[slot];
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipMemcpyAsync(dev_table, tab, sizeof(smc::BatchEntry) * n_models,
                         hipMemcpyHostToDevice, s),
          "batch table upload");
  const bool timed = (flags & SMC_F_TIMING) != 0;
  smc::LaunchArgs a;
  memset(&a, 0, sizeof a);
  a.table = dev_table;
  a.n_models = n_models;
  a.total_work = work;
  a.ctr = dev_ctr;
  a.order_hist = (unsigned int*)(dev_ctr + 4);
  a.max_lines = max_lines;
  a.hot = hot_of(ctx, t, any_ext, true);
  const smc::Shape sh = shape_of(ctx, t, true, work, budget > 0 || any_virtual, any_ext);
  HIP_TRY(smc::launch_iteration(a, true, sh, max_jb, timed ? ctx->ev_start : nullptr,
                                timed ? ctx->ev_stop : nullptr, s),
          "batch launch");
  HIP_TRY(hipEventRecord(ctx->slot_done[slot], s), "hipEventRecord");
  ctx->slot_used[slot] = true;
  ctx->next_slot = (slot + 1) % kBatchSlots;
  ctx->batch_timed = timed;
  for (int k = 0; k < n_models; ++k) {
    smc_model* m = models[k];
    m->has_T = true;
    m->ran = true;
    m->timed = false;
    m->last_flags = params[k].flags & ~SMC_F_TIMING;
    m->last_work = tab[k].it.n_work;
    m->last_virtual = params[k].n_virtual > 0;
  }
  return ok();
}

}  // namespace

extern "C" {

int smc_batch_run(smc_ctx* ctx, smc_model* const* models, const smc_iter_params* params,
                  int n_models, const smc_tune* tune, uint32_t flags, void* stream) {
  return batch_launch(ctx, models, params, n_models, tune, flags, stream, nullptr, nullptr);
}

int smc_measure_atomic_rate(double* d_table, uint64_t n_doubles, uint32_t n_rounds, int scattered,
                            int n_cu, void* stream, double* atomics_per_s) {
  if (!d_table || !atomics_per_s) return fail(SMC_EINVAL, "null table or output");
  if (n_doubles < 64 || n_rounds == 0 || n_cu < 1)
    return fail(SMC_EINVAL, "need n_doubles >= 64, n_rounds >= 1, n_cu >= 1");
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t a = nullptr, b = nullptr;
  HIP_TRY(hipEventCreate(&a), "hipEventCreate");
  hipError_t e = hipEventCreate(&b);
  // an untimed launch brings the table into the caches, then the timed one
  if (e == hipSuccess) e = smc::launch_atomic_rate(d_table, n_doubles, n_rounds, scattered, n_cu, s);
  if (e == hipSuccess) e = hipEventRecord(a, s);
  if (e == hipSuccess) e = smc::launch_atomic_rate(d_table, n_doubles, n_rounds, scattered, n_cu, s);
  if (e == hipSuccess) e = hipEventRecord(b, s);
  if (e == hipSuccess) e = hipEventSynchronize(b);
  float ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
  (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  if (e != hipSuccess) return hip_fail(e, "atomic-rate measurement");
  const double n_atomics = 8.0 * n_cu * 256.0 * (double)n_rounds;
  *atomics_per_s = ms > 0.0f ? n_atomics / (ms * 1e-3) : 0.0;
  return ok();
}

int smc_batch_run_static(smc_ctx* ctx, smc_model* const* models, const smc_iter_params* params,
                         int n_models, const smc_tune* tune, uint32_t flags, void* stream) {
  if (!ctx) return fail(SMC_EINVAL, "null context");
  if (n_models > SMC_STATIC_MAX_MODELS)
    return fail(SMC_EINVAL,
                "n_models=%d exceeds the %d models the static scratch holds (use smc_batch_run)",
                n_models, SMC_STATIC_MAX_MODELS);
  // the scratch keeps the last call's contents: the reset kernel clears the
  // queue heads and histogram, and the upload rewrites the table
  return batch_launch(ctx, models, params, n_models, tune, flags, stream,
                      reinterpret_cast<smc::BatchEntry*>(ctx->scratch + kScratchTableOffset),
                      reinterpret_cast<unsigned long long*>(ctx->scratch));
}

int smc_batch_autotune(smc_ctx* ctx, smc_model* const* models, const smc_iter_params* params,
                       int n_models, const smc_tune* candidates, int n_candidates,
                       smc_tune* best, double* best_ms, void* stream) {
  if (!ctx || !models || !params || !best) return fail(SMC_EINVAL, "null argument");
  if (n_models < 1 || n_models > smc::kMaxBatchModels)
    return fail(SMC_EINVAL, "n_models=%d outside [1, %d]", n_models, smc::kMaxBatchModels);
  for (int k = 0; k < n_models; ++k)
    if (!(params[k].T_inner > 0.0))
      return fail(SMC_EINVAL, "autotuning needs T_inner > 0 for every model (model %d)", k);
  // each trial times the whole batch twice and keeps the faster run; a
  // candidate replaces the current choice only when it is at least
  // kTuneMargin faster (iterations of one batch vary by a few per cent)
  constexpr int kTrialRuns = 2;
  constexpr double kTuneMargin = 0.02;
  auto trial = [&](const smc_tune& t, double* ms) -> int {
    double fastest = INFINITY;
    for (int i = 0; i < kTrialRuns; ++i) {
      int rc = smc_batch_run(ctx, models, params, n_models, &t, SMC_F_TIMING, stream);
      if (rc) return rc;
      double run_ms = 0.0;
      rc = smc_batch_read_timing(ctx, &run_ms);
      if (rc) return rc;
      if (run_ms < fastest) fastest = run_ms;
    }
    *ms = fastest;
    return SMC_OK;
  };
  smc_tune cur;
  memset(&cur, 0, sizeof cur);
  double cur_ms = 0.0;
  if (candidates && n_candidates > 0) {
    double bms = INFINITY;
    for (int i = 0; i < n_candidates; ++i) {
      double ms;
      int rc = trial(candidates[i], &ms);
      if (rc) return rc;
      if (ms < bms) {
        bms = ms;
        cur = candidates[i];
      }
    }
    cur_ms = bms;
  } else {
    // coordinate search from the defaults: hand-off budget, lanes per
    // handed-off history, wavefronts per CU of the group-per-packet kernel,
    // then workgroups per CU
    int rc = trial(cur, &cur_ms);
    if (rc) return rc;
    const uint32_t budgets[] = {256, 1024, 4096, UINT32_MAX};
    const uint32_t lanes[] = {16, 32, 64};
    const int32_t waves[] = {4, 8, 16};
    const int32_t blocks[] = {1, 2, 3};
    for (int dim = 0; dim < 4; ++dim) {
      const int n = dim == 0 ? 4 : 3;
      for (int i = 0; i < n; ++i) {
        smc_tune t = cur;
        if (dim == 0) t.long_budget = budgets[i];
        if (dim == 1) t.long_lanes = lanes[i];
        if (dim == 2) t.long_waves_per_cu = waves[i];
        if (dim == 3) t.blocks_per_cu = blocks[i];
        if (dim == 3 && blocks[i] > ctx->transport_blocks_per_cu[1]) continue;
        double ms;
        rc = trial(t, &ms);
        if (rc) return rc;
        if (ms < cur_ms * (1.0 - kTuneMargin)) {
          cur_ms = ms;
          cur = t;
        }
      }
    }
  }
  *best = cur;
  if (best_ms) *best_ms = cur_ms;
  return ok();
}

int smc_batch_read_timing(smc_ctx* ctx, double* transport_ms) {
  if (!ctx || !transport_ms) return fail(SMC_EINVAL, "null context or output");
  if (!ctx->batch_timed) return fail(SMC_EINVAL, "the last batch was not timed");
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  HIP_TRY(hipEventSynchronize(ctx->ev_stop), "hipEventSynchronize");
  float ms = 0.0f;
  HIP_TRY(hipEventElapsedTime(&ms, ctx->ev_start, ctx->ev_stop), "hipEventElapsedTime");
  *transport_ms = (double)ms;
  return ok();
}

int smc_read_estimators(smc_model* m, double* J, double* nubar, double* jblue, double* T_R,
                        double* W, void* stream) {
  if (!m) return fail(SMC_EINVAL, "null model");
  if (!m->ran) return fail(SMC_EINVAL, "no iteration has run");
  if (jblue && !(m->last_flags & SMC_F_JBLUE))
    return fail(SMC_EINVAL, "J_blue was not tallied in the last iteration");
  HIP_TRY(hipSetDevice(m->ctx->device), "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  const size_t S = (size_t)m->dev.S, L = (size_t)m->dev.L;
  int rc;
  if ((rc = sync_copy_out(J, m->dev.out_shell, S * 8, s))) return rc;
  if ((rc = sync_copy_out(nubar, m->dev.out_shell + S, S * 8, s))) return rc;
  if ((rc = sync_copy_out(T_R, m->dev.out_shell + 2 * S, S * 8, s))) return rc;
  if ((rc = sync_copy_out(W, m->dev.out_shell + 3 * S, S * 8, s))) return rc;
  if ((rc = sync_copy_out(jblue, m->dev.jblue, S * L * 8, s))) return rc;
  HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
  return ok();
}

int smc_read_spectrum(smc_model* m, double* L_nu, double* scalars6, void* stream) {
  if (!m) return fail(SMC_EINVAL, "null model");
  if (!m->ran) return fail(SMC_EINVAL, "no iteration has run");
  HIP_TRY(hipSetDevice(m->ctx->device), "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  int rc;
  if ((rc = sync_copy_out(L_nu, m->dev.out_spec, ((size_t)m->dev.n_bins + 2) * 8, s))) return rc;
  if ((rc = sync_copy_out(scalars6, m->dev.scalars, 6 * 8, s))) return rc;
  HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
  return ok();
}

int smc_read_counters(smc_model* m, uint64_t* counters, void* stream) {
  if (!m || !counters) return fail(SMC_EINVAL, "null model or output");
  if (!m->ran) return fail(SMC_EINVAL, "no iteration has run");
  HIP_TRY(hipSetDevice(m->ctx->device), "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  int rc = sync_copy_out(counters, m->dev.counters, SMC_N_COUNTERS * 8, s);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
  return ok();
}

int smc_read_virtual_spectrum(smc_model* m, double* L_nu, double* L_total, uint64_t* counts,
                              void* stream) {
  if (!m || !L_nu || !L_total) return fail(SMC_EINVAL, "null model or output");
  if (!m->ran) return fail(SMC_EINVAL, "no iteration has run");
  if (!m->last_virtual) return fail(SMC_EINVAL, "the last iteration ran no virtual packets");
  HIP_TRY(hipSetDevice(m->ctx->device), "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  const size_t NB = (size_t)m->dev.n_bins + 2;
  int rc;
  if ((rc = sync_copy_out(L_nu, m->dev.out_vspec, NB * 8, s))) return rc;
  if ((rc = sync_copy_out(L_total, m->dev.out_vspec + NB, 8, s))) return rc;
  if (counts && (rc = sync_copy_out(counts, m->dev.vcounts, 3 * 8, s))) return rc;
  HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
  return ok();
}

int smc_read_packets(smc_model* m, smc_packet_out* out, uint64_t n, void* stream) {
  if (!m || !out) return fail(SMC_EINVAL, "null model or output");
  if (!m->ran) return fail(SMC_EINVAL, "no iteration has run");
  if (!(m->last_flags & SMC_F_PACKETS))
    return fail(SMC_EINVAL, "packet records were not written in the last iteration");
  if (n > m->last_work)
    return fail(SMC_EINVAL, "asked for %llu records, the last iteration ran %llu packets",
                (unsigned long long)n, (unsigned long long)m->last_work);
  HIP_TRY(hipSetDevice(m->ctx->device), "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  int rc = sync_copy_out(out, m->dev.packets, n * sizeof(smc_packet_out), s);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
  return ok();
}

int smc_model_set_tune(smc_model* m, const smc_tune* t) {
  if (!m) return fail(SMC_EINVAL, "null model");
  if (!t) {
    memset(&m->tune, 0, sizeof m->tune);
    return ok();
  }
  if (int rc = check_tune(*t)) return rc;
  m->tune = *t;
  return ok();
}

int smc_model_get_tune(smc_model* m, smc_tune* t) {
  if (!m || !t) return fail(SMC_EINVAL, "null model or output");
  *t = m->tune;
  if (t->blocks_per_cu == 0) t->blocks_per_cu = m->ctx->transport_blocks_per_cu[0];
  if (t->long_lanes == 0) t->long_lanes = lanes_of(*t, m->dev.mode == SMC_MACROATOM, false);
  if (t->long_waves_per_cu == 0)
    t->long_waves_per_cu = default_long_waves(m->ctx, false, *t, m->dev.mode == SMC_MACROATOM);
  if (t->long_budget == 0)
    t->long_budget = m->dev.mode == SMC_MACROATOM ? kDefaultLongBudgetWide : kDefaultLongBudget;
  return ok();
}

int smc_read_timing(smc_model* m, double* transport_ms) {
  if (!m || !transport_ms) return fail(SMC_EINVAL, "null model or output");
  if (!m->ran || !m->timed) return fail(SMC_EINVAL, "the last iteration was not timed");
  HIP_TRY(hipSetDevice(m->ctx->device), "hipSetDevice");
  HIP_TRY(hipEventSynchronize(m->ev_stop), "hipEventSynchronize");
  float ms = 0.0f;
  HIP_TRY(hipEventElapsedTime(&ms, m->ev_start, m->ev_stop), "hipEventElapsedTime");
  *transport_ms = (double)ms;
  return ok();
}

struct smc_graph {
  smc_ctx* ctx;
  std::vector<smc_model*> models;
  std::vector<smc_plasma*> plasmas;     // per model, or nullptr: updated after each iteration
  std::vector<smc_iter_params> last;   // parameters of the last iteration, per model
  smc::BatchEntry* host_tables;        // pinned, n_iter * n_models
  smc::BatchEntry* dev_tables;
  unsigned long long* dev_ctr;
  hipGraph_t graph;
  hipGraphExec_t exec;
};

static void release_graph(smc_graph* g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->host_tables) (void)hipHostFree(g->host_tables);
  if (g->dev_tables) (void)hipFree(g->dev_tables);
  if (g->dev_ctr) (void)hipFree(g->dev_ctr);
  delete g;
}

static int graph_capture(smc_ctx* ctx, smc_model* const* models, const smc_iter_params* params,
                         int n_models, int n_iter, const smc_tune* tune,
                         smc_plasma* const* plasmas, const smc_plasma_params* plasma_params,
                         smc_graph** out) {
  if (!ctx || !models || !params || !out) return fail(SMC_EINVAL, "null argument");
  *out = nullptr;
  if (n_models < 1 || n_models > smc::kMaxBatchModels || n_iter < 1 || n_iter > 1000)
    return fail(SMC_EINVAL, "n_models must lie in [1, %d] and n_iter in [1, 1000]",
                smc::kMaxBatchModels);
  smc_tune t;
  memset(&t, 0, sizeof t);
  if (tune)
    t = *tune;
  else if (n_models == 1 && models[0])
    t = models[0]->tune;
  if (int rc = check_tune(t)) return rc;
  bool any_macro = false;
  for (int k = 0; k < n_models; ++k)
    if (models[k] && models[k]->dev.mode == SMC_MACROATOM) any_macro = true;
  const uint32_t budget = budget_of(t, any_macro, n_models > 1);
  for (int k = 0; k < n_models; ++k) {
    if (!models[k] || models[k]->ctx != ctx)
      return fail(SMC_EINVAL, "model %d is null or of another context", k);
    for (int j = 0; j < k; ++j)
      if (models[j] == models[k]) return fail(SMC_EINVAL, "model %d appears twice", k);
    if (!(params[k].T_inner > 0.0) && !models[k]->has_T)
      return fail(SMC_EINVAL, "model %d: the first captured iteration needs T_inner > 0", k);
  }
  // plasma updates after every iteration, from the model's own field
  std::vector<smc::DevPlasma> pdev(plasmas ? n_models : 0);
  for (int k = 0; plasmas && k < n_models; ++k) {
    if (!plasmas[k]) continue;
    if (plasmas[k]->model != models[k])
      return fail(SMC_EINVAL, "plasma %d does not belong to model %d", k, k);
    if (!plasma_params) return fail(SMC_EINVAL, "plasma updates need their parameters");
    if (plasma_params[k].T_R || plasma_params[k].W)
      return fail(SMC_EINVAL, "a captured plasma update takes the model's own field");
    if (int rc = plasma_args(plasmas[k], &plasma_params[k], true, &pdev[k])) return rc;
    if (pdev[k].jb_detailed)
      for (int i = 0; i < n_iter; ++i)
        if (!(params[(size_t)i * n_models + k].flags & SMC_F_JBLUE))
          return fail(SMC_EINVAL, "model %d: detailed J_b needs J_blue in every iteration", k);
  }
  HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  smc_graph* g = new (std::nothrow) smc_graph();
  if (!g) return fail(SMC_ENOMEM, "host allocation failed");
  g->ctx = ctx;
  g->models.assign(models, models + n_models);
  g->plasmas.assign((size_t)n_models, nullptr);
  if (plasmas) g->plasmas.assign(plasmas, plasmas + n_models);
  const size_t n_ent = (size_t)n_iter * (size_t)n_models;
  hipError_t e = hipHostMalloc((void**)&g->host_tables, n_ent * sizeof(smc::BatchEntry),
                               hipHostMallocDefault);
  if (e == hipSuccess) e = hipMalloc((void**)&g->dev_tables, n_ent * sizeof(smc::BatchEntry));
  if (e == hipSuccess) e = hipMalloc((void**)&g->dev_ctr, kCtlBytes);
  if (e != hipSuccess) {
    release_graph(g);
    return hip_fail(e, "graph table allocation");
  }
  std::vector<uint64_t> work(n_iter, 0), max_jb(n_iter, 0);
  std::vector<char> any_virtual(n_iter, 0), any_ext(n_iter, 0);
  uint32_t max_lines = 0;
  for (int k = 0; k < n_models; ++k)
    if ((uint32_t)models[k]->dev.L > max_lines) max_lines = (uint32_t)models[k]->dev.L;
  for (int i = 0; i < n_iter; ++i) {
    for (int k = 0; k < n_models; ++k) {
      smc::BatchEntry& be = g->host_tables[(size_t)i * n_models + k];
      smc_iter_params p = params[(size_t)i * n_models + k];
      p.flags &= ~SMC_F_TIMING;
      // later iterations may take T_inner from the device
      smc_model tmp = *models[k];
      tmp.has_T = true;
      int rc = make_iter(&tmp, &p, budget, &be.it);
      if (rc) {
        release_graph(g);
        return rc;
      }
      be.m = models[k]->dev;
      be.work_begin = work[i];
      be.long_begin = 0;
      work[i] += be.it.n_work;
      if (be.it.n_virtual > 0) any_virtual[i] = 1;
      if (be.it.n_virtual > 0 || models[k]->dev.mode == SMC_MACROATOM) any_ext[i] = 1;
      const uint64_t jb = jblue_entries(models[k], p.flags);
      if (jb > max_jb[i]) max_jb[i] = jb;
      if (i == n_iter - 1) g->last.push_back(p);
    }
  }
  // the device tables are filled before capture; the graph only launches
  e = hipMemcpy(g->dev_tables, g->host_tables, n_ent * sizeof(smc::BatchEntry),
                hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    release_graph(g);
    return hip_fail(e, "graph table upload");
  }
  // record on a private stream (the caller's may be the null stream, which
  // cannot capture); the graph is launched later on the caller's stream
  hipStream_t s = nullptr;
  e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    if (s) (void)hipStreamDestroy(s);
    release_graph(g);
    return hip_fail(e, "hipStreamBeginCapture");
  }
  hipError_t le = hipSuccess;
  for (int i = 0; i < n_iter && le == hipSuccess; ++i) {
    smc::LaunchArgs a;
    memset(&a, 0, sizeof a);
    const bool multi = n_models > 1;
    if (multi) {
      a.table = g->dev_tables + (size_t)i * n_models;
      a.n_models = n_models;
      a.total_work = work[i];
      a.ctr = g->dev_ctr;
      a.order_hist = (unsigned int*)(g->dev_ctr + 4);
    } else {
      a.single = g->host_tables[i];
      a.n_models = 1;
      a.total_work = work[i];
      a.ctr = models[0]->dev.counters + smc::CTR_QUEUE;
      a.order_hist = models[0]->order_hist;
    }
    a.max_lines = max_lines;
    a.hot = hot_of(ctx, t, any_ext[i], multi);
    const smc::Shape sh =
        shape_of(ctx, t, multi, work[i], budget > 0 || any_virtual[i], any_ext[i]);
    le = smc::launch_iteration(a, multi, sh, max_jb[i], nullptr, nullptr, s);
    for (int k = 0; plasmas && k < n_models && le == hipSuccess; ++k)
      if (plasmas[k]) le = smc::launch_plasma_update(pdev[k], s);
  }
  e = hipStreamEndCapture(s, &g->graph);
  (void)hipStreamDestroy(s);
  if (le != hipSuccess || e != hipSuccess) {
    release_graph(g);
    return hip_fail(le != hipSuccess ? le : e, "graph capture");
  }
  e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    release_graph(g);
    return hip_fail(e, "hipGraphInstantiate");
  }
  *out = g;
  return ok();
}

int smc_graph_capture(smc_ctx* ctx, smc_model* const* models, const smc_iter_params* params,
                      int n_models, int n_iter, const smc_tune* tune, void* stream,
                      smc_graph** out) {
  (void)stream;
  return graph_capture(ctx, models, params, n_models, n_iter, tune, nullptr, nullptr, out);
}

int smc_graph_capture_plasma(smc_ctx* ctx, smc_model* const* models,
                             const smc_iter_params* params, int n_models, int n_iter,
                             const smc_tune* tune, smc_plasma* const* plasmas,
                             const smc_plasma_params* plasma_params, void* stream,
                             smc_graph** out) {
  (void)stream;
  if (!plasmas) return fail(SMC_EINVAL, "null plasma array");
  return graph_capture(ctx, models, params, n_models, n_iter, tune, plasmas, plasma_params,
                       out);
}

int smc_graph_launch(smc_graph* g, void* stream) {
  if (!g) return fail(SMC_EINVAL, "null graph");
  HIP_TRY(hipSetDevice(g->ctx->device), "hipSetDevice");
  HIP_TRY(hipGraphLaunch(g->exec, (hipStream_t)stream), "hipGraphLaunch");
  for (size_t k = 0; k < g->models.size(); ++k) {
    smc_model* m = g->models[k];
    m->has_T = true;
    m->ran = true;
    m->timed = false;
    m->last_flags = g->last[k].flags;
    m->last_work = g->last[k].packet_ids ? g->last[k].n_ids : g->last[k].n_packets;
    m->last_virtual = g->last[k].n_virtual > 0;
    if (g->plasmas[k]) g->plasmas[k]->updated = true;
  }
  return ok();
}

int smc_graph_destroy(smc_graph* g) {
  if (g) {
    HIP_TRY(hipSetDevice(g->ctx->device), "hipSetDevice");
    HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");  // no replay in flight
  }
  release_graph(g);
  return ok();
}

}  // extern "C"

// ---------------------------------------------------------------------------
// plasma state and Sobolev depths
// ---------------------------------------------------------------------------

namespace {

int validate_plasma(const smc_plasma_desc* d, int32_t S, int64_t L) {
  if (!d) return fail(SMC_EINVAL, "null plasma description");
  if (S < 1 || S > kMaxShells) return fail(SMC_EINVAL, "n_shells=%d outside [1, %d]", S, kMaxShells);
  if (L < 0 || L > INT32_MAX) return fail(SMC_EINVAL, "n_lines=%lld outside [0, 2^31)", (long long)L);
  const int32_t E = d->n_elements, NI = d->n_ions, NL = d->n_levels;
  if (E < 1 || E > smc::kPlasmaMaxElements)
    return fail(SMC_EINVAL, "n_elements=%d outside [1, %d]", E, smc::kPlasmaMaxElements);
  if (NI < E || NI > smc::kPlasmaMaxIons)
    return fail(SMC_EINVAL, "n_ions=%d outside [n_elements, %d]", NI, smc::kPlasmaMaxIons);
  if (NL < NI) return fail(SMC_EINVAL, "n_levels=%d below n_ions=%d", NL, NI);
  if (!d->element_ion_ptr || !d->ion_chi || !d->ion_zeta || !d->ion_level_ptr ||
      !d->level_energy || !d->level_g || !d->level_metastable || !d->number_density)
    return fail(SMC_EINVAL, "null atomic-data or density array");
  if (L > 0 && (!d->line_lower || !d->line_upper || !d->line_f))
    return fail(SMC_EINVAL, "null line arrays");
  if (d->element_ion_ptr[0] != 0 || d->element_ion_ptr[E] != NI)
    return fail(SMC_EINVAL, "element_ion_ptr must run from 0 to n_ions");
  for (int32_t e = 0; e < E; ++e)
    if (!(d->element_ion_ptr[e + 1] > d->element_ion_ptr[e]))
      return fail(SMC_EINVAL, "element %d has no ion stage", e);
  if (d->ion_level_ptr[0] != 0 || d->ion_level_ptr[NI] != NL)
    return fail(SMC_EINVAL, "ion_level_ptr must run from 0 to n_levels");
  for (int32_t i = 0; i < NI; ++i) {
    if (!(d->ion_level_ptr[i + 1] > d->ion_level_ptr[i]))
      return fail(SMC_EINVAL, "ion %d has no level", i);
    const int32_t g0 = d->ion_level_ptr[i];
    if (d->level_energy[g0] != 0.0 || !d->level_metastable[g0])
      return fail(SMC_EINVAL, "the first level of ion %d must be a metastable ground state "
                  "(energy 0)", i);
    if (!(d->ion_zeta[i] >= 0.0 && d->ion_zeta[i] <= 1.0))
      return fail(SMC_EINVAL, "ion_zeta[%d] must lie in [0, 1]", i);
  }
  for (int32_t e = 0; e < E; ++e)
    for (int32_t i = d->element_ion_ptr[e]; i < d->element_ion_ptr[e + 1] - 1; ++i)
      if (!(d->ion_chi[i] > 0.0) || !isfinite(d->ion_chi[i]))
        return fail(SMC_EINVAL, "ion_chi[%d] must be finite and > 0", i);
  for (int32_t l = 0; l < NL; ++l) {
    if (!(d->level_energy[l] >= 0.0) || !isfinite(d->level_energy[l]))
      return fail(SMC_EINVAL, "level_energy[%d] must be finite and >= 0", l);
    if (!(d->level_g[l] > 0.0) || !isfinite(d->level_g[l]))
      return fail(SMC_EINVAL, "level_g[%d] must be finite and > 0", l);
  }
  for (int64_t k = 0; k < L; ++k) {
    const int32_t lo = d->line_lower[k], up = d->line_upper[k];
    if (lo < 0 || lo >= NL || up < 0 || up >= NL)
      return fail(SMC_EINVAL, "line %lld: level index out of range", (long long)k);
    // same ion: the ion whose level range holds lo also holds up
    const int32_t* it = std::upper_bound(d->ion_level_ptr, d->ion_level_ptr + NI + 1, lo);
    const int32_t ion = (int32_t)(it - d->ion_level_ptr) - 1;
    if (up < d->ion_level_ptr[ion] || up >= d->ion_level_ptr[ion + 1])
      return fail(SMC_EINVAL, "line %lld joins levels of different ions", (long long)k);
    if (!(d->level_energy[up] > d->level_energy[lo]))
      return fail(SMC_EINVAL, "line %lld: upper level must lie above the lower", (long long)k);
    if (!(d->line_f[k] >= 0.0) || !isfinite(d->line_f[k]))
      return fail(SMC_EINVAL, "line_f[%lld] must be finite and >= 0", (long long)k);
  }
  const int64_t n_dens = (int64_t)S * E;
  for (int64_t j = 0; j < n_dens; ++j)
    if (!(d->number_density[j] >= 0.0) || !isfinite(d->number_density[j]))
      return fail(SMC_EINVAL, "number_density[%lld] must be finite and >= 0", (long long)j);
  // NLTE ions: distinct, small enough for the LDS system, every level joined
  // to the ground state by the ion's lines
  const int32_t NN = d->n_nlte_ions;
  if (NN < 0 || NN > smc::kNlteMaxIons || NN > NI)
    return fail(SMC_EINVAL, "n_nlte_ions=%d outside [0, min(n_ions, %d)]", NN, smc::kNlteMaxIons);
  if (NN > 0 && (!d->nlte_ions || (L > 0 && !d->line_upsilon)))
    return fail(SMC_EINVAL, "NLTE ions need nlte_ions and line_upsilon");
  for (int32_t j = 0; j < NN; ++j) {
    const int32_t ion = d->nlte_ions[j];
    if (ion < 0 || ion >= NI) return fail(SMC_EINVAL, "nlte_ions[%d]=%d out of range", j, ion);
    for (int32_t q = 0; q < j; ++q)
      if (d->nlte_ions[q] == ion) return fail(SMC_EINVAL, "NLTE ion %d listed twice", ion);
    const int32_t l0 = d->ion_level_ptr[ion], n = d->ion_level_ptr[ion + 1] - l0;
    if (n > smc::kNlteMaxLevels)
      return fail(SMC_EINVAL, "NLTE ion %d has %d levels (at most %d)", ion, n,
                  smc::kNlteMaxLevels);
    std::vector<int32_t> root(n);
    for (int32_t v = 0; v < n; ++v) root[v] = v;
    auto find = [&](int32_t v) {
      while (root[v] != v) v = root[v] = root[root[v]];
      return v;
    };
    for (int64_t k = 0; k < L; ++k) {
      const int32_t lo = d->line_lower[k] - l0, up = d->line_upper[k] - l0;
      if (lo < 0 || lo >= n) continue;
      if (!(d->line_upsilon[k] >= 0.0) || !isfinite(d->line_upsilon[k]))
        return fail(SMC_EINVAL, "line_upsilon[%lld] must be finite and >= 0", (long long)k);
      root[find(lo)] = find(up);
    }
    for (int32_t v = 1; v < n; ++v)
      if (find(v) != find(0))
        return fail(SMC_EINVAL, "level %d of NLTE ion %d is not joined to its ground state by "
                    "lines", v, ion);
    int64_t count = 0;
    for (int64_t k = 0; k < L; ++k)
      count += d->line_lower[k] >= l0 && d->line_lower[k] < l0 + n;
    if (count > smc::kNlteMaxLines)
      return fail(SMC_EINVAL, "NLTE ion %d has %lld lines (at most %d)", ion, (long long)count,
                  smc::kNlteMaxLines);
  }
  return SMC_OK;
}

// lines of each NLTE ion (the lines whose lower level is in the ion), in
// line order
std::vector<int64_t> nlte_line_offsets(const smc_plasma_desc* d, int64_t L,
                                       std::vector<smc::NlteLine>* recs) {
  std::vector<int64_t> ptr(1, 0);
  for (int32_t j = 0; j < d->n_nlte_ions; ++j) {
    const int32_t ion = d->nlte_ions[j];
    const int32_t l0 = d->ion_level_ptr[ion], l1 = d->ion_level_ptr[ion + 1];
    int64_t count = 0;
    for (int64_t k = 0; k < L; ++k) {
      if (d->line_lower[k] < l0 || d->line_lower[k] >= l1) continue;
      ++count;
      if (recs) {
        smc::NlteLine r;
        memset(&r, 0, sizeof r);
        r.line = (int32_t)k;
        r.lo = (int16_t)(d->line_lower[k] - l0);
        r.up = (int16_t)(d->line_upper[k] - l0);
        recs->push_back(r);
      }
    }
    ptr.push_back(ptr.back() + count);
  }
  return ptr;
}

smc::PlasmaLayout plasma_layout_of(const smc_plasma_desc* d, int32_t S, int64_t L) {
  smc::PlasmaLayout l;
  memset(&l, 0, sizeof l);
  const uint64_t E = (uint64_t)d->n_elements, NI = (uint64_t)d->n_ions;
  const uint64_t NL = (uint64_t)d->n_levels, SS = (uint64_t)S, LL = (uint64_t)L;
  uint64_t off = 0;
  auto take = [&](uint64_t bytes) {
    const uint64_t o = off;
    off = align_up(off + (bytes ? bytes : 1));
    return o;
  };
  l.elem_ion_ptr = take((E + 1) * 4);
  l.ion_chi = take(NI * 8);
  l.ion_zeta = take(NI * 8);
  l.ion_level_ptr = take((NI + 1) * 4);
  l.level_energy = take(NL * 8);
  l.level_g = take(NL * 8);
  l.level_meta = take(NL);
  l.level_ion = take(NL * 4);
  l.line_f = take(LL * 8);
  l.lines = take(LL * sizeof(smc::PlasmaLine));
  l.density = take(SS * E * 8);
  l.field = take(2 * SS * 8);
  l.partition = take(SS * NI * 8);
  l.ion_density = take(SS * NI * 8);
  l.level_pop = take(SS * NL * 8);
  l.level_x = take(SS * NL * 8);
  l.clamped = take(2 * 8);
  const uint64_t NN = (uint64_t)d->n_nlte_ions;
  const uint64_t n_nlte_lines = NN ? (uint64_t)nlte_line_offsets(d, L, nullptr).back() : 0;
  l.nlte_ions = take(NN * 4);
  l.nlte_line_ptr = take((NN + 1) * 4);
  l.nlte_lines = take(n_nlte_lines * sizeof(smc::NlteLine));
  l.nlte_lev_ptr = take(NN * (smc::kNlteMaxLevels + 1) * 4);
  l.nlte_ent = take(2 * n_nlte_lines * 4);
  l.line_upsilon = take(NN ? LL * 8 : 0);
  l.macro_lines = take(LL * sizeof(smc::MacroLine));
  l.em_via = take(3 * LL * 4);
  l.em_kind = take(3 * LL);
  l.total = off;
  return l;
}

int h2d(uint8_t* base, uint64_t off, const void* src, size_t bytes, hipStream_t s,
        const char* what) {
  if (bytes == 0) return SMC_OK;
  HIP_TRY(hipMemcpyAsync(base + off, src, bytes, hipMemcpyHostToDevice, s), what);
  return SMC_OK;
}

}  // namespace

extern "C" {

int smc_plasma_workspace_bytes(const smc_plasma_desc* desc, int32_t n_shells, int64_t n_lines,
                               uint64_t* bytes) {
  if (!bytes) return fail(SMC_EINVAL, "null output pointer");
  int rc = validate_plasma(desc, n_shells, n_lines);
  if (rc) return rc;
  *bytes = plasma_layout_of(desc, n_shells, n_lines).total;
  return ok();
}

int smc_plasma_load(smc_model* model, const smc_plasma_desc* d, void* d_workspace,
                    uint64_t ws_bytes, void* stream, smc_plasma** out) {
  if (!model || !out) return fail(SMC_EINVAL, "null model or output pointer");
  *out = nullptr;
  const int32_t S = model->dev.S;
  const int64_t L = model->dev.L;
  int rc = validate_plasma(d, S, L);
  if (rc) return rc;
  if (!d_workspace || ((uintptr_t)d_workspace % kAlign) != 0)
    return fail(SMC_EINVAL, "workspace must be a non-null, 256-byte aligned device pointer");
  const smc::PlasmaLayout lay = plasma_layout_of(d, S, L);
  if (ws_bytes < lay.total)
    return fail(SMC_ENOMEM, "workspace of %llu bytes is smaller than the %llu needed",
                (unsigned long long)ws_bytes, (unsigned long long)lay.total);
  HIP_TRY(hipSetDevice(model->ctx->device), "hipSetDevice");
  if ((rc = check_workspace(d_workspace, model->ctx->device))) return rc;
  hipStream_t s = (hipStream_t)stream;
  uint8_t* base = (uint8_t*)d_workspace;
  const size_t E = (size_t)d->n_elements, NI = (size_t)d->n_ions, NL = (size_t)d->n_levels;

  // A macroatom model loaded without tables: its rows follow this atom's
  // lines.  Row i holds the lines with upper level i as deactivations (line
  // order), the same lines as internal jumps down, then the lines with lower
  // level i as internal jumps up; em_line is the line of a deactivation and
  // -(j+1) for a jump to level j.
  std::vector<int64_t> ma_ptr;
  std::vector<int32_t> ma_line, ma_via;
  std::vector<uint8_t> ma_kind;
  if (model->derived_tables) {
    if (model->n_levels != d->n_levels)
      return fail(SMC_EINVAL, "the model has %d macro-atom levels, the atom %d", model->n_levels,
                  d->n_levels);
    std::vector<int32_t> up((size_t)L);
    HIP_TRY(hipMemcpyAsync(up.data(), model->base + model->lay.line_upper, (size_t)L * 4,
                           hipMemcpyDeviceToHost, s),
            "read line_upper");
    HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
    for (int64_t k = 0; k < L; ++k)
      if (up[(size_t)k] != d->line_upper[k])
        return fail(SMC_EINVAL, "the model's line_upper[%lld] = %d is not the atom's %d",
                    (long long)k, up[(size_t)k], d->line_upper[k]);
    std::vector<int64_t> n_down(NL, 0), n_up(NL, 0);
    for (int64_t k = 0; k < L; ++k) {
      ++n_down[(size_t)d->line_upper[k]];
      ++n_up[(size_t)d->line_lower[k]];
    }
    ma_ptr.assign(NL + 1, 0);
    for (size_t i = 0; i < NL; ++i) ma_ptr[i + 1] = ma_ptr[i] + 2 * n_down[i] + n_up[i];
    std::vector<int64_t> c_emit(NL), c_down(NL), c_up(NL);
    for (size_t i = 0; i < NL; ++i) {
      c_emit[i] = ma_ptr[i];
      c_down[i] = ma_ptr[i] + n_down[i];
      c_up[i] = ma_ptr[i] + 2 * n_down[i];
    }
    ma_line.resize((size_t)(3 * L));
    ma_via.resize((size_t)(3 * L));
    ma_kind.resize((size_t)(3 * L));
    for (int64_t k = 0; k < L; ++k) {
      const int32_t lo = d->line_lower[k], hi = d->line_upper[k];
      const size_t je = (size_t)c_emit[(size_t)hi]++, jd = (size_t)c_down[(size_t)hi]++;
      const size_t ju = (size_t)c_up[(size_t)lo]++;
      ma_line[je] = (int32_t)k;
      ma_via[je] = (int32_t)k;
      ma_kind[je] = smc::kMacroEmit;
      ma_line[jd] = -(lo + 1);
      ma_via[jd] = (int32_t)k;
      ma_kind[jd] = smc::kMacroDown;
      ma_line[ju] = -(hi + 1);
      ma_via[ju] = (int32_t)k;
      ma_kind[ju] = smc::kMacroUp;
    }
    if ((rc = h2d(model->base, model->lay.level_ptr, ma_ptr.data(), (NL + 1) * 8, s,
                  "upload level_ptr")) ||
        (rc = h2d(model->base, model->lay.em_line, ma_line.data(), ma_line.size() * 4, s,
                  "upload em_line")) ||
        (rc = h2d(base, lay.em_via, ma_via.data(), ma_via.size() * 4, s, "upload em_via")) ||
        (rc = h2d(base, lay.em_kind, ma_kind.data(), ma_kind.size(), s, "upload em_kind")))
      return rc;
  }

  // host-side index tables: the ion of every level, and the per-line
  // record (level indices; the coefficient is set on the device)
  std::vector<int32_t> level_ion(NL);
  for (size_t i = 0; i < NI; ++i)
    for (int32_t l = d->ion_level_ptr[i]; l < d->ion_level_ptr[i + 1]; ++l)
      level_ion[(size_t)l] = (int32_t)i;
  std::vector<smc::PlasmaLine> lines((size_t)L);
  for (int64_t k = 0; k < L; ++k) {
    smc::PlasmaLine& r = lines[(size_t)k];
    r.coef_g = 0.0;
    r.lower = d->line_lower[k];
    r.upper = d->line_upper[k];
  }
  if ((rc = h2d(base, lay.elem_ion_ptr, d->element_ion_ptr, (E + 1) * 4, s, "upload ions")) ||
      (rc = h2d(base, lay.ion_chi, d->ion_chi, NI * 8, s, "upload ion_chi")) ||
      (rc = h2d(base, lay.ion_zeta, d->ion_zeta, NI * 8, s, "upload ion_zeta")) ||
      (rc = h2d(base, lay.ion_level_ptr, d->ion_level_ptr, (NI + 1) * 4, s, "upload levels")) ||
      (rc = h2d(base, lay.level_energy, d->level_energy, NL * 8, s, "upload level_energy")) ||
      (rc = h2d(base, lay.level_g, d->level_g, NL * 8, s, "upload level_g")) ||
      (rc = h2d(base, lay.level_meta, d->level_metastable, NL, s, "upload metastable")) ||
      (rc = h2d(base, lay.level_ion, level_ion.data(), NL * 4, s, "upload level_ion")) ||
      (rc = h2d(base, lay.line_f, d->line_f, (size_t)L * 8, s, "upload line_f")) ||
      (rc = h2d(base, lay.lines, lines.data(), (size_t)L * sizeof(smc::PlasmaLine), s,
                "upload lines")) ||
      (rc = h2d(base, lay.density, d->number_density, (size_t)S * E * 8, s, "upload density")))
    return rc;
  const int32_t NN = d->n_nlte_ions;
  std::vector<smc::NlteLine> nlte_recs;
  std::vector<int32_t> nlte_ptr32, lev_ptr, ent;
  if (NN > 0) {
    const std::vector<int64_t> ptr = nlte_line_offsets(d, L, &nlte_recs);
    nlte_ptr32.assign(ptr.begin(), ptr.end());
    // per level of each NLTE ion, its lines in line order: the assembly of
    // row r visits only these
    const int32_t LP = smc::kNlteMaxLevels + 1;
    lev_ptr.assign((size_t)NN * LP, 0);
    ent.resize(2 * nlte_recs.size());
    for (int32_t j = 0; j < NN; ++j) {
      const int32_t ion = d->nlte_ions[j];
      const int32_t n = d->ion_level_ptr[ion + 1] - d->ion_level_ptr[ion];
      int32_t* lp = &lev_ptr[(size_t)j * LP];
      for (int64_t e = ptr[j]; e < ptr[j + 1]; ++e) {
        ++lp[nlte_recs[e].lo + 1];
        ++lp[nlte_recs[e].up + 1];
      }
      for (int32_t r = 0; r < n; ++r) lp[r + 1] += lp[r];
      for (int32_t r = n + 1; r < LP; ++r) lp[r] = lp[n];
      std::vector<int32_t> fill(lp, lp + n);
      int32_t* out = &ent[2 * (size_t)ptr[j]];
      for (int64_t e = ptr[j]; e < ptr[j + 1]; ++e) {
        const int32_t pos = (int32_t)(e - ptr[j]);
        const smc::NlteLine& r = nlte_recs[e];
        out[fill[r.lo]++] = (pos << 16) | (r.up << 1) | 1;
        out[fill[r.up]++] = (pos << 16) | (r.lo << 1);
      }
    }
    if ((rc = h2d(base, lay.nlte_ions, d->nlte_ions, (size_t)NN * 4, s, "upload nlte_ions")) ||
        (rc = h2d(base, lay.nlte_line_ptr, nlte_ptr32.data(), (size_t)(NN + 1) * 4, s,
                  "upload NLTE line offsets")) ||
        (rc = h2d(base, lay.nlte_lines, nlte_recs.data(),
                  nlte_recs.size() * sizeof(smc::NlteLine), s, "upload NLTE lines")) ||
        (rc = h2d(base, lay.nlte_lev_ptr, lev_ptr.data(), lev_ptr.size() * 4, s,
                  "upload NLTE level offsets")) ||
        (rc = h2d(base, lay.nlte_ent, ent.data(), ent.size() * 4, s, "upload NLTE entries")) ||
        (rc = h2d(base, lay.line_upsilon, d->line_upsilon, (size_t)L * 8, s,
                  "upload line_upsilon")))
      return rc;
  }

  smc_plasma* p = new (std::nothrow) smc_plasma;
  if (!p) return fail(SMC_ENOMEM, "host allocation failed");
  memset(p, 0, sizeof *p);
  p->model = model;
  p->lay = lay;
  p->base = base;
  smc::DevPlasma& dp = p->dev;
  dp.S = S;
  dp.E = d->n_elements;
  dp.n_ions = d->n_ions;
  dp.n_levels = d->n_levels;
  dp.L = (int32_t)L;
  dp.Lp = model->dev.Lp;
  dp.t_exp = model->dev.t_exp;
  dp.elem_ion_ptr = (const int32_t*)(base + lay.elem_ion_ptr);
  dp.ion_chi = (const double*)(base + lay.ion_chi);
  dp.ion_zeta = (const double*)(base + lay.ion_zeta);
  dp.ion_level_ptr = (const int32_t*)(base + lay.ion_level_ptr);
  dp.level_energy = (const double*)(base + lay.level_energy);
  dp.level_g = (const double*)(base + lay.level_g);
  dp.level_meta = (const uint8_t*)(base + lay.level_meta);
  dp.level_ion = (const int32_t*)(base + lay.level_ion);
  dp.line_f = (const double*)(base + lay.line_f);
  dp.lines = (smc::PlasmaLine*)(base + lay.lines);
  dp.density = (const double*)(base + lay.density);
  dp.partition = (double*)(base + lay.partition);
  dp.ion_density = (double*)(base + lay.ion_density);
  dp.level_pop = (double*)(base + lay.level_pop);
  dp.level_x = (double*)(base + lay.level_x);
  dp.clamped = (unsigned long long*)(base + lay.clamped);
  dp.n_e = const_cast<double*>(model->dev.n_e);
  dp.tau = const_cast<double*>(model->dev.tau);
  dp.line_nu = model->dev.line_nu;
  p->n_nlte = NN;
  dp.n_nlte = 0;  // set per update
  dp.nlte_ions = (const int32_t*)(base + lay.nlte_ions);
  dp.nlte_line_ptr = (const int32_t*)(base + lay.nlte_line_ptr);
  dp.nlte_lines = (smc::NlteLine*)(base + lay.nlte_lines);
  dp.nlte_lev_ptr = (const int32_t*)(base + lay.nlte_lev_ptr);
  dp.nlte_ent = (const int32_t*)(base + lay.nlte_ent);
  dp.line_upsilon = (const double*)(base + lay.line_upsilon);
  dp.macro = 0;  // set per update
  dp.macro_detailed = 0;
  dp.macro_lines = (smc::MacroLine*)(base + lay.macro_lines);
  dp.em_via = (const int32_t*)(base + lay.em_via);
  dp.em_kind = (const uint8_t*)(base + lay.em_kind);
  dp.n_em = model->dev.n_em;
  dp.level_ptr = model->dev.level_ptr;
  dp.em_cum = const_cast<double*>(model->dev.em_cum);
  // the host staging vectors must stay alive until the copies have run
  hipError_t e = smc::launch_plasma_lines(dp, (int)nlte_recs.size(), s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    delete p;
    return hip_fail(e, "plasma set-up");
  }
  *out = p;
  return ok();
}

int smc_plasma_update(smc_plasma* p, const smc_plasma_params* pp, void* stream) {
  if (!p || !pp) return fail(SMC_EINVAL, "null plasma or parameters");
  const smc_model* m = p->model;
  smc::DevPlasma d;
  int rc = plasma_args(p, pp, m->ran, &d);
  if (rc) return rc;
  if ((d.jb_detailed || d.macro_detailed) && !(m->last_flags & SMC_F_JBLUE))
    return fail(SMC_EINVAL, "the model's last iteration did not tally J_blue");
  const int32_t S = p->dev.S;
  if (pp->T_R) {
    for (int32_t i = 0; i < S; ++i) {
      if (!(pp->T_R[i] > 0.0) || !isfinite(pp->T_R[i]))
        return fail(SMC_EINVAL, "T_R[%d] must be finite and > 0", i);
      if (!(pp->W[i] > 0.0) || !isfinite(pp->W[i]))
        return fail(SMC_EINVAL, "W[%d] must be finite and > 0", i);
    }
  }
  HIP_TRY(hipSetDevice(m->ctx->device), "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  if (pp->T_R) {
    double* field = (double*)(p->base + p->lay.field);
    HIP_TRY(hipMemcpyAsync(field, pp->T_R, (size_t)S * 8, hipMemcpyHostToDevice, s),
            "upload T_R");
    HIP_TRY(hipMemcpyAsync(field + S, pp->W, (size_t)S * 8, hipMemcpyHostToDevice, s),
            "upload W");
    HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
    d.T_R = field;
    d.W = field + S;
  }
  HIP_TRY(smc::launch_plasma_update(d, s), "plasma update");
  p->updated = true;
  if (p->model->derived_tables) p->model->tables_ready = true;
  return ok();
}

int smc_plasma_read(smc_plasma* p, double* n_e, double* ion_density, double* partition,
                    double* level_pop, double* tau_sobolev, uint64_t* counts, void* stream) {
  if (!p) return fail(SMC_EINVAL, "null plasma");
  if (!p->updated) return fail(SMC_EINVAL, "the plasma has not been updated");
  HIP_TRY(hipSetDevice(p->model->ctx->device), "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  const smc::DevPlasma& d = p->dev;
  const size_t S = (size_t)d.S, NI = (size_t)d.n_ions, NL = (size_t)d.n_levels;
  const size_t L = (size_t)d.L;
  int rc;
  if ((rc = sync_copy_out(n_e, d.n_e, S * 8, s))) return rc;
  if ((rc = sync_copy_out(ion_density, d.ion_density, S * NI * 8, s))) return rc;
  if ((rc = sync_copy_out(partition, d.partition, S * NI * 8, s))) return rc;
  if ((rc = sync_copy_out(level_pop, d.level_pop, S * NL * 8, s))) return rc;
  if ((rc = sync_copy_out(counts, d.clamped, 2 * 8, s))) return rc;
  if (tau_sobolev && L > 0)
    HIP_TRY(copy_rows(tau_sobolev, L * 8, d.tau, (size_t)d.Lp * 8, L * 8, S,
                      hipMemcpyDeviceToHost, s),
            "read tau_sobolev");
  HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
  return ok();
}

int smc_model_read_macroatom(smc_model* m, int64_t* level_ptr, int32_t* em_line, double* em_cum,
                             void* stream) {
  if (!m) return fail(SMC_EINVAL, "null model");
  if (m->dev.mode == SMC_SCATTER || m->dev.L == 0)
    return fail(SMC_EINVAL, "the model has no macro-atom tables");
  if (m->derived_tables && !m->tables_ready)
    return fail(SMC_EINVAL, "the model's tables have not been derived yet");
  HIP_TRY(hipSetDevice(m->ctx->device), "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  const size_t n_em = (size_t)m->dev.n_em;
  const size_t n_cum = m->dev.mode == SMC_MACROATOM ? (size_t)m->dev.S * n_em : n_em;
  int rc;
  if ((rc = sync_copy_out(level_ptr, m->dev.level_ptr, ((size_t)m->n_levels + 1) * 8, s)))
    return rc;
  if ((rc = sync_copy_out(em_line, m->dev.em_line, n_em * 4, s))) return rc;
  if ((rc = sync_copy_out(em_cum, m->dev.em_cum, n_cum * 8, s))) return rc;
  HIP_TRY(hipStreamSynchronize(s), "hipStreamSynchronize");
  return ok();
}

int smc_plasma_free(smc_plasma* p) {
  delete p;
  return ok();
}

}  // extern "C"
