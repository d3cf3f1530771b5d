// smc_internal.h -- device-side model layout shared by the kernels and the
// host runtime of libsmc (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smc {

// Byte layout of one model inside the caller's workspace; every region is
// 256-byte aligned.  Offsets are relative to the workspace base.
struct Layout {
  uint64_t r_bounds, n_e, volume, v_bounds;        // shells
  uint64_t line_nu, tau;                            // lines (rows padded to 4)
  uint64_t line_upper, level_ptr, em_line, em_cum;  // downbranch tables
  uint64_t raw;        // [2S + NB + 2] J_raw, nubar_raw, spectrum raw
  uint64_t lsum;       // [4] u64 escaped, reabsorbed, capped lab energy in units of 2^-60 (+ pad)
  uint64_t counters;   // [CTR_TOTAL] u64: event counters, work-queue head,
                       // hand-off count, hand-off queue head
  uint64_t longs;      // [n_packets_max] LongState: histories handed to the group kernel
  uint64_t long_order; // [n_packets_max] u64: hand-off indices in processing order
  uint64_t long_hist;  // [2 * kOrderBuckets] u32: bucket counts, then bucket cursors
  uint64_t jblue;      // [S*L] raw, normalised in place by the finaliser
  uint64_t out_shell;  // [6S] J, nubar, T_R, W, jblue scale, pad
  uint64_t out_spec;   // [NB + 2] L_nu
  uint64_t vraw;       // [NB + 2] v-packet lab energy * exp(-tau_v) per bin
  uint64_t vcounts;    // [4] u64 v-packets launched, counted, resonances swept (+ pad)
  uint64_t out_vspec;  // [NB + 3] v-packet L_nu, then the summed luminosity
  uint64_t scalars;    // [8] L_emitted, L_reabsorbed, L_capped, L_inner, T_used, T_next, ...
  uint64_t packets;    // [n_packets_max] smc_packet_out
  uint64_t total;
};

// State of a packet handed from the lane-per-packet kernel to the
// group-per-packet kernel after `long_budget` flight segments (128 bytes).
struct LongState {
  uint64_t slot, pid;
  double r, mu, nu, E, mu0, nu_cmf0;
  uint64_t n_seg, n_pass, hash, draw;
  int32_t shell, next_line, last_line;
  uint32_t n_esc, n_line, pad;
};

// v-packets whose optical depth exceeds this are not counted
constexpr double kTauVirtualMax = 30.0;
constexpr uint32_t kMaxVirtual = 16;
// a macro atom making this many internal jumps without deactivating ends its
// packet as CAPPED
constexpr uint32_t kMacroMaxSteps = 100000;

// Luminosity sums are kept in fixed point (energy x 2^60 rounded to an
// integer), so that their totals, and the T_inner update that follows from
// them, do not depend on the order in which packets end.
constexpr double kLScale = 0x1p60;

// The group kernel takes handed-off histories in order of a predicted
// length (lines to the red times distance from the inner boundary, larger
// first), sorted by counting into this many buckets.
constexpr int kOrderBuckets = 1024;

// counters[] slots after the SMC_N_COUNTERS event counters
enum { CTR_QUEUE = SMC_N_COUNTERS, CTR_LONG_COUNT = SMC_N_COUNTERS + 1,
       CTR_LONG_QUEUE = SMC_N_COUNTERS + 2, CTR_TOTAL = SMC_N_COUNTERS + 3 };

// Everything a kernel needs about one model.
struct DevModel {
  int32_t S;
  int32_t L;
  int32_t Lp;              // tau_S row stride (L rounded up to a multiple of 4)
  int32_t n_bins;
  int32_t mode;
  int32_t pad;
  double t_exp;
  double ct;
  double nu_min, nu_max;
  uint64_t seed;
  int64_t n_em;            // macro-atom table entries per probability set
  const double* r_bounds;  // [S+1] radii
  const double* n_e;       // [S]
  const double* volume;    // [S]
  const double* line_nu;   // [Lp]
  const double* tau;       // [S*Lp]
  const int32_t* line_upper;
  const int64_t* level_ptr;
  const int32_t* em_line;
  const double* em_cum;
  double* raw;             // J_raw[S], nubar_raw[S], spec_raw[NB+2]
  unsigned long long* lsum;  // [4] fixed-point energy sums (kLScale)
  unsigned long long* counters;  // [CTR_TOTAL]
  double* jblue;           // [S*L] or nullptr
  double* out_shell;       // J, nubar, T_R, W, jblue scale, each [S]
  double* out_spec;        // [NB+2]
  double* vraw;            // [NB+2]
  unsigned long long* vcounts;  // [4]
  double* out_vspec;       // [NB+3]
  double* scalars;         // [8]
  void* packets;           // smc_packet_out records or nullptr
  LongState* longs;        // hand-off buffer
  uint64_t* long_order;    // [long_cap] this model's share of the launch-wide processing order
  uint64_t long_cap;
};

// One iteration of one model.
struct DevIter {
  uint64_t n_packets;      // N (energy 1/N)
  uint64_t n_work;         // packets in this launch
  const uint64_t* ids;     // device ids or nullptr (= slot index)
  uint64_t max_segments;
  uint32_t iteration;
  uint32_t flags;
  uint32_t long_budget;    // segments before a history moves to the group kernel (0: never)
  uint32_t n_virtual;      // v-packets per packet launch (0: none; then every history is
                           // handed to the group kernel right after injection)
  double T_param;          // > 0 overrides the device-resident T_inner
  double L_requested;
  double damping;
};

// One model of a launch: its arrays, its iteration, and its place in the
// launch-wide packet and hand-off numbering.
struct BatchEntry {
  DevModel m;
  DevIter it;
  uint64_t work_begin;     // first launch-wide packet index of this model
  uint64_t long_begin;     // first launch-wide hand-off index (set on the device)
};

// Arguments of every transport-path kernel.  A launch over one model passes
// its entry by value (`single`); a launch over many passes a device table.
struct LaunchArgs {
  BatchEntry single;
  const BatchEntry* table; // [n_models] (multi-model launches)
  int32_t n_models;
  int32_t pad;
  uint64_t total_work;     // packets over all models
  unsigned long long* ctr; // [3] work-queue head, hand-off total, hand-off queue head
  unsigned int* order_hist;  // [2 * kOrderBuckets] bucket counts, then cursors
  uint32_t max_lines;      // largest line count of the launch's models
  uint32_t hot;            // hand-off positions [0, hot) run at the highest wave priority,
                           // [hot, 3 hot) and [3 hot, 7 hot) one and two steps lower
};

// scalars[] slots
enum { SC_L_EMITTED = 0, SC_L_REABSORBED = 1, SC_L_CAPPED = 2, SC_L_INNER = 3,
       SC_T_USED = 4, SC_T_NEXT = 5 };

// Launch shape of one iteration (or one batch).
struct Shape {
  int transport_grid;
  int long_grid;   // wavefronts of the group-per-packet kernel
  int long_lanes;  // lanes per handed-off history: 16, 32 or 64 (64 without the extended
                   // code: the wavefront-per-history kernel)
  bool long_ext;   // some model of the launch runs v-packets or the macroatom mode: the
                   // group kernel variant with that code (more registers)
};

// Host-side launchers implemented in smc_kernels.hip.  `multi` selects the
// multi-model kernels (a.table valid) instead of the single-model ones.
hipError_t launch_geometry(const DevModel& m, const double* v_bounds, hipStream_t s);
hipError_t launch_iteration(const LaunchArgs& a, bool multi, const Shape& shape,
                            uint64_t max_jblue, hipEvent_t ev_start, hipEvent_t ev_stop,
                            hipStream_t s);
hipError_t transport_occupancy(bool multi, int* blocks_per_cu);
hipError_t long_occupancy(bool multi, int lanes, bool ext, int* blocks_per_cu);
int transport_block_threads();
int long_block_threads();
constexpr int kMaxBatchModels = 1024;

// ---------------------------------------------------------------------------
// plasma state and Sobolev depths
// ---------------------------------------------------------------------------
constexpr int kPlasmaMaxIons = 2048;     // per-shell ion tables live in LDS
constexpr int kPlasmaMaxElements = 256;
constexpr int kNlteMaxIons = 64;
constexpr int kNlteMaxLevels = 64;       // an NLTE system (n x n+1) lives in LDS
constexpr int kNlteMaxLines = 2048;      // lines of one NLTE ion (their level entries too)

// Per-line constants of the Sobolev depth, derived once at load (16 bytes).
struct PlasmaLine {
  double coef_g;           // (pi e^2 / m_e c) f (c / nu) t_exp g_l
  int32_t lower, upper;    // global level indices
};

// Per-line constants of an NLTE ion's rates, derived once at load (64 bytes).
struct NlteLine {
  double A_ul, B_ul, B_lu;  // Einstein coefficients (B for J in intensity units)
  double c_ul;              // 8.629e-6 Upsilon / g_u: C_ul = c_ul / T_e^{1/2}
  double g_ratio;           // g_u / g_l: C_lu = C_ul g_ratio exp(-h nu / k T_e)
  double nu;
  int32_t line;             // global line index
  int16_t lo, up;           // level indices within the ion
  int32_t pad[2];
};

// Per-line Einstein coefficients of the macro-atom rates, derived once at load.
struct MacroLine {
  double A_ul, B_ul, B_lu;  // B for J in intensity units
  double pad;
};

// Entry kinds of a macro-atom row (see launch_plasma_update)
constexpr uint8_t kMacroEmit = 0, kMacroDown = 1, kMacroUp = 2;

struct PlasmaLayout {
  uint64_t elem_ion_ptr;   // [E+1] i32
  uint64_t ion_chi, ion_zeta;  // [n_ions]
  uint64_t ion_level_ptr;  // [n_ions+1] i32
  uint64_t level_energy, level_g;  // [n_levels]
  uint64_t level_meta;     // [n_levels] u8
  uint64_t level_ion;      // [n_levels] i32
  uint64_t line_f;         // [L] staging of the oscillator strengths
  uint64_t lines;          // [L] PlasmaLine
  uint64_t density;        // [S*E]
  uint64_t field;          // [2S] T_R, W given by the host
  uint64_t partition, ion_density;  // [S*n_ions]
  uint64_t level_pop;      // [S*n_levels] populations n
  uint64_t level_x;        // [S*n_levels] n / g
  uint64_t clamped;        // [2] u64: inverted lines, singular NLTE systems
  uint64_t nlte_ions;      // [n_nlte] i32
  uint64_t nlte_line_ptr;  // [n_nlte+1] i32 offsets into nlte_lines
  uint64_t nlte_lines;     // NlteLine records of every NLTE ion's lines
  uint64_t nlte_lev_ptr;   // [n_nlte][kNlteMaxLevels+1] i32: level r's entries of ion j are
                           // nlte_ent[2 nlte_line_ptr[j] + ptr[r] .. + ptr[r+1])
  uint64_t nlte_ent;       // [2 * NLTE lines] i32: (line position << 16) | (other level << 1) |
                           // (1 if the level is the line's lower one), by level, in line order
  uint64_t line_upsilon;   // [L] staging of the collision strengths
  uint64_t macro_lines;    // [L] MacroLine (macro-atom tables derived on the device)
  uint64_t em_via;         // [3L] i32: the line of each macro-atom entry
  uint64_t em_kind;        // [3L] u8: kMacroEmit / kMacroDown / kMacroUp
  uint64_t total;
};

struct DevPlasma {
  int32_t S, E, n_ions, n_levels;
  int32_t L, Lp;
  int32_t ionization, excitation;
  double delta;
  double t_exp;
  const int32_t* elem_ion_ptr;
  const double* ion_chi;
  const double* ion_zeta;
  const int32_t* ion_level_ptr;
  const double* level_energy;
  const double* level_g;
  const uint8_t* level_meta;
  const int32_t* level_ion;
  const double* line_f;
  PlasmaLine* lines;
  const double* density;
  const double* T_R;       // [S] radiation field of this update
  const double* W;         // [S]
  double* partition;
  double* ion_density;
  double* level_pop;
  double* level_x;
  unsigned long long* clamped;
  int32_t n_nlte;          // NLTE ions of this update (0: none)
  int32_t jb_detailed;     // J_b from `jblue` (else W B_nu(T_R))
  const int32_t* nlte_ions;
  const int32_t* nlte_line_ptr;
  NlteLine* nlte_lines;
  const int32_t* nlte_lev_ptr;
  const int32_t* nlte_ent;
  const double* line_upsilon;
  const double* jblue;     // the model's normalised J_blue [S*L], or nullptr
  double* n_e;             // the model's [S]
  double* tau;             // the model's [S*Lp]
  const double* line_nu;   // the model's [Lp]
  // macro-atom tables derived from this update (macro != 0): the model's
  // rows and per-shell cumulative probabilities
  int32_t macro;
  int32_t macro_detailed;  // J_b of the upward jumps from `jblue` (else W B_nu(T_R))
  int64_t n_em;
  const int64_t* level_ptr;  // the model's [n_levels+1]
  const int32_t* em_via;
  const uint8_t* em_kind;
  MacroLine* macro_lines;
  double* em_cum;          // the model's [S*n_em]
};

// Launcher implemented in smc_measure.hip: 8 * n_cu workgroups of 256 lanes,
// each lane adding 1.0 to a double of `table` at a new pseudo-random place in
// each of n_rounds rounds (a wavefront's 64 consecutive doubles, or with
// `scattered` a place per lane).
hipError_t launch_atomic_rate(double* table, uint64_t n_doubles, uint32_t n_rounds, int scattered,
                              int n_cu, hipStream_t s);

// Launchers implemented in smc_plasma.hip.
hipError_t launch_plasma_lines(const DevPlasma& p, int n_nlte_lines, hipStream_t s);
hipError_t launch_plasma_update(const DevPlasma& p, hipStream_t s);

}  // namespace smc
