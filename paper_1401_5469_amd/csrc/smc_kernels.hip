// smc_kernels.hip -- gfx950 kernels of the r-packet Monte Carlo transport
// (Kerzendorf & Sim 2014, sections 2.1-2.9).
//
// Every kernel of the transport path comes in two instantiations: one for a
// single model (its description travels as a kernel argument, so per-model
// values are wave-uniform and live in scalar registers) and one for a launch
// over many models of uneven size (a device table; each lane carries the
// model of its current packet).  All arithmetic on positions, directions,
// frequencies and energies is FP64.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "../../include/smc.h"
#include "smc_internal.h"

namespace smc {
namespace {

// CGS constants (CODATA 2018)
constexpr double kC = 2.99792458e10;
constexpr double kH = 6.62607015e-27;
constexpr double kKB = 1.380649e-16;
constexpr double kSigmaSB = 5.670374419e-5;
constexpr double kSigmaT = 6.6524587321e-25;
constexpr double kZeta5 = 1.0369277551433699263;
constexpr double kPi = 3.14159265358979323846;
constexpr double kZeta4 = 1.0823232337111381915;  // pi^4 / 90 = sum over l of l^-4
constexpr int kPlanckTerms = 1000;

constexpr int kBlock = 256;
constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al. 2011).  Draw d of packet p in iteration i is
// the 64-bit word (x[2j+1] << 32) | x[2j], j = d%2, of the block x with
// counter {d/2, p_lo, p_hi, i} and key {seed_lo, seed_hi}.
// ---------------------------------------------------------------------------
struct Block {
  uint64_t a, b;  // the block's two 64-bit draws
};

__device__ __forceinline__ Block philox_block(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1) {
  constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint32_t hi0 = __umulhi(M0, c0), lo0 = M0 * c0;
    const uint32_t hi1 = __umulhi(M1, c2), lo1 = M1 * c2;
    const uint32_t n0 = hi1 ^ c1 ^ k0;
    const uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  Block r;
  r.a = ((uint64_t)c1 << 32) | (uint64_t)c0;
  r.b = ((uint64_t)c3 << 32) | (uint64_t)c2;
  return r;
}

__device__ __forceinline__ uint64_t fnv_word(uint64_t h, uint64_t w) {
  return (h ^ w) * 0x100000001b3ull;
}
__device__ __forceinline__ uint64_t fnv_event(uint64_t h, int kind, int shell, int64_t line,
                                              int64_t emit) {
  h = fnv_word(h, (uint64_t)(int64_t)kind);
  h = fnv_word(h, (uint64_t)(int64_t)shell);
  h = fnv_word(h, (uint64_t)line);
  return fnv_word(h, (uint64_t)emit);
}

// first-order Doppler factor for homologous flow, D = 1 - mu r / (c t)
__device__ __forceinline__ double doppler(double r, double mu, double ct) {
  return 1.0 - (mu * r) / ct;
}

// closest redward line: first k with nu_k < nu_cmf in the non-increasing list
__device__ __forceinline__ int32_t first_below(const double* __restrict__ nu, int32_t n,
                                               double nu_cmf) {
  int32_t lo = 0, hi = n;
  while (lo < hi) {
    const int32_t mid = lo + ((hi - lo) >> 1);
    if (nu[mid] < nu_cmf)
      hi = mid;
    else
      lo = mid + 1;
  }
  return lo;
}

enum { EV_SHELL_OUT = 1, EV_SHELL_IN = 2, EV_ESCATTER = 3, EV_LINE = 4 };

// ---------------------------------------------------------------------------
// model set-up (section 2.1): radii r = v t_exp, shell volumes, and the
// initial radiation field of section 2.8 (T_R = 10^4 K, geometric dilution at
// the shell centre)
// ---------------------------------------------------------------------------

__global__ void geometry_kernel(DevModel m, const double* __restrict__ v_bounds) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i <= m.S) const_cast<double*>(m.r_bounds)[i] = v_bounds[i] * m.t_exp;
  if (i < m.S) {
    const double ri = v_bounds[i] * m.t_exp, ro = v_bounds[i + 1] * m.t_exp;
    const_cast<double*>(m.volume)[i] = 4.0 * kPi / 3.0 * (ro * ro * ro - ri * ri * ri);
    const double r_inner = v_bounds[0] * m.t_exp;
    const double rc = 0.5 * (v_bounds[i] + v_bounds[i + 1]) * m.t_exp;
    const double q = r_inner / rc;
    m.out_shell[2 * m.S + i] = 10000.0;
    m.out_shell[3 * m.S + i] = 0.5 * (1.0 - sqrt(1.0 - q * q));
  }
  if (i < 8) m.scalars[i] = 0.0;
}

// the model entry of a launch
#define ENTRY(a, k) (kMulti ? (a).table[(k)] : (a).single)

// ---------------------------------------------------------------------------
// zero every tally of the iteration and fix T_inner (no memset: graph-safe);
// blockIdx.y selects the model
// ---------------------------------------------------------------------------
template <bool kMulti>
__global__ void reset_kernel(LaunchArgs a) {
  const int k = kMulti ? (int)blockIdx.y : 0;
  const DevModel& m = ENTRY(a, k).m;
  const DevIter& it = ENTRY(a, k).it;
  const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const size_t n_raw = 2 * (size_t)m.S + (size_t)m.n_bins + 2;
  for (size_t i = tid; i < n_raw; i += stride) m.raw[i] = 0.0;
  if (tid < 4) m.lsum[tid] = 0ull;
  for (size_t i = tid; i < n_raw - 2 * (size_t)m.S; i += stride) m.vraw[i] = 0.0;
  if (tid < 4) m.vcounts[tid] = 0ull;
  if (tid < CTR_TOTAL) m.counters[tid] = 0ull;
  if (m.jblue && (it.flags & SMC_F_JBLUE)) {
    const size_t n = (size_t)m.S * (size_t)m.L;
    for (size_t i = tid; i < n; i += stride) m.jblue[i] = 0.0;
  }
  if (tid == 0) m.scalars[SC_T_USED] = it.T_param > 0.0 ? it.T_param : m.scalars[SC_T_NEXT];
  if (kMulti && k == 0 && tid < 3) a.ctr[tid] = 0ull;
  if (k == 0)
    for (size_t i = tid; i < (size_t)kOrderBuckets; i += stride) a.order_hist[i] = 0u;
}

// ---------------------------------------------------------------------------
// The transport (sections 2.4-2.7, 2.9) runs in two kernels.
//
// transport_kernel: one packet per lane.  A persistent grid pulls packets from
// a launch-wide work queue (one atomic per wavefront per refill), so a lane
// whose packet ends picks up the next one, from any model of the launch,
// while its neighbours are still marching.  A history still alive after
// `long_budget` flight segments is saved to its model's hand-off buffer and
// its lane moves on: in a line-forest model a few per cent of the packets
// carry about half of the segments, and a lane-per-packet wavefront runs
// those latency-bound.
//
// long_kernel: one packet per group of G = 16, 32 or 64 lanes, for the
// handed-off histories.  The G lanes hold the next 2G draws of the packet's
// stream with their logarithms precomputed, and the next G lines of its
// shell, so a segment's dependent chain is only the geometry and frame
// arithmetic; J_blue updates go out from the lanes that own the passed lines
// in parallel.  The uniform per-packet arithmetic is repeated in every lane
// of a group, so narrower groups put more histories through each
// instruction; wider ones march more lines per step.
//
// Both follow the arithmetic of the FP64 reference formulation step by step,
// with its operand order and correctly rounded quotients and roots, so a
// history reproduces to the last bit; the one departure is the depth left
// after the lines a group passes at once, a sum in prefix order (which can
// change a comparison only when both sides agree to a few ulps).
// Estimator tallies: J and nu-bar accumulate in registers while a packet
// stays in one shell of one model, event counters and luminosity sums in a
// private LDS slot per lane (per group) while it stays on one model; both reach
// HBM with atomics only when that changes.  The spectrum takes one atomic
// per escaping packet, J_blue one per passed resonance.
// ---------------------------------------------------------------------------

__device__ __forceinline__ double to_uniform(uint64_t w) {
  return ((double)(w >> 12) + 0.5) * 0x1p-52;
}

struct StreamKey {
  uint32_t k0, k1;  // seed words
  uint32_t p0, p1;  // packet id words
  uint32_t iter;
};

__device__ __forceinline__ Block stream_block(const StreamKey& s, uint32_t blk) {
  return philox_block(blk, s.p0, s.p1, s.iter, s.k0, s.k1);
}

// four-draw window of one lane's stream (two blocks)
struct RngWindow {
  uint64_t w0, w1, w2, w3;  // draws 2*block .. 2*block+3
  uint32_t block;           // block index of w0, w1
  uint32_t pos;             // next draw relative to w0
};

__device__ __forceinline__ uint64_t rng_word(const RngWindow& g, uint32_t i) {
  const uint64_t lo = (i & 1) ? g.w1 : g.w0;
  const uint64_t hi = (i & 1) ? g.w3 : g.w2;
  return (i & 2) ? hi : lo;
}

__device__ __forceinline__ double rng_next(RngWindow& g) {
  const double u = to_uniform(rng_word(g, g.pos));
  g.pos += 1;
  return u;
}

// make at least `need` (<= 3) draws available
__device__ __forceinline__ void rng_topup(RngWindow& g, uint32_t need, const StreamKey& s) {
  if (g.pos + need > 4) {
    g.w0 = g.w2;
    g.w1 = g.w3;
    g.block += 1;
    g.pos -= 2;
    const Block nb = stream_block(s, g.block + 1);
    g.w2 = nb.a;
    g.w3 = nb.b;
    if (g.pos + need > 4) {
      g.w0 = g.w2;
      g.w1 = g.w3;
      g.block += 1;
      g.pos -= 2;
      const Block nb2 = stream_block(s, g.block + 1);
      g.w2 = nb2.a;
      g.w3 = nb2.b;
    }
  }
}

// Planck sampling in x = h nu / k T from five uniforms (mixture term l with
// weight l^-4 / zeta(4), then a Gamma(4, l) deviate)
__device__ __forceinline__ double planck_from(double u_l, double u1, double u2, double u3,
                                              double u4) {
  const double target = u_l * kZeta4;
  double acc = 0.0;
  int l = 1;
  for (; l <= kPlanckTerms; ++l) {
    const double dl = (double)l;
    acc += 1.0 / (dl * dl * dl * dl);
    if (acc >= target) break;
  }
  if (l > kPlanckTerms) l = kPlanckTerms;
  return -log(((u1 * u2) * u3) * u4) / (double)l;
}

// Correctly rounded FP64 quotients and square roots.  Wherever the FP64
// reference formulation divides or takes a root, the kernels produce the
// correctly rounded result, bit for bit what an IEEE division or square root
// gives, so that histories reproduce to the last bit.
//
// Division: a reciprocal estimate of the divisor b refined by two Newton
// steps (y), a product q = a y, and one correction with the exact remainder,
// q + (a - b q) y, each step a fused multiply-add (Markstein 1990, "Computation
// of elementary functions on the IBM RISC System/6000 processor").  These are
// the steps of the general gfx950 division sequence without its operand
// scaling and special-case fix-up, which are identities when b and 1/b are
// normal, |a| >= 2^-900 (or a == 0) and a/b is normal: every quotient the
// transport forms satisfies that.  A divisor used more than once (c t, the
// Doppler factor of an event) keeps its refined reciprocal.
struct Divisor {
  double b, y;  // divisor and its refined reciprocal
};

__device__ __forceinline__ Divisor divisor(double b) {
  double y = __builtin_amdgcn_rcp(b);
  double e = fma(-b, y, 1.0);
  y = fma(y, e, y);
  e = fma(-b, y, 1.0);
  y = fma(y, e, y);
  return Divisor{b, y};
}

__device__ __forceinline__ double quot(double a, const Divisor& d) {
  const double q = a * d.y;
  const double r = fma(-d.b, q, a);
  return fma(r, d.y, q);
}

// a / b where |a| may be arbitrarily small (optical depths left after many
// lines, tiny opacities): the general sequence outside the range above
__device__ __forceinline__ double quot_checked(double a, const Divisor& d) {
  const double aa = fabs(a), ab = fabs(d.b);
  if (aa >= 0x1p-900 && ab >= 0x1p-900 && aa <= 0x1p900 && ab <= 0x1p900) return quot(a, d);
  return a / d.b;
}

// Square root: reciprocal square-root estimate, then the coupled Newton
// iteration for sqrt(x) and 1/(2 sqrt(x)) with two exact-residual corrections
// (Markstein 1990; the gfx950 sqrt sequence without its scaling of x below
// 2^-767).  The transport takes roots of squared distances only, which the
// radius range the library accepts ([2^-300, 2^300] cm) keeps at zero or in
// [2^-700, 2^700]; zero gives zero.
__device__ __forceinline__ double root(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y;
  double h = y * 0.5;
  const double r = fma(-h, g, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  double d = fma(-g, g, x);
  g = fma(d, h, g);
  d = fma(-g, g, x);
  g = fma(d, h, g);
  return x > 0.0 ? g : 0.0;
}

// root(x) for x > 0 (a radius after a move: at least the inner boundary's)
__device__ __forceinline__ double root_pos(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y;
  double h = y * 0.5;
  const double r = fma(-h, g, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  double d = fma(-g, g, x);
  g = fma(d, h, g);
  d = fma(-g, g, x);
  return fma(d, h, g);
}

// distance along (r, mu) to the boundary of shell [r_in, r_out] met first
// (ray-sphere intersection; a tangent ray misses the inner sphere)
// (from the squared radii; q is +0 when r_x^2 = b, so its clamp keeps the sign)
__device__ __forceinline__ double shell_distance_sq(double r, double mu, double rmu, double r_in2,
                                                    double r_out2, bool& inward) {
  const double b = r * r * ((1.0 - mu) * (1.0 + mu));
  inward = mu < 0.0 && b < r_in2;
  const double q = fmax((inward ? r_in2 : r_out2) - b, 0.0);
  const double sq = root(q);
  const double d = inward ? -rmu - sq : sq - rmu;
  return d < 0.0 ? 0.0 : d;
}

__device__ __forceinline__ double shell_distance(double r, double mu, double rmu, double r_in,
                                                 double r_out, bool& inward) {
  return shell_distance_sq(r, mu, rmu, r_in * r_in, r_out * r_out, inward);
}


// The entry a transition row [lo, hi) selects for a uniform draw u: the first
// j in [lo, hi - 1) with cum[j] > u, else the row's last entry (section 2.5).
// Rows are non-decreasing (checked when the model is loaded), so bisection
// finds the entry a scan from lo would stop at, in log2(hi - lo) loads whose
// count hardly varies between the lanes of a wavefront.
__device__ __forceinline__ int64_t row_select(const double* cum, int64_t lo, int64_t hi,
                                              double u) {
  int64_t a = lo, b = hi - 1;
  while (a < b) {
    const int64_t mid = a + ((b - a) >> 1);
    if (cum[mid] > u)
      b = mid;
    else
      a = mid + 1;
  }
  return a;
}

// spectrum bin of an escaping lab frequency (section 2.9): n_bins is the
// underflow slot (also taken by a NaN), n_bins+1 the overflow slot
__device__ __forceinline__ int spectrum_bin(const DevModel& m, double nu) {
  if (!(nu >= m.nu_min)) return m.n_bins;
  const double dnu_bin = (m.nu_max - m.nu_min) / (double)m.n_bins;
  const double f = floor((nu - m.nu_min) / dnu_bin);
  return f >= (double)m.n_bins ? m.n_bins + 1 : (int)f;
}

__device__ __forceinline__ void write_record(const DevModel& m, uint64_t slot, uint64_t pid,
                                             int status, int shell, double nu, double E,
                                             double mu, double r, double mu0, double nu_cmf0,
                                             uint64_t n_seg, uint32_t n_esc, uint32_t n_line,
                                             uint64_t n_pass, uint64_t hash, int32_t last_line) {
  smc_packet_out rec;
  rec.id = pid;
  rec.status = status;
  rec.shell = shell;
  rec.nu = nu;
  rec.energy = E;
  rec.mu = mu;
  rec.r = r;
  rec.mu0 = mu0;
  rec.nu_cmf0 = nu_cmf0;
  rec.n_segments = n_seg;
  rec.n_escatter = n_esc;
  rec.n_line = n_line;
  rec.n_passes = n_pass;
  rec.hash = hash;
  rec.last_line = last_line;
  static_cast<smc_packet_out*>(m.packets)[slot] = rec;
}

// Make the values available in registers at this point (the compiler
// inserts the wait for any load that produced them here).
__device__ __forceinline__ void settle() {}
template <typename T, typename... R>
__device__ __forceinline__ void settle(const T& x, const R&... rest) {
  asm volatile("" ::"v"(x));
  settle(rest...);
}

// per-lane tally slot in LDS: luminosity sums and event counters of the
// lane's current model
struct LaneTally {
  unsigned long long L[3];  // fixed-point escaped, reabsorbed, capped energy
  unsigned long long c[SMC_N_COUNTERS];
  unsigned long long vc[3];  // v-packets launched, counted, resonances swept
};

__device__ __forceinline__ void lane_tally_clear(LaneTally& t) {
  t.L[0] = t.L[1] = t.L[2] = 0ull;
  t.vc[0] = t.vc[1] = t.vc[2] = 0ull;
#pragma unroll
  for (int i = 0; i < SMC_N_COUNTERS; ++i) t.c[i] = 0ull;
}

__device__ __forceinline__ void lane_tally_flush(const DevModel& m, LaneTally& t) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
    if (t.L[i]) atomicAdd(&m.lsum[i], t.L[i]);
#pragma unroll
  for (int i = 0; i < SMC_N_COUNTERS; ++i)
    if (t.c[i]) atomicAdd(&m.counters[i], t.c[i]);
#pragma unroll
  for (int i = 0; i < 3; ++i)
    if (t.vc[i]) atomicAdd(&m.vcounts[i], t.vc[i]);
  lane_tally_clear(t);
}

// end of a history: luminosity and event tallies (section 2.9 spectrum with
// one global atomic)
__device__ __forceinline__ void lane_tally_end(const DevModel& m, LaneTally& t, int status,
                                               double nu, double E, uint64_t n_seg,
                                               uint64_t n_pass, uint32_t n_line,
                                               uint32_t n_esc, bool dead_atom) {
  const unsigned long long q = (unsigned long long)__double2ll_rn(E * kLScale);
  if (status == SMC_ESCAPED) {
    unsafeAtomicAdd(&m.raw[2 * m.S + spectrum_bin(m, nu)], E);
    t.L[0] += q;
    t.c[SMC_C_ESCAPED] += 1;
  } else if (status == SMC_REABSORBED) {
    t.L[1] += q;
    t.c[SMC_C_REABSORBED] += 1;
  } else {
    t.L[2] += q;
    t.c[SMC_C_CAPPED] += 1;
  }
  // every segment ends in exactly one of line event, Thomson or crossing,
  // except a last one whose macro atom never deactivated
  t.c[SMC_C_SEGMENTS] += n_seg;
  t.c[SMC_C_LINE_PASSES] += n_pass;
  t.c[SMC_C_LINE_EVENTS] += n_line;
  t.c[SMC_C_ESCATTERS] += n_esc;
  t.c[SMC_C_CROSSINGS] += n_seg - n_line - n_esc - (dead_atom ? 1 : 0);
}

// the per-model values the segment loop of a lane reads
struct View {
  const double* r_bounds;
  const double* n_e;
  const double* line_nu;
  const double* tau;
  double* jblue;          // nullptr when J_blue is not tallied
  const int32_t* line_upper;  // downbranch tables
  const int64_t* level_ptr;
  const int32_t* em_line;
  const double* em_cum;
  double ct;
  Divisor rct;            // c t with its refined reciprocal
  uint64_t max_segments, budget;
  int32_t S, L, Lp;
  bool downbranch;         // emission rows shared by all shells, no internal jumps
  bool macroatom;          // internal jumps, one probability set per shell
  int64_t n_em;
  bool records;           // per-packet records (and their event hash) are kept
  uint32_t k0, k1, iter;  // random-number key and counter word
  uint32_t n_virtual;     // v-packets per packet launch
  double e_unit;          // comoving energy of an injected packet, 1/N
};

__device__ __forceinline__ View make_view(const DevModel& m, const DevIter& it) {
  View v;
  v.r_bounds = m.r_bounds;
  v.n_e = m.n_e;
  v.line_nu = m.line_nu;
  v.tau = m.tau;
  v.jblue = (m.jblue != nullptr && (it.flags & SMC_F_JBLUE)) ? m.jblue : nullptr;
  v.line_upper = m.line_upper;
  v.level_ptr = m.level_ptr;
  v.em_line = m.em_line;
  v.em_cum = m.em_cum;
  v.ct = m.ct;
  v.rct = divisor(m.ct);
  v.max_segments = it.max_segments;
  // with v-packets every history goes to the group kernel before its first
  // segment; otherwise after long_budget segments (never when 0)
  v.budget = it.n_virtual ? 0ull : ((it.long_budget > 0 && m.longs) ? it.long_budget : ~0ull);
  v.S = m.S;
  v.L = m.L;
  v.Lp = m.Lp;
  v.downbranch = m.mode == SMC_DOWNBRANCH;
  v.macroatom = m.mode == SMC_MACROATOM;
  v.n_em = m.n_em;
  v.records = m.packets != nullptr && (it.flags & SMC_F_PACKETS);
  v.k0 = (uint32_t)m.seed;
  v.k1 = (uint32_t)(m.seed >> 32);
  v.iter = it.iteration;
  v.n_virtual = it.n_virtual;
  v.e_unit = 1.0 / (double)it.n_packets;
  return v;
}

// ---------------------------------------------------------------------------
// lane-per-packet kernel
// ---------------------------------------------------------------------------
// The multi-model build keeps its per-lane model view in registers (188
// VGPRs, 2 wavefronts per SIMD); held to 128 it spills the rarely used view
// fields and runs 4 wavefronts per SIMD, 6 % faster on a 64-model launch.
template <bool kMulti>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kMulti ? 4 : 1)))
void transport_kernel(LaunchArgs a) {
  extern __shared__ unsigned char lds_raw[];
  LaneTally* lane_tally = reinterpret_cast<LaneTally*>(lds_raw);
  uint64_t* work_begin = reinterpret_cast<uint64_t*>(lds_raw + sizeof(LaneTally) * kBlock);
  LaneTally& tly = lane_tally[threadIdx.x];
  lane_tally_clear(tly);
  if (kMulti) {
    for (int i = threadIdx.x; i <= a.n_models; i += blockDim.x)
      work_begin[i] = i < a.n_models ? a.table[i].work_begin : a.total_work;
    __syncthreads();
  }
  const int lane = threadIdx.x & (kWave - 1);
  unsigned long long* queue = kMulti ? a.ctr : a.single.m.counters + CTR_QUEUE;
  const uint64_t total_work = kMulti ? a.total_work : a.single.it.n_work;

  // the lane's current model
  int model = kMulti ? -1 : 0;
  uint64_t model_end = 0;
  View v = make_view(a.single.m, a.single.it);
  int tally_model = kMulti ? -1 : 0;

  // packet state
  uint64_t slot = 0, pid = 0;
  double r = 0.0, mu = 0.0, nu = 0.0, E = 0.0, mu0 = 0.0, nu_cmf0 = 0.0;
  int32_t shell = 0, next_line = 0, last_line = -1;
  uint64_t n_seg = 0, n_pass = 0, hash = 0;
  uint32_t n_esc = 0, n_line = 0;
  bool handoff_tried = false;
  RngWindow g;
  StreamKey sk;
  sk.k0 = v.k0;
  sk.k1 = v.k1;
  sk.iter = v.iter;
  sk.p0 = sk.p1 = 0;
  // cached shell parameters
  int32_t c_shell = -1;
  double c_rin = 0.0, c_rout = 0.0, c_ne = 0.0;
  // line window: lines wbase..wbase+3 of shell wshell of the current model,
  // and the J_blue the lane has tallied on them since the window was loaded
  int32_t wbase = -8, wshell = -1;
  double wn0 = 0, wn1 = 0, wn2 = 0, wn3 = 0, wt0 = 0, wt1 = 0, wt2 = 0, wt3 = 0;
  double wj0 = 0, wj1 = 0, wj2 = 0, wj3 = 0;
  // The window's J_blue leaves in one atomic per line when the window does,
  // issued after the next window's loads: a wait for those loads then never
  // includes these atomics, which complete while the lane computes.
  auto flush_window_jblue = [&](double* jrow) {
    if (jrow) {
      if (wj0 != 0.0) unsafeAtomicAdd(&jrow[wbase], wj0);
      if (wj1 != 0.0) unsafeAtomicAdd(&jrow[wbase + 1], wj1);
      if (wj2 != 0.0) unsafeAtomicAdd(&jrow[wbase + 2], wj2);
      if (wj3 != 0.0) unsafeAtomicAdd(&jrow[wbase + 3], wj3);
    }
    wj0 = wj1 = wj2 = wj3 = 0.0;
  };
  auto jblue_row = [&](int32_t sh) {
    return (v.jblue && sh >= 0) ? v.jblue + (size_t)sh * (size_t)v.L : (double*)nullptr;
  };
  // J and nu-bar of one shell of one model, held in registers
  double acc_J = 0.0, acc_nb = 0.0;
  int acc_shell = -1, acc_model = -1;

  bool active = false, exhausted = false;

  for (;;) {
    // ---- refill finished lanes from the work queue, one atomic per wave
    const bool need = !active && !exhausted;
    const unsigned long long need_mask = __ballot(need);
    if (need_mask) {
      const int leader = __ffsll((long long)need_mask) - 1;
      unsigned long long base = 0;
      if (lane == leader) base = atomicAdd(queue, (unsigned long long)__popcll(need_mask));
      base = __shfl(base, leader, kWave);
      if (need) {
        const unsigned long long below = need_mask & ((1ull << lane) - 1ull);
        const uint64_t gidx = base + (uint64_t)__popcll(below);
        if (gidx < total_work) {
          if (kMulti && (model < 0 || gidx >= model_end || gidx < work_begin[model])) {
            // packet of another model: locate it, switch the lane's view
            int lo = 0, hi = a.n_models - 1;
            while (lo < hi) {
              const int mid = (lo + hi + 1) >> 1;
              if (work_begin[mid] <= gidx)
                lo = mid;
              else
                hi = mid - 1;
            }
            flush_window_jblue(jblue_row(wshell));
            model = lo;
            model_end = work_begin[lo + 1];
            v = make_view(a.table[model].m, a.table[model].it);
            sk.k0 = v.k0;
            sk.k1 = v.k1;
            sk.iter = v.iter;
            c_shell = -1;
            wshell = -1;
          }
          const DevModel& m = ENTRY(a, model).m;
          const DevIter& it = ENTRY(a, model).it;
          // ---- injection at the inner boundary (section 2.4)
          slot = kMulti ? gidx - work_begin[model] : gidx;
          pid = it.ids ? it.ids[slot] : slot;
          sk.p0 = (uint32_t)pid;
          sk.p1 = (uint32_t)(pid >> 32);
          // draws 0..5: mu, the Planck mixture term, four Gamma(4) uniforms
          const Block b0 = stream_block(sk, 0), b1 = stream_block(sk, 1);
          const Block b2 = stream_block(sk, 2), b3 = stream_block(sk, 3);
          g.w0 = b2.a;
          g.w1 = b2.b;
          g.w2 = b3.a;
          g.w3 = b3.b;
          g.block = 2;
          g.pos = 2;
          mu = sqrt(to_uniform(b0.a));  // zero limb darkening
          const double x = planck_from(to_uniform(b0.b), to_uniform(b1.a), to_uniform(b1.b),
                                       to_uniform(b2.a), to_uniform(b2.b));
          const double T_inner = m.scalars[SC_T_USED];
          const double r_inner = v.r_bounds[0];
          const double nu_cmf = x * kKB * T_inner / kH;
          const double D0 = doppler(r_inner, mu, v.ct);
          nu = nu_cmf / D0;
          E = (1.0 / (double)it.n_packets) / D0;
          r = r_inner;
          mu0 = mu;
          nu_cmf0 = nu_cmf;
          shell = 0;
          next_line = v.L > 0 ? first_below(v.line_nu, v.L, nu_cmf) : 0;
          n_seg = n_pass = 0;
          n_esc = n_line = 0;
          hash = 0xcbf29ce484222325ull;
          last_line = -1;
          handoff_tried = false;
          active = true;
        } else {
          exhausted = true;
        }
      }
    }
    if (__ballot(active) == 0ull) break;
    if (!active) continue;
    if (kMulti && tally_model != model) {
      if (tally_model >= 0) lane_tally_flush(a.table[tally_model].m, tly);
      tally_model = model;
    }

    int status = SMC_LIVE;
    bool dead_atom = false;  // the history ended in a macro atom that never deactivated
    if (n_seg >= v.max_segments) {
      status = SMC_CAPPED;
    } else if (n_seg >= v.budget && !handoff_tried) {
      // ---- hand the history to the group-per-packet kernel
      handoff_tried = true;
      const DevModel& m = ENTRY(a, model).m;
      const unsigned long long h = atomicAdd(&m.counters[CTR_LONG_COUNT], 1ull);
      if (h < m.long_cap) {
        LongState st;
        st.slot = slot;
        st.pid = pid;
        st.r = r;
        st.mu = mu;
        st.nu = nu;
        st.E = E;
        st.mu0 = mu0;
        st.nu_cmf0 = nu_cmf0;
        st.n_seg = n_seg;
        st.n_pass = n_pass;
        st.hash = hash;
        st.draw = 2ull * g.block + g.pos;
        st.shell = shell;
        st.next_line = next_line;
        st.last_line = last_line;
        st.n_esc = n_esc;
        st.n_line = n_line;
        st.pad = 0;
        m.longs[h] = st;
        active = false;
        continue;
      }
    }
    if (status == SMC_LIVE) {
      // ---- one flight segment (section 2.6)
      n_seg += 1;
      rng_topup(g, 3, sk);  // tau_event + at most two event draws
      const double tau0 = -log(rng_next(g));
      const int sh = shell;
      if (sh != c_shell) {
        c_shell = sh;
        c_rin = v.r_bounds[sh];
        c_rout = v.r_bounds[sh + 1];
        c_ne = v.n_e[sh];
        // wait for these loads here, on a shell change, rather than at every
        // segment (where the wait would also cover the J_blue atomics in flight)
        settle(c_rin, c_rout, c_ne);
      }
      const double rmu = r * mu;
      const double D = 1.0 - quot(mu * r, v.rct);
      const double nu_cmf = nu * D;
      const double e_cmf = E * D;
      bool inward;
      const double d_shell = shell_distance(r, mu, rmu, c_rin, c_rout, inward);
      const double kappa = kSigmaT * c_ne * D;  // Thomson opacity with D
      const Divisor rkappa = divisor(kappa);
      const double ct_over_nu = quot(v.ct, divisor(nu));
      const Divisor rnn = divisor(nu * nu);  // J_blue weight E nu_k / nu^2

      // line march: pass redward lines while d_line is the shortest distance;
      // tau_rem is the optical depth left for electrons after the lines passed
      double tau_rem = tau0;
      double d_electron = kappa > 0.0 ? quot_checked(tau_rem, rkappa) : INFINITY;
      int32_t k = next_line;
      bool line_hit = false;
      double d_line = 0.0, nu_hit = 0.0;
      const double* __restrict__ tau_row = v.tau + (size_t)sh * (size_t)v.Lp;
      const bool jb_on = v.jblue != nullptr;
      bool stop = k >= v.L;
      while (!stop) {
        const int32_t base = k & ~3;
        if (base != wbase || sh != wshell) {
          const double2* pn = reinterpret_cast<const double2*>(v.line_nu + base);
          const double2* pt = reinterpret_cast<const double2*>(tau_row + base);
          const double2 n01 = pn[0], n23 = pn[1], t01 = pt[0], t23 = pt[1];
          flush_window_jblue(jblue_row(wshell));
          wn0 = n01.x; wn1 = n01.y; wn2 = n23.x; wn3 = n23.y;
          wt0 = t01.x; wt1 = t01.y; wt2 = t23.x; wt3 = t23.y;
          wbase = base;
          wshell = sh;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const double nu_k = j == 0 ? wn0 : j == 1 ? wn1 : j == 2 ? wn2 : wn3;
          const double tau_k = j == 0 ? wt0 : j == 1 ? wt1 : j == 2 ? wt2 : wt3;
          if (!stop && base + j >= k) {
            if (base + j >= v.L) {
              stop = true;
            } else {
              double dl = (nu_cmf - nu_k) * ct_over_nu;
              dl = dl < 0.0 ? 0.0 : dl;
              if (!(dl < d_electron && dl < d_shell)) {
                stop = true;
              } else {
                n_pass += 1;
                if (jb_on) {
                  const double w = quot(E * nu_k, rnn);
                  if (j == 0) wj0 += w;
                  if (j == 1) wj1 += w;
                  if (j == 2) wj2 += w;
                  if (j == 3) wj3 += w;
                }
                if (tau_k + kappa * dl > tau_rem) {
                  line_hit = true;
                  d_line = dl;
                  nu_hit = nu_k;
                  stop = true;
                } else {
                  tau_rem -= tau_k;
                  if (kappa > 0.0) d_electron = quot_checked(tau_rem, rkappa);
                  k = base + j + 1;
                }
              }
            }
          }
        }
      }
      next_line = k;

      // event choice: line, else electron, else boundary
      const bool escat = !line_hit && d_electron < d_shell;
      const bool cross = !line_hit && !escat;
      const double d = line_hit ? d_line : (escat ? d_electron : d_shell);

      // J and nu-bar estimators (section 2.7), register-accumulated per shell
      if (acc_shell != sh || acc_model != model) {
        if (acc_shell >= 0) {
          const DevModel& am = ENTRY(a, acc_model).m;
          unsafeAtomicAdd(&am.raw[acc_shell], acc_J);
          unsafeAtomicAdd(&am.raw[am.S + acc_shell], acc_nb);
        }
        acc_shell = sh;
        acc_model = model;
        acc_J = 0.0;
        acc_nb = 0.0;
      }
      const double jc = e_cmf * d * D;
      acc_J += jc;
      acc_nb += jc * nu_cmf;

      // move along the flight path
      const double r_new = root_pos(r * r + d * d + 2.0 * r * d * mu);
      double mu_new = quot(rmu + d, divisor(r_new));
      mu_new = mu_new > 1.0 ? 1.0 : (mu_new < -1.0 ? -1.0 : mu_new);

      if (cross) {
        const int kind = inward ? EV_SHELL_IN : EV_SHELL_OUT;
        r = inward ? c_rin : c_rout;
        mu = mu_new;
        if (v.records) hash = fnv_event(hash, kind, sh, -1, -1);
        shell = sh + (inward ? -1 : 1);
        if (shell >= v.S)
          status = SMC_ESCAPED;
        else if (shell < 0)
          status = SMC_REABSORBED;
      } else {
        // Thomson (coherent, isotropic in the comoving frame) or line
        // interaction (branch draw, then direction; section 2.5)
        const double D_old = 1.0 - quot(mu_new * r_new, v.rct);
        const double e_cmf_ev = E * D_old;
        double nu_cmf_out = nu * D_old;
        int32_t emit = k;
        if (line_hit) {
          const double u_branch = rng_next(g);
          nu_cmf_out = nu_hit;
          if (v.downbranch) {
            const int32_t up = v.line_upper[k];
            const int64_t j = row_select(v.em_cum, v.level_ptr[up], v.level_ptr[up + 1], u_branch);
            emit = v.em_line[j];
            nu_cmf_out = v.line_nu[emit];
          } else if (v.macroatom) {
            // internal jumps until deactivation, one draw per step from this
            // shell's rows (section 2.5)
            const double* cum = v.em_cum + (size_t)sh * (size_t)v.n_em;
            int32_t level = v.line_upper[k];
            double u = u_branch;
            uint32_t steps = 0;
            emit = -1;
            for (;;) {
              const int64_t j = row_select(cum, v.level_ptr[level], v.level_ptr[level + 1], u);
              const int32_t target = v.em_line[j];
              if (target >= 0) {
                emit = target;
                break;
              }
              level = -target - 1;
              if (++steps >= kMacroMaxSteps) break;
              rng_topup(g, 2, sk);  // this step's draw and the direction draw
              u = rng_next(g);
            }
            if (emit >= 0) nu_cmf_out = v.line_nu[emit];
          }
        }
        if (emit < 0) {
          // a macro atom that never deactivated: the packet ends here
          r = r_new;
          mu = mu_new;
          status = SMC_CAPPED;
          dead_atom = true;
        } else {
          const double mu_out = 2.0 * rng_next(g) - 1.0;
          const Divisor rD = divisor(1.0 - quot(mu_out * r_new, v.rct));
          r = r_new;
          mu = mu_out;
          nu = quot(nu_cmf_out, rD);
          E = quot(e_cmf_ev, rD);
          if (line_hit) {
            next_line = emit + 1;
            n_line += 1;
            last_line = k;
            if (v.records) hash = fnv_event(hash, EV_LINE, sh, k, emit);
          } else {
            n_esc += 1;
            if (v.records) hash = fnv_event(hash, EV_ESCATTER, sh, -1, -1);
          }
        }
      }
    }

    if (status != SMC_LIVE) {
      const DevModel& m = ENTRY(a, model).m;
      lane_tally_end(m, tly, status, nu, E, n_seg, n_pass, n_line, n_esc, dead_atom);
      if (m.packets != nullptr && (ENTRY(a, model).it.flags & SMC_F_PACKETS))
        write_record(m, slot, pid, status, shell, nu, E, mu, r, mu0, nu_cmf0, n_seg, n_esc,
                     n_line, n_pass, hash, last_line);
      active = false;
    }
  }

  if (acc_shell >= 0) {
    const DevModel& am = ENTRY(a, acc_model).m;
    unsafeAtomicAdd(&am.raw[acc_shell], acc_J);
    unsafeAtomicAdd(&am.raw[am.S + acc_shell], acc_nb);
  }
  flush_window_jblue(jblue_row(wshell));
  if (tally_model >= 0) lane_tally_flush(ENTRY(a, tally_model).m, tly);
}

// ---------------------------------------------------------------------------
// hand-off numbering over the models of a multi-model launch
// ---------------------------------------------------------------------------
__global__ void long_prefix_kernel(LaunchArgs a, BatchEntry* table) {
  if (threadIdx.x != 0) return;
  unsigned long long total = 0;
  for (int k = 0; k < a.n_models; ++k) {
    table[k].long_begin = total;
    unsigned long long n = table[k].m.counters[CTR_LONG_COUNT];
    if (n > table[k].m.long_cap) n = table[k].m.long_cap;
    total += n;
  }
  a.ctr[1] = total;
  a.ctr[2] = 0ull;
}

// ---------------------------------------------------------------------------
// processing order of the handed-off histories: a counting sort into
// kOrderBuckets buckets of the key below, largest first.  Launch-wide position
// q of the order lives in the long_order array of the model whose hand-off
// range [long_begin, long_begin + count) holds q.
// ---------------------------------------------------------------------------
template <bool kMulti>
__device__ __forceinline__ uint64_t long_total(const LaunchArgs& a) {
  if (kMulti) return a.ctr[1];
  const uint64_t n = a.single.m.counters[CTR_LONG_COUNT];
  return n > a.single.m.long_cap ? a.single.m.long_cap : n;
}

// model whose hand-off range holds launch-wide index q
template <bool kMulti>
__device__ __forceinline__ int long_owner(const LaunchArgs& a, uint64_t q) {
  if (!kMulti) return 0;
  int lo = 0, hi = a.n_models - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.table[mid].long_begin <= q)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Processing order of the handed-off histories: the larger the product of
// (a) the fraction of the line list still to the red and (b) 0.1 plus the
// distance from the inner boundary as a fraction of the ejecta's depth, the
// earlier.  Lines to the red bound the work left; a history close to the
// inner boundary is likely to be reabsorbed soon, one far from it has to
// diffuse through the line forest first.  On the paper-scale model at its
// converged inner temperature the radius ranks the remaining length far
// better than the lines alone (rank correlation 0.75 against 0.41), and the
// longest histories start with the first wave of the group kernel.  The 0.1
// keeps the lines' order among histories handed over at the inner boundary
// (all of them, with v-packets).
template <bool kMulti>
__device__ __forceinline__ int bucket_of_long(const LaunchArgs& a, uint64_t q) {
  const int k = long_owner<kMulti>(a, q);
  const DevModel& m = ENTRY(a, k).m;
  const LongState& st = m.longs[q - ENTRY(a, k).long_begin];
  const double r0 = m.r_bounds[0], r1 = m.r_bounds[m.S];
  double x = (st.r - r0) / (r1 - r0);
  x = x < 0.0 ? 0.0 : (x > 1.0 ? 1.0 : x);
  const double f = (double)(m.L - st.next_line) / ((double)a.max_lines + 1.0);
  const int b = (int)((x + 0.1) / 1.1 * f * (double)kOrderBuckets);
  return b >= kOrderBuckets ? kOrderBuckets - 1 : (b < 0 ? 0 : b);
}

template <bool kMulti>
__global__ void order_count_kernel(LaunchArgs a) {
  const uint64_t n = long_total<kMulti>(a);
  for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
       q += (uint64_t)gridDim.x * blockDim.x)
    atomicAdd(&a.order_hist[bucket_of_long<kMulti>(a, q)], 1u);
}

// cursor[b] = histories in buckets above b (one workgroup of kOrderBuckets)
__global__ __launch_bounds__(kOrderBuckets) void order_scan_kernel(LaunchArgs a) {
  __shared__ unsigned int buf[kOrderBuckets];
  const int t = threadIdx.x;
  const int b = kOrderBuckets - 1 - t;  // thread t takes bucket b, from the top down
  const unsigned int c = a.order_hist[b];
  buf[t] = c;
  __syncthreads();
  for (int off = 1; off < kOrderBuckets; off <<= 1) {
    const unsigned int add = t >= off ? buf[t - off] : 0u;
    __syncthreads();
    buf[t] += add;
    __syncthreads();
  }
  a.order_hist[kOrderBuckets + b] = buf[t] - c;
}

template <bool kMulti>
__global__ void order_place_kernel(LaunchArgs a) {
  const uint64_t n = long_total<kMulti>(a);
  for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
       q += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t pos =
        atomicAdd(&a.order_hist[kOrderBuckets + bucket_of_long<kMulti>(a, q)], 1u);
    const int j = long_owner<kMulti>(a, pos);
    ENTRY(a, j).m.long_order[pos - ENTRY(a, j).long_begin] = q;
  }
}

// ---------------------------------------------------------------------------
// group-per-packet kernel for the handed-off histories
// ---------------------------------------------------------------------------
__device__ __forceinline__ double readlane_f64(double x, int src) {
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, src);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), src);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// x moved by a DPP row shift (both 32-bit halves); a lane whose source lies
// outside its row of 16 reads 0
template <int kCtrl>
__device__ __forceinline__ double dpp_shr_f64(double x) {
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)b, kCtrl, 0xF, 0xF, true);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), kCtrl, 0xF, 0xF,
                                                         true);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// x moved by DPP (both 32-bit halves); lanes the control does not write keep 0
template <int kCtrl, int kRowMask>
__device__ __forceinline__ double dpp_f64(double x) {
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, kCtrl, kRowMask,
                                                            0xF, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(
      0, (int)(uint32_t)(b >> 32), kCtrl, kRowMask, 0xF, false);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// x of the next lower wave lane (DPP wave_shr:1); lane 0 reads 0
__device__ __forceinline__ double wave_shr1_f64(double x) {
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)b, 0x138, 0xF, 0xF, true);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), 0x138, 0xF, 0xF,
                                                         true);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ __forceinline__ double join_u32(uint32_t lo, uint32_t hi) {
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Copy one double per active lane from HBM to LDS without passing through
// registers: the two words land at lo[lane] and hi[lane] (lane = wave lane).
// The wavefront waits for the copy only where it reads the LDS words.
__device__ __forceinline__ void copy_f64_to_lds(const double* src, uint32_t* lo, uint32_t* hi) {
  typedef __attribute__((address_space(1))) void* global_ptr;
  typedef __attribute__((address_space(3))) void* lds_ptr;
  const uint32_t* w = reinterpret_cast<const uint32_t*>(src);
  __builtin_amdgcn_global_load_lds((global_ptr)(w), (lds_ptr)lo, 4, 0, 0);
  __builtin_amdgcn_global_load_lds((global_ptr)(w + 1), (lds_ptr)hi, 4, 0, 0);
}

// Lane groups of G = 16, 32 or 64 lanes (aligned, one packet each).  Values
// that are uniform over a group live in every lane of it; with G = 64 they
// are wave-uniform and the compiler keeps the integer ones in scalar
// registers.
template <int G>
struct Group {
  static constexpr unsigned long long kMask = G == 64 ? ~0ull : ((1ull << G) - 1ull);
  int lane, base;  // lane within the group, first wave lane of the group

  // a group-uniform integer (scalar register when G = 64)
  __device__ __forceinline__ int uni(int x) const {
    if constexpr (G == 64) return __builtin_amdgcn_readfirstlane(x);
    return x;
  }
  // lane `src` (group-uniform) of the group's copy of x
  __device__ __forceinline__ double bcast(double x, int src) const {
    if constexpr (G == 64) return readlane_f64(x, src);
    return __shfl(x, base + src, kWave);
  }
  __device__ __forceinline__ unsigned long long bcast_u64(unsigned long long x, int src) const {
    if constexpr (G == 64) {
      const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, src);
      const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), src);
      return ((unsigned long long)hi << 32) | lo;
    }
    return __shfl(x, base + src, kWave);
  }
  // this group's bits of a wave ballot
  __device__ __forceinline__ unsigned long long bits(unsigned long long w) const {
    if constexpr (G == 64) return w;
    return (w >> base) & kMask;
  }
  // the entry of transition row [lo, hi) (group-uniform bounds) a uniform
  // draw u selects: the first j in [lo, hi - 1) with cum[j] > u, else the
  // last entry (section 2.5); G entries per round, one coalesced load and a
  // ballot each
  __device__ __forceinline__ int64_t row_select(const double* cum, int64_t lo, int64_t hi,
                                                double u) const {
    for (int64_t b = lo; b < hi - 1; b += G) {
      const int64_t j = b + lane;
      const unsigned long long above = bits(__ballot(j < hi - 1 && cum[j] > u));
      if (above) return b + (int64_t)__builtin_ctzll(above);
    }
    return hi - 1;
  }
  // inclusive prefix sum over the group (row shifts within rows of 16 lanes,
  // then the row broadcasts of lanes 15 and 31)
  __device__ __forceinline__ double prefix_sum(double x) const {
    x += dpp_shr_f64<0x111>(x);  // row_shr:1
    x += dpp_shr_f64<0x112>(x);  // row_shr:2
    x += dpp_shr_f64<0x114>(x);  // row_shr:4
    x += dpp_shr_f64<0x118>(x);  // row_shr:8
    if constexpr (G >= 32) x += dpp_f64<0x142, 0xA>(x);  // row_bcast:15 into rows 1 and 3
    if constexpr (G == 64) x += dpp_f64<0x143, 0xC>(x);  // row_bcast:31 into rows 2 and 3
    return x;
  }
};

// ---------------------------------------------------------------------------
// virtual packets (section 2.9), run by a group for its history's launches
// ---------------------------------------------------------------------------

// Follow one v-packet from (r, mu) in `shell`, lines from index k on, along
// its straight path to the outer boundary; tau_v is the Sobolev depth of
// every resonance reached before each shell boundary plus the Thomson depth
// of every shell piece, with the quantities of each piece taken at its start
// as for the packets themselves.  The group tests G lines per step: the
// reached lines of a window form a prefix (d_line grows along the list), a
// prefix sum over the group gives their running depth.  Returns true with
// tau when the v-packet leaves the outer boundary with tau <= kTauVirtualMax;
// `passes` counts the resonances swept (up to the one that passes the cut).
template <int G>
__device__ bool virtual_path(const Group<G>& grp, const View& v, double r, double mu, int shell,
                             int32_t k, double nu_lab, double& tau_out, uint64_t& passes) {
  const double ct_over_nu = quot(v.ct, divisor(nu_lab));
  double tau = 0.0;
  for (;;) {
    const double r_in = v.r_bounds[shell], r_out = v.r_bounds[shell + 1];
    const double ne = v.n_e[shell];
    const double rmu = r * mu;
    const double D = 1.0 - quot(mu * r, v.rct);
    const double nu_cmf = nu_lab * D;
    bool inward;
    const double d_shell = shell_distance(r, mu, rmu, r_in, r_out, inward);
    const double kappa = kSigmaT * ne * D;
    const size_t row = (size_t)shell * (size_t)v.Lp;
    while (k < v.L) {
      const int32_t line = k + grp.lane;
      const bool in = line < v.L;
      const int32_t lc = in ? line : v.L - 1;
      const double nk = v.line_nu[lc];
      const double tk = v.tau[row + lc];
      double dl = (nu_cmf - nk) * ct_over_nu;
      dl = dl < 0.0 ? 0.0 : dl;
      const bool reach = in && dl < d_shell;
      const int n_reach = __popcll(grp.bits(__ballot(reach)));
      const double cum = grp.prefix_sum(reach ? tk : 0.0);
      const unsigned long long over =
          grp.bits(__ballot(reach && tau + cum > kTauVirtualMax));
      if (over) {
        passes += (uint64_t)(__builtin_ctzll(over) + 1);
        return false;
      }
      passes += (uint64_t)n_reach;
      if (n_reach > 0) tau += grp.bcast(cum, grp.uni(n_reach - 1));
      k += n_reach;
      if (n_reach < G) break;
    }
    tau += kappa * d_shell;
    if (tau > kTauVirtualMax) return false;
    const double r_new = root_pos(r * r + d_shell * d_shell + 2.0 * r * d_shell * mu);
    double mu_new = quot(rmu + d_shell, divisor(r_new));
    mu_new = mu_new > 1.0 ? 1.0 : (mu_new < -1.0 ? -1.0 : mu_new);
    r = inward ? r_in : r_out;
    mu = mu_new;
    shell += inward ? -1 : 1;
    if (shell >= v.S) {
      tau_out = tau;
      return true;
    }
    if (shell < 0) return false;  // only a ray grazing the inner boundary by rounding
  }
}

// The N_v v-packets of one packet launch (injection, e = 0, or the e-th
// interaction): the launching packet's position, comoving frequency, energy
// and next redward line; directions uniform in (mu_min, 1) from the packet's
// second stream (draw e * N_v + j, key word 0 xor 0x56504B54); comoving
// weights 2 mu_v / N_v at injection, (1 - mu_min) / (2 N_v) otherwise; lab
// energy E_v / D and frequency nu_cmf / D into the v-packet spectrum.
template <int G>
__device__ void launch_virtual(const Group<G>& grp, const View& v, const DevModel& m,
                               const StreamKey& sk, uint64_t e, bool injection, double r,
                               int shell, int32_t k, double nu_cmf, double e_cmf,
                               LaneTally& tly, bool leader) {
  const uint32_t nv = v.n_virtual;
  StreamKey vk = sk;
  vk.k0 ^= 0x56504B54u;
  // group lane j < N_v holds draw e * N_v + j
  const uint64_t dv = e * (uint64_t)nv + (uint64_t)(grp.lane < (int)nv ? grp.lane : 0);
  const Block b = stream_block(vk, (uint32_t)(dv >> 1));
  const double u_lane = to_uniform((dv & 1) ? b.b : b.a);
  // a true division: at injection r = r_inner gives exactly mu_min = 0
  const double x = v.r_bounds[0] / r;
  double q = 1.0 - x * x;
  q = q < 0.0 ? 0.0 : q;
  const double mu_min = -sqrt(q);
  uint64_t passes = 0, counted = 0;
  for (uint32_t j = 0; j < nv; ++j) {
    const double u = grp.bcast(u_lane, grp.uni((int)j));
    const double mu_v = mu_min + (1.0 - mu_min) * u;
    const double w = injection ? 2.0 * mu_v / (double)nv : (1.0 - mu_min) / (2.0 * (double)nv);
    const Divisor rD = divisor(1.0 - quot(mu_v * r, v.rct));
    const double nu_lab = quot(nu_cmf, rD);
    double tau = 0.0;
    if (virtual_path(grp, v, r, mu_v, shell, k, nu_lab, tau, passes)) {
      counted += 1;
      if (leader) unsafeAtomicAdd(&m.vraw[spectrum_bin(m, nu_lab)], quot(e_cmf * w, rD) * exp(-tau));
    }
  }
  if (leader) {
    tly.vc[0] += nv;
    tly.vc[1] += counted;
    tly.vc[2] += passes;
  }
}

constexpr int kLongBlock = 64;

// One handed-off history per group of G lanes, 64/G histories per wavefront.
// The group holds the next 2G draws of its packet's stream with their
// logarithms precomputed, and the next G lines of its shell; a segment tests
// all G lines at once (each lane against the optical depth left after the
// live lines below it), and J_blue updates leave from every reached lane
// together.  A group whose packet ends takes the next one from the hand-off
// queue while the other groups of its wavefront keep marching.
template <bool kMulti, int G, bool kExt>
__device__ __forceinline__ void long_body(const LaunchArgs& a) {
  constexpr int kGroups = kWave / G;
  __shared__ LaneTally tly_all[kGroups];  // one tally slot per group, its lane 0 writes it
  // next window of each group, copied ahead straight from HBM: low and high
  // words of the line frequencies, then of the Sobolev depths, by wave lane
  __shared__ uint32_t pf[4][kWave];
  // each group's draws 2 rb .. 2 rb + 2G - 1 in draw order: uniforms and
  // their -log, at 2 x (the group's first wave lane)
  __shared__ double dr_u[2 * kWave], dr_l[2 * kWave];
  // lane masks of a group's window
  using Mask = typename std::conditional<G == 64, unsigned long long, uint32_t>::type;
  constexpr Mask kFull = G == 64 ? (Mask)~0ull : (Mask)((1ull << G) - 1ull);
  Group<G> grp;
  grp.lane = threadIdx.x & (G - 1);
  grp.base = threadIdx.x & ~(G - 1);
  const bool leader = grp.lane == 0;
  LaneTally& tly = tly_all[threadIdx.x / G];
  const unsigned long long n_long = long_total<kMulti>(a);
  unsigned long long* queue = kMulti ? a.ctr + 2 : a.single.m.counters + CTR_LONG_QUEUE;
  if (leader) lane_tally_clear(tly);
  int tally_model = kMulti ? -1 : 0;
  double acc_J = 0.0, acc_nb = 0.0;
  int acc_shell = -1, acc_model = -1;

  // the group's current history
  bool have = false, drained = false;
  int model = 0, tier = 0;
  View v;
  StreamKey sk;
  uint64_t slot = 0, pid = 0, n_seg = 0, n_pass = 0, hash = 0;
  double mu0 = 0.0, nu_cmf0 = 0.0;
  uint32_t draw = 0, rb = 0, n_esc = 0, n_line = 0;
  double r = 0.0, mu = 0.0, nu = 0.0, E = 0.0;
  int32_t shell = 0, next_line = 0, last_line = -1;
  // line wbase + i of shell wshell in group lane i: frequency, depth, the
  // summed depth of the window's lines before it, and the J_blue the history
  // has left on it since the window was installed (the following window of
  // the same shell waits in pf); wx_at = wx of line wx_k
  int32_t wbase = -1, wshell = -1, wx_k = -1;
  double wn = 0.0, wt = 0.0, wx = 0.0, jb_acc = 0.0, wx_at = 0.0;
  Mask wlive = 0;  // lanes of the window that hold a line
  int32_t c_shell = -1;
  double c_rin = 0.0, c_rout = 0.0, c_ne = 0.0;

  // move the group's window of 2G draws to start at the next one (draws
  // 2(rb + i) and 2(rb + i) + 1 from group lane i's counter block)
  auto refill_draws = [&]() {
    rb = draw >> 1;
    const Block blk = stream_block(sk, rb + grp.lane);
    const double ua = to_uniform(blk.a), ub = to_uniform(blk.b);
    const int o = 2 * (int)threadIdx.x;
    dr_u[o] = ua;
    dr_u[o + 1] = ub;
    dr_l[o] = -log(ua);
    dr_l[o + 1] = -log(ub);
    __builtin_amdgcn_wave_barrier();
  };
  // draw d (2 rb <= d < 2 rb + 2G) of the group's history
  auto draw_u = [&](uint32_t d) { return dr_u[2 * grp.base + (int)(d - 2u * rb)]; };
  auto draw_l = [&](uint32_t d) { return dr_l[2 * grp.base + (int)(d - 2u * rb)]; };

  for (;;) {
    bool fetched = false;
    if (!have && !drained) {
      unsigned long long pos = 0;
      if (leader) pos = atomicAdd(queue, 1ull);
      pos = grp.bcast_u64(pos, 0);
      fetched = true;
      if (pos >= n_long) {
        drained = true;
      } else {
        // position -> hand-off index -> model and slot in its buffer
        const int jo = grp.uni(long_owner<kMulti>(a, pos));
        const uint64_t gidx = ENTRY(a, jo).m.long_order[pos - ENTRY(a, jo).long_begin];
        model = grp.uni(long_owner<kMulti>(a, gidx));
        const uint64_t idx = gidx - ENTRY(a, model).long_begin;
        tier = pos < a.hot ? 3 : (pos < 3ull * a.hot ? 2 : (pos < 7ull * a.hot ? 1 : 0));
        if (kMulti && tally_model != model) {
          if (tally_model >= 0 && leader) lane_tally_flush(a.table[tally_model].m, tly);
          tally_model = model;
        }
        v = make_view(ENTRY(a, model).m, ENTRY(a, model).it);
        const LongState st = ENTRY(a, model).m.longs[idx];
        slot = st.slot;
        pid = st.pid;
        mu0 = st.mu0;
        nu_cmf0 = st.nu_cmf0;
        n_seg = st.n_seg;
        n_pass = st.n_pass;
        hash = st.hash;
        draw = (uint32_t)st.draw;
        r = st.r;
        mu = st.mu;
        nu = st.nu;
        E = st.E;
        shell = st.shell;
        next_line = st.next_line;
        last_line = st.last_line;
        n_esc = st.n_esc;
        n_line = st.n_line;
        sk.k0 = v.k0;
        sk.k1 = v.k1;
        sk.iter = v.iter;
        sk.p0 = (uint32_t)pid;
        sk.p1 = (uint32_t)(pid >> 32);
        refill_draws();
        wbase = -1;
        wshell = -1;
        c_shell = -1;
        have = true;
        if (kExt && v.n_virtual && st.n_seg == 0)
          launch_virtual(grp, v, ENTRY(a, model).m, sk, 0, true, r, 0, next_line, nu_cmf0,
                         v.e_unit, tly, leader);
        // wait for the history's loads here, once per history, so that the
        // segment loop never inherits a pending load (and with it a wait for
        // the copies and atomics it issues itself)
        settle(slot, pid, mu0, nu_cmf0, n_seg, n_pass, hash, draw, r, mu, nu, E, shell,
               next_line, last_line, n_esc, n_line);
        settle(v.r_bounds, v.n_e, v.line_nu, v.tau, v.jblue, v.line_upper, v.level_ptr,
               v.em_line, v.em_cum, v.ct, v.rct.y, v.max_segments, v.S, v.L, v.Lp,
               (int)v.downbranch, (int)v.macroatom, (int)v.records, sk.k0, sk.k1, sk.iter);
      }
    }
    if (__ballot(have) == 0ull) break;  // every group drained
    if (__ballot(fetched)) {
      // the wavefront issues at the priority of its most urgent history
      if (__ballot(have && tier == 3))
        __builtin_amdgcn_s_setprio(3);
      else if (__ballot(have && tier == 2))
        __builtin_amdgcn_s_setprio(2);
      else if (__ballot(have && tier == 1))
        __builtin_amdgcn_s_setprio(1);
      else
        __builtin_amdgcn_s_setprio(0);
    }
    if (!have) continue;

    // ---- one flight segment of the group's history
    int status = SMC_LIVE;
    bool dead_atom = false;  // the history ended in a macro atom that never deactivated
    do {
      if (n_seg >= v.max_segments) {
        status = SMC_CAPPED;
        break;
      }
      n_seg += 1;
      if (draw + 3 > 2u * (rb + G)) refill_draws();
      const double tau0 = draw_l(draw);
      draw += 1;
      const int sh = shell;
      if (sh != c_shell) {
        c_shell = sh;
        c_rin = v.r_bounds[sh];
        c_rout = v.r_bounds[sh + 1];
        c_ne = v.n_e[sh];
        // wait for these loads here, on the rare shell change, so that the
        // segment code after the branch has nothing in flight to wait for
        asm volatile("" ::"v"(c_rin), "v"(c_rout), "v"(c_ne));
      }
      const double rmu = r * mu;
      const double D = 1.0 - quot(mu * r, v.rct);
      const double nu_cmf = nu * D;
      const double e_cmf = E * D;
      bool inward;
      const double d_shell = shell_distance(r, mu, rmu, c_rin, c_rout, inward);
      const double kappa = kSigmaT * c_ne * D;
      const Divisor rkappa = divisor(kappa);
      const Divisor rnu = divisor(nu);
      const double ct_over_nu = quot(v.ct, rnu);
      // J_blue weight per unit line frequency, E / nu^2: a lane sums it over
      // its line's passages and multiplies by nu_k when the window changes
      const double jb_f = E * rnu.y * rnu.y;
      const bool jb_row = v.jblue != nullptr;

      // line march over the window: lane j tests line wbase+j against the
      // optical depth left after the live lines before it, tau - (X_j - X_k)
      // with X the window's summed depths and k the first live line; the
      // first lane that stops the march decides
      double tau_ev = tau0;  // left after the windows already passed
      int32_t k = next_line;
      bool line_hit = false;
      double d_line = 0.0, nu_hit = 0.0, tau_rem = tau0;
      while (k < v.L) {
        if (sh != wshell || k < wbase || k >= wbase + G) {
          // The following window of the same shell was copied ahead from
          // HBM into LDS by the direct global-to-LDS load; anything else (a
          // new shell, a jump after a downbranch emission) is loaded now.
          // Nothing outside this block waits for those copies, and the old
          // window's J_blue leaves in one atomic per lane.
          const bool ahead = sh == wshell && k == wbase + G;
          const int32_t line = k + grp.lane;
          const bool in = line < v.L;
          const size_t row = (size_t)sh * (size_t)v.Lp;
          const double jb_out = jb_acc * wn;
          if (ahead) {
            const double n_raw = join_u32(pf[0][threadIdx.x], pf[1][threadIdx.x]);
            const double t_raw = join_u32(pf[2][threadIdx.x], pf[3][threadIdx.x]);
            wn = in ? n_raw : 1.0;
            wt = in ? t_raw : 0.0;
          } else {
            const int32_t lc = line < v.Lp ? line : v.Lp - 1;
            const double n_raw = v.line_nu[lc];
            const double t_raw = v.tau[row + lc];
            wn = in ? n_raw : 1.0;
            wt = in ? t_raw : 0.0;
          }
          // the window is in registers (and its LDS copy free for reuse)
          // before the next copy and the atomic are issued
          asm volatile("s_waitcnt lgkmcnt(0)" ::"v"(wn), "v"(wt) : "memory");
          const int32_t next = k + G + grp.lane;
          const int32_t nc = next < v.Lp ? next : v.Lp - 1;
          copy_f64_to_lds(v.line_nu + nc, &pf[0][0], &pf[1][0]);
          copy_f64_to_lds(v.tau + row + nc, &pf[2][0], &pf[3][0]);
          if (v.jblue && wshell >= 0 && jb_out != 0.0)
            unsafeAtomicAdd(&v.jblue[(size_t)wshell * (size_t)v.L + wbase + grp.lane], jb_out);
          jb_acc = 0.0;
          wbase = k;
          wshell = sh;
          // summed depth of the group's lanes below each lane
          const double incl = grp.prefix_sum(wt);
          const double below = wave_shr1_f64(incl);
          wx = grp.lane == 0 ? 0.0 : below;
          wx_k = k;
          wx_at = 0.0;
          const int32_t n_in = v.L - k;
          wlive = n_in >= G ? kFull : (Mask)(((Mask)1 << n_in) - 1);
        }
        if (wx_k != k) {
          wx_at = grp.bcast(wx, k - wbase);
          wx_k = k;
        }
        // live lanes: lines k .. L - 1 of the window
        const Mask live = wlive & (Mask)(kFull << (k - wbase));
        const double dl = fmax((nu_cmf - wn) * ct_over_nu, 0.0);
        const double rem = tau_ev - (wx - wx_at);  // tau itself at line k
        const double de = kappa > 0.0 ? quot_checked(rem, rkappa) : INFINITY;
        // lanes whose line lies beyond the Thomson event or the boundary, and
        // lanes whose line would absorb if reached
        const Mask far = (Mask)grp.bits(__ballot(dl >= de)) | (Mask)grp.bits(__ballot(dl >= d_shell));
        const Mask deep = (Mask)grp.bits(__ballot(wt + kappa * dl > rem));
        const Mask stop = (far | deep) & live;
        // the first stopping lane (none: 0), and whether its line absorbs
        const Mask low = stop & (Mask)(0 - stop);
        const Mask hit_low = low & deep & (Mask)~far;
        // J_blue: every line reached up to the stop, the interacting one included
        const Mask reached = live & ((Mask)(low - 1) | hit_low);
        if (jb_row && ((reached >> grp.lane) & 1)) jb_acc += jb_f;
        n_pass += (uint64_t)(G == 64 ? __builtin_popcountll((unsigned long long)reached)
                                     : __builtin_popcount((uint32_t)reached));
        if (low) {
          const int fl = grp.uni(G == 64 ? __builtin_ctzll((unsigned long long)low)
                                         : __builtin_ctz((uint32_t)low));
          k = wbase + fl;
          if (hit_low) {
            line_hit = true;
            d_line = grp.bcast(dl, fl);
            nu_hit = grp.bcast(wn, fl);
          } else {
            tau_rem = grp.bcast(rem, fl);
          }
          break;
        }
        // every live line of the window passed
        const int top = grp.uni(G == 64 ? 63 - __builtin_clzll((unsigned long long)wlive)
                                        : 31 - __builtin_clz((uint32_t)wlive));
        tau_ev -= grp.bcast(wx + wt, top) - wx_at;
        tau_rem = tau_ev;
        k = wbase + top + 1;
      }
      next_line = k;
      // the next march in this shell starts at the line after the
      // interacting one (scatter mode) or here after a Thomson event: fetch
      // its summed depth while this event's transforms run
      {
        const int32_t kn = line_hit ? k + 1 : k;
        if (wshell == sh && kn >= wbase && kn < wbase + G) {
          wx_at = grp.bcast(wx, kn - wbase);
          wx_k = kn;
        }
      }

      const double d_electron =
          (!line_hit && kappa > 0.0) ? quot_checked(tau_rem, rkappa) : INFINITY;
      const bool escat = !line_hit && d_electron < d_shell;
      const bool cross = !line_hit && !escat;
      const double d = line_hit ? d_line : (escat ? d_electron : d_shell);

      if (acc_shell != sh || acc_model != model) {
        if (acc_shell >= 0 && leader) {
          const DevModel& am = ENTRY(a, acc_model).m;
          unsafeAtomicAdd(&am.raw[acc_shell], acc_J);
          unsafeAtomicAdd(&am.raw[am.S + acc_shell], acc_nb);
        }
        acc_shell = sh;
        acc_model = model;
        acc_J = 0.0;
        acc_nb = 0.0;
      }
      const double jc = e_cmf * d * D;
      acc_J += jc;
      acc_nb += jc * nu_cmf;

      const double r_new = root_pos(r * r + d * d + 2.0 * r * d * mu);
      const double mu_new = fmin(fmax(quot(rmu + d, divisor(r_new)), -1.0), 1.0);
      if (cross) {
        const int kind = inward ? EV_SHELL_IN : EV_SHELL_OUT;
        r = inward ? c_rin : c_rout;
        mu = mu_new;
        if (v.records) hash = fnv_event(hash, kind, sh, -1, -1);
        shell = sh + (inward ? -1 : 1);
        if (shell >= v.S) status = SMC_ESCAPED;
        if (shell < 0) status = SMC_REABSORBED;
      } else {
        const double D_old = 1.0 - quot(mu_new * r_new, v.rct);
        const double e_cmf_ev = E * D_old;
        double nu_cmf_out;
        int32_t emit = k;
        if (line_hit) {
          const double u_branch = draw_u(draw);
          draw += 1;
          nu_cmf_out = nu_hit;
          if (v.downbranch) {
            const int32_t up = v.line_upper[k];
            const int64_t j =
                grp.row_select(v.em_cum, v.level_ptr[up], v.level_ptr[up + 1], u_branch);
            emit = v.em_line[j];
            nu_cmf_out = v.line_nu[emit];
          } else if (kExt && v.macroatom) {
            // internal jumps until deactivation, one draw per step from this
            // shell's rows (section 2.5)
            const double* cum = v.em_cum + (size_t)sh * (size_t)v.n_em;
            int32_t level = v.line_upper[k];
            double u = u_branch;
            uint32_t steps = 0;
            emit = -1;
            for (;;) {
              const int64_t j = grp.row_select(cum, v.level_ptr[level], v.level_ptr[level + 1], u);
              const int32_t target = v.em_line[j];
              if (target >= 0) {
                emit = target;
                break;
              }
              level = -target - 1;
              if (++steps >= kMacroMaxSteps) break;
              if (draw + 2 > 2u * (rb + G)) refill_draws();  // this step's and the direction's
              u = draw_u(draw);
              draw += 1;
            }
            if (emit < 0) {
              // a macro atom that never deactivated: the packet ends here
              mu = mu_new;
              r = r_new;
              status = SMC_CAPPED;
              dead_atom = true;
              break;
            }
            nu_cmf_out = v.line_nu[emit];
          }
        } else {
          nu_cmf_out = nu * D_old;
        }
        const double mu_out = 2.0 * draw_u(draw) - 1.0;
        draw += 1;
        const Divisor rD = divisor(1.0 - quot(mu_out * r_new, v.rct));
        r = r_new;
        mu = mu_out;
        nu = quot(nu_cmf_out, rD);
        E = quot(e_cmf_ev, rD);
        if (line_hit) {
          next_line = emit + 1;
          n_line += 1;
          last_line = k;
          if (v.records) hash = fnv_event(hash, EV_LINE, sh, k, emit);
        } else {
          n_esc += 1;
          if (v.records) hash = fnv_event(hash, EV_ESCATTER, sh, -1, -1);
        }
        if (kExt && v.n_virtual)
          launch_virtual(grp, v, ENTRY(a, model).m, sk, (uint64_t)n_esc + n_line, false, r, sh,
                         next_line, nu_cmf_out, e_cmf_ev, tly, leader);
      }
    } while (false);

    if (status != SMC_LIVE) {
      if (v.jblue && wshell >= 0 && jb_acc != 0.0)
        unsafeAtomicAdd(&v.jblue[(size_t)wshell * (size_t)v.L + wbase + grp.lane], jb_acc * wn);
      jb_acc = 0.0;
      wshell = -1;
      if (leader) {
        const DevModel& m = ENTRY(a, model).m;
        lane_tally_end(m, tly, status, nu, E, n_seg, n_pass, n_line, n_esc, dead_atom);
        if (v.records)
          write_record(m, slot, pid, status, shell, nu, E, mu, r, mu0, nu_cmf0, n_seg, n_esc,
                       n_line, n_pass, hash, last_line);
      }
      have = false;
    }
  }
  if (leader) {
    if (acc_shell >= 0) {
      const DevModel& am = ENTRY(a, acc_model).m;
      unsafeAtomicAdd(&am.raw[acc_shell], acc_J);
      unsafeAtomicAdd(&am.raw[am.S + acc_shell], acc_nb);
    }
    if (tally_model >= 0) lane_tally_flush(ENTRY(a, tally_model).m, tly);
  }
}

// ---------------------------------------------------------------------------
// wavefront-per-history kernel for the handed-off histories of the plain
// line modes (scatter, downbranch) without v-packets
// ---------------------------------------------------------------------------
// A history's segments form one dependent chain (where one segment ends sets
// up the next), so the time of one segment in one wavefront bounds the pass
// once few histories are left.  Here every per-history value is uniform over
// the wavefront: its integers live in scalar registers, its branches are
// scalar, and a value held by one lane (a draw, the distance to the
// interacting line) reaches the others by a lane read.  The 64 lanes test the
// next 64 lines of the shell at once.  The common segment, a line event
// inside the current window of lines, runs straight through the inner loop;
// window and shell changes, draw refills, a march across several windows and
// the downbranch emission sit in branches off that path.  Arithmetic and
// operand order are those of the group kernel.
template <bool kMulti>
__device__ __forceinline__ void solo_body(const LaunchArgs& a) {
  __shared__ LaneTally tly;
  // next window, copied ahead straight from HBM: low and high words of the
  // line frequencies, then of the Sobolev depths, by lane
  __shared__ uint32_t pf[4][kWave];
  // the history's draws 2 rb .. 2 rb + 127 in draw order: uniforms and their
  // -log (read back at a wave-uniform address, one LDS broadcast each)
  __shared__ double dr_u[2 * kWave], dr_l[2 * kWave];
  const int lane = threadIdx.x;
  const bool leader = lane == 0;
  const unsigned long long n_long = long_total<kMulti>(a);
  unsigned long long* queue = kMulti ? a.ctr + 2 : a.single.m.counters + CTR_LONG_QUEUE;
  if (leader) lane_tally_clear(tly);
  int tally_model = kMulti ? -1 : 0;
  double acc_J = 0.0, acc_nb = 0.0;
  int acc_shell = -1, acc_model = -1;
  const Group<64> grp{lane, 0};

  for (;;) {
    // ---- the next handed-off history, in the processing order
    unsigned long long pos = 0;
    if (leader) pos = atomicAdd(queue, 1ull);
    pos = grp.bcast_u64(pos, 0);
    if (pos >= n_long) break;
    const int jo = grp.uni(long_owner<kMulti>(a, pos));
    const uint64_t gidx = ENTRY(a, jo).m.long_order[pos - ENTRY(a, jo).long_begin];
    const int model = grp.uni(long_owner<kMulti>(a, gidx));
    const uint64_t idx = gidx - ENTRY(a, model).long_begin;
    if (pos < a.hot)
      __builtin_amdgcn_s_setprio(3);
    else if (pos < 3ull * a.hot)
      __builtin_amdgcn_s_setprio(2);
    else if (pos < 7ull * a.hot)
      __builtin_amdgcn_s_setprio(1);
    else
      __builtin_amdgcn_s_setprio(0);
    if (kMulti && tally_model != model) {
      if (tally_model >= 0 && leader) lane_tally_flush(a.table[tally_model].m, tly);
      tally_model = model;
    }
    View v = make_view(ENTRY(a, model).m, ENTRY(a, model).it);
    // values the segment loop rarely reads, and that decide nothing, stay in
    // vector registers, which leaves the scalar ones to the history's
    // counters and line indices
    asm volatile("" : "+v"(v.line_upper), "+v"(v.level_ptr), "+v"(v.em_line), "+v"(v.em_cum));
    const LongState st = ENTRY(a, model).m.longs[idx];
    // the history's integers are wave-uniform: scalar registers
    uint64_t n_seg = grp.bcast_u64(st.n_seg, 0), n_pass = grp.bcast_u64(st.n_pass, 0);
    uint64_t hash = grp.bcast_u64(st.hash, 0);
    uint32_t draw = (uint32_t)grp.uni((int)st.draw), n_esc = (uint32_t)grp.uni((int)st.n_esc);
    uint32_t n_line = (uint32_t)grp.uni((int)st.n_line);
    double r = st.r, mu = st.mu, nu = st.nu, E = st.E;
    int32_t shell = grp.uni(st.shell), next_line = grp.uni(st.next_line);
    int32_t last_line = grp.uni(st.last_line);
    StreamKey sk;
    sk.k0 = v.k0;
    sk.k1 = v.k1;
    sk.iter = v.iter;
    sk.p0 = (uint32_t)st.pid;
    sk.p1 = (uint32_t)(st.pid >> 32);
    asm volatile("" : "+v"(sk.k0), "+v"(sk.k1), "+v"(sk.p0), "+v"(sk.p1), "+v"(sk.iter));
    const bool use_jb = v.jblue != nullptr;
    // draws 2(rb + i) and 2(rb + i) + 1 from lane i's counter block
    uint32_t rb = draw >> 1;
    auto refill_draws = [&]() {
      rb = draw >> 1;
      const Block blk = stream_block(sk, rb + lane);
      const double ua = to_uniform(blk.a), ub = to_uniform(blk.b);
      __syncthreads();  // the last draws read have been used
      dr_u[2 * lane] = ua;
      dr_u[2 * lane + 1] = ub;
      dr_l[2 * lane] = -log(ua);
      dr_l[2 * lane + 1] = -log(ub);
      __syncthreads();
    };
    refill_draws();
    // line wbase + i of shell wshell in lane i: frequency, depth, the summed
    // depth of the window's lines before it, and the J_blue the history has
    // left on it since the window was installed; wx_at = wx of line wx_k
    int32_t wbase = -1, wshell = -1, wx_k = -1;
    double wn = 0.0, wt = 0.0, wx = 0.0, jb_acc = 0.0, wx_at = 0.0;
    unsigned long long wlive = 0ull;  // lanes of the window that hold a line
    // the shell's bounds and sigma_T n_e, and whether its opacity takes the
    // short quotient x / kappa (sigma_T n_e >= 2^-898, D in (1/2, 3/2)); below
    // that the distance to a Thomson event exceeds 2^840 cm, beyond every
    // chord of a shell (radii <= 2^300 cm), exactly as with no electrons
    int32_t c_shell = -1;
    double c_rin = 0.0, c_rout = 0.0, c_rin2 = 0.0, c_rout2 = 0.0, c_sig = 0.0;
    bool c_kfast = true;
    int status = SMC_LIVE;

    // ---- the history's flight segments (section 2.6); segments left before
    // the cap, counted down (a scalar test)
    uint64_t seg_left = v.max_segments > n_seg ? v.max_segments - n_seg : 0ull;
    for (;;) {
      if (seg_left == 0ull) {
        status = SMC_CAPPED;
        break;
      }
      seg_left -= 1;
      // the draws this segment may take: tau_event, then the branch and
      // direction draws of a line event (or the direction of a Thomson one)
      if (draw + 3 > 2u * (rb + kWave)) refill_draws();
      const uint32_t di = draw - 2u * rb;
      const double tau0 = dr_l[di], u1 = dr_u[di + 1], u2 = dr_u[di + 2];
      const int sh = shell;
      if (sh != c_shell) {
        c_shell = sh;
        c_rin = v.r_bounds[sh];
        c_rout = v.r_bounds[sh + 1];
        const double ne = v.n_e[sh];
        // wait for these loads here, on the rare shell change
        asm volatile("" ::"v"(c_rin), "v"(c_rout), "v"(ne));
        c_rin2 = c_rin * c_rin;
        c_rout2 = c_rout * c_rout;
        c_sig = kSigmaT * ne;
        c_kfast = __ballot(c_sig >= 0x1p-898) != 0ull;
      }
      const double rmu = r * mu;
      const double D = 1.0 - quot(mu * r, v.rct);
      const double nu_cmf = nu * D;
      const double e_cmf = E * D;
      bool inward;
      const double d_shell = shell_distance_sq(r, mu, rmu, c_rin2, c_rout2, inward);
      const double kappa = c_sig * D;
      const Divisor rkappa = divisor(kappa);
      // distance to the Thomson event with optical depth x left
      auto elec = [&](double x) { return c_kfast ? quot(x, rkappa) : (double)INFINITY; };
      const Divisor rnu = divisor(nu);
      const double ct_over_nu = quot(v.ct, rnu);
      // J_blue weight per unit line frequency, E / nu^2: a lane sums it over
      // its line's passages and multiplies by nu_k when the window changes
      const double jb_f = E * rnu.y * rnu.y;

      // line march over the window: lane j tests line wbase+j against the
      // optical depth left after the live lines before it, tau - (X_j - X_k)
      // with X the window's summed depths and k the first live line; the
      // first lane that stops the march decides
      double tau_ev = tau0;  // left after the windows already passed
      int32_t k = next_line;
      bool line_hit = false;
      double d_line = 0.0, nu_hit = 0.0, tau_rem = tau0;
      while (k < v.L) {
        if ((sh != wshell) | (k < wbase) | (k >= wbase + kWave)) {
          // The following window of the same shell was copied ahead from
          // HBM into LDS by the direct global-to-LDS load; anything else (a
          // new shell, a jump after a downbranch emission) is loaded now.
          // Nothing outside this block waits for those copies, and the old
          // window's J_blue leaves in one atomic per lane after them.
          const bool ahead = sh == wshell && k == wbase + kWave;
          const int32_t line = k + lane;
          const bool in = line < v.L;
          const size_t row = (size_t)sh * (size_t)v.Lp;
          const double jb_out = jb_acc * wn;
          const int32_t jb_shell = wshell, jb_base = wbase;
          if (ahead) {
            const double n_raw = join_u32(pf[0][lane], pf[1][lane]);
            const double t_raw = join_u32(pf[2][lane], pf[3][lane]);
            wn = in ? n_raw : 1.0;
            wt = in ? t_raw : 0.0;
          } else {
            const int32_t lc = line < v.Lp ? line : v.Lp - 1;
            const double n_raw = v.line_nu[lc];
            const double t_raw = v.tau[row + lc];
            wn = in ? n_raw : 1.0;
            wt = in ? t_raw : 0.0;
          }
          asm volatile("s_waitcnt lgkmcnt(0)" ::"v"(wn), "v"(wt) : "memory");
          const int32_t next = k + kWave + lane;
          const int32_t nc = next < v.Lp ? next : v.Lp - 1;
          copy_f64_to_lds(v.line_nu + nc, &pf[0][0], &pf[1][0]);
          copy_f64_to_lds(v.tau + row + nc, &pf[2][0], &pf[3][0]);
          if (v.jblue && jb_shell >= 0 && jb_out != 0.0)
            unsafeAtomicAdd(&v.jblue[(size_t)jb_shell * (size_t)v.L + jb_base + lane], jb_out);
          jb_acc = 0.0;
          wbase = k;
          wshell = sh;
          // summed depth of the lanes below: the inclusive sum moved up a lane
          wx = wave_shr1_f64(grp.prefix_sum(wt));
          wx_k = k;
          wx_at = 0.0;
          const int32_t n_in = v.L - k;
          wlive = n_in >= kWave ? ~0ull : ((1ull << n_in) - 1ull);
        }
        if (wx_k != k) {
          wx_at = grp.bcast(wx, k - wbase);
          wx_k = k;
        }
        // live lanes: lines k .. L - 1 of the window
        const unsigned long long live = wlive & (~0ull << (k - wbase));
        // (the difference of two finite frequencies is +0 when they are
        // equal, so the clamp at 0 keeps the sign of every zero)
        const double dl = fmax((nu_cmf - wn) * ct_over_nu, 0.0);
        const double rem = tau_ev - (wx - wx_at);  // tau itself at line k
        // lanes whose line lies beyond the Thomson event or the boundary, and
        // lanes whose line would absorb if reached
        const unsigned long long far_e = __ballot(dl >= quot(rem, rkappa));
        const unsigned long long far = (c_kfast ? far_e : 0ull) | __ballot(dl >= d_shell);
        const unsigned long long deep = __ballot(wt + kappa * dl > rem);
        const unsigned long long stop = (far | deep) & live;
        // the first stopping lane (none: 0), and whether its line absorbs
        const unsigned long long low = stop & (0ull - stop);
        const unsigned long long hit_low = low & deep & ~far;
        // J_blue: every line reached up to the stop, the interacting one included
        const unsigned long long reached = live & ((low - 1ull) | hit_low);
        if (use_jb) {
          if (__builtin_amdgcn_inverse_ballot_w64(reached)) jb_acc += jb_f;
        }
        n_pass += (uint64_t)__builtin_popcountll(reached);
        if (low) {
          const int first = (int)__builtin_ctzll(low);
          k = wbase + first;
          if (hit_low) {
            line_hit = true;
            d_line = grp.bcast(dl, first);
            nu_hit = grp.bcast(wn, first);
          } else {
            tau_rem = grp.bcast(rem, first);
          }
          break;
        }
        // every live line of the window passed
        const int top = 63 - (int)__builtin_clzll(wlive);
        tau_ev -= grp.bcast(wx + wt, top) - wx_at;
        tau_rem = tau_ev;
        k = wbase + top + 1;
      }
      next_line = k;

      // the next march in this shell starts at the line after the
      // interacting one (scatter mode) or here after a Thomson event: fetch
      // its summed depth while this event's transforms run
      {
        const int32_t kn = line_hit ? k + 1 : k;
        if ((wshell == sh) & (kn >= wbase) & (kn < wbase + kWave)) {
          wx_at = grp.bcast(wx, kn - wbase);
          wx_k = kn;
        }
      }
      if (acc_shell != sh || acc_model != model) {
        if (acc_shell >= 0 && leader) {
          const DevModel& am = ENTRY(a, acc_model).m;
          unsafeAtomicAdd(&am.raw[acc_shell], acc_J);
          unsafeAtomicAdd(&am.raw[am.S + acc_shell], acc_nb);
        }
        acc_shell = sh;
        acc_model = model;
        acc_J = 0.0;
        acc_nb = 0.0;
      }

      if (line_hit) {
        // ---- line interaction (section 2.5): J and nu-bar over the flight
        // (section 2.7), move, branch draw, new direction
        const double d = d_line;
        const double jc = e_cmf * d * D;
        acc_J += jc;
        acc_nb += jc * nu_cmf;
        const double r_new = root_pos(r * r + d * d + 2.0 * r * d * mu);
        const double mu_new = fmin(fmax(quot(rmu + d, divisor(r_new)), -1.0), 1.0);
        const double D_old = 1.0 - quot(mu_new * r_new, v.rct);
        const double e_cmf_ev = E * D_old;
        double nu_cmf_out = nu_hit;
        int32_t emit = k;
        if (v.downbranch) {
          const int32_t up = v.line_upper[k];
          const int64_t j = grp.row_select(v.em_cum, v.level_ptr[up], v.level_ptr[up + 1], u1);
          emit = grp.uni(v.em_line[j]);
          nu_cmf_out = v.line_nu[emit];
        }
        const double mu_out = 2.0 * u2 - 1.0;
        const Divisor rD = divisor(1.0 - quot(mu_out * r_new, v.rct));
        r = r_new;
        mu = mu_out;
        nu = quot(nu_cmf_out, rD);
        E = quot(e_cmf_ev, rD);
        draw += 3;
        next_line = emit + 1;
        n_line += 1;
        last_line = k;
        if (v.records) hash = fnv_event(hash, EV_LINE, sh, k, emit);
        continue;
      }
      // ---- no line reached first: Thomson event or shell boundary
      const double d_electron = elec(tau_rem);
      const bool escat = d_electron < d_shell;
      const double d = escat ? d_electron : d_shell;
      const double jc = e_cmf * d * D;
      acc_J += jc;
      acc_nb += jc * nu_cmf;
      const double r_new = root_pos(r * r + d * d + 2.0 * r * d * mu);
      const double mu_new = fmin(fmax(quot(rmu + d, divisor(r_new)), -1.0), 1.0);
      if (escat) {
        // coherent, isotropic in the comoving frame (section 2.5)
        const double D_old = 1.0 - quot(mu_new * r_new, v.rct);
        const double e_cmf_ev = E * D_old;
        const double nu_cmf_out = nu * D_old;
        const double mu_out = 2.0 * u1 - 1.0;
        const Divisor rD = divisor(1.0 - quot(mu_out * r_new, v.rct));
        r = r_new;
        mu = mu_out;
        nu = quot(nu_cmf_out, rD);
        E = quot(e_cmf_ev, rD);
        draw += 2;
        n_esc += 1;
        if (v.records) hash = fnv_event(hash, EV_ESCATTER, sh, -1, -1);
        continue;
      }
      const int kind = inward ? EV_SHELL_IN : EV_SHELL_OUT;
      r = inward ? c_rin : c_rout;
      mu = mu_new;
      draw += 1;
      if (v.records) hash = fnv_event(hash, kind, sh, -1, -1);
      shell = sh + (inward ? -1 : 1);
      if (shell >= v.S) {
        status = SMC_ESCAPED;
        break;
      }
      if (shell < 0) {
        status = SMC_REABSORBED;
        break;
      }
    }
    n_seg = v.max_segments - seg_left;

    // ---- end of the history
    if (v.jblue && wshell >= 0 && jb_acc != 0.0)
      unsafeAtomicAdd(&v.jblue[(size_t)wshell * (size_t)v.L + wbase + lane], jb_acc * wn);
    if (leader) {
      const DevModel& m = ENTRY(a, model).m;
      lane_tally_end(m, tly, status, nu, E, n_seg, n_pass, n_line, n_esc, false);
      if (v.records)
        write_record(m, st.slot, st.pid, status, shell, nu, E, mu, r, st.mu0, st.nu_cmf0, n_seg,
                     n_esc, n_line, n_pass, hash, last_line);
    }
  }
  if (leader) {
    if (acc_shell >= 0) {
      const DevModel& am = ENTRY(a, acc_model).m;
      unsafeAtomicAdd(&am.raw[acc_shell], acc_J);
      unsafeAtomicAdd(&am.raw[am.S + acc_shell], acc_nb);
    }
    if (tally_model >= 0) lane_tally_flush(ENTRY(a, tally_model).m, tly);
  }
}

template <bool kMulti, int G, bool kExt>
__global__ __launch_bounds__(kLongBlock) void long_kernel(LaunchArgs a) {
  long_body<kMulti, G, kExt>(a);
}

template <bool kMulti>
__global__ __launch_bounds__(kLongBlock) void solo_kernel(LaunchArgs a) {
  solo_body<kMulti>(a);
}

// ---------------------------------------------------------------------------
// estimator normalisation and radiation-field update (sections 2.7, 2.8);
// blockIdx.x selects the model
// ---------------------------------------------------------------------------
template <bool kMulti>
__global__ void finalise_kernel(LaunchArgs a) {
  const int k = kMulti ? (int)blockIdx.x : 0;
  const DevModel& m = ENTRY(a, k).m;
  const DevIter& it = ENTRY(a, k).it;
  const int S = m.S;
  const double T = m.scalars[SC_T_USED];
  const double r_inner = m.r_bounds[0];
  // L_i = 4 pi r_i^2 sigma T^4; packet energies are in units of L_i dt
  const double L_inner = 4.0 * kPi * r_inner * r_inner * kSigmaSB * (T * T) * (T * T);
  for (int i = threadIdx.x; i < S; i += blockDim.x) {
    const double f = L_inner / (4.0 * kPi * m.volume[i]);
    const double J = f * m.raw[i];
    const double nb = f * m.raw[S + i];
    m.out_shell[i] = J;
    m.out_shell[S + i] = nb;
    m.out_shell[4 * S + i] = f * m.t_exp / kC;
    if (J > 0.0) {
      const double T_R = (kH / kKB) * (kPi * kPi * kPi * kPi / (360.0 * kZeta5)) * nb / J;
      m.out_shell[2 * S + i] = T_R;
      m.out_shell[3 * S + i] = kPi * J / (kSigmaSB * (T_R * T_R) * (T_R * T_R));
    }
  }
  const double dnu = (m.nu_max - m.nu_min) / (double)m.n_bins;
  for (int b = threadIdx.x; b < m.n_bins + 2; b += blockDim.x)
    m.out_spec[b] = L_inner * m.raw[2 * S + b] / dnu;
  if (it.n_virtual) {
    for (int b = threadIdx.x; b < m.n_bins + 2; b += blockDim.x)
      m.out_vspec[b] = L_inner * m.vraw[b] / dnu;
    if (threadIdx.x == 0) {
      double sum = 0.0;
      for (int b = 0; b < m.n_bins + 2; ++b) sum += m.vraw[b];
      m.out_vspec[m.n_bins + 2] = L_inner * sum;
    }
  }
  if (threadIdx.x == 0) {
    const double L_emit = L_inner * ((double)m.lsum[0] / kLScale);
    m.scalars[SC_L_EMITTED] = L_emit;
    m.scalars[SC_L_REABSORBED] = L_inner * ((double)m.lsum[1] / kLScale);
    m.scalars[SC_L_CAPPED] = L_inner * ((double)m.lsum[2] / kLScale);
    m.scalars[SC_L_INNER] = L_inner;
    // raise T_inner when the emergent luminosity is short of the request
    m.scalars[SC_T_NEXT] = (it.L_requested > 0.0 && L_emit > 0.0)
                               ? T * pow(it.L_requested / L_emit, 0.25 * it.damping)
                               : T;
  }
}

// J_blue normalisation: blockIdx.y selects the model
template <bool kMulti>
__global__ void jblue_scale_kernel(LaunchArgs a) {
  const int k = kMulti ? (int)blockIdx.y : 0;
  const DevModel& m = ENTRY(a, k).m;
  if (!m.jblue || !(ENTRY(a, k).it.flags & SMC_F_JBLUE)) return;
  const size_t n = (size_t)m.S * (size_t)m.L;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const double* scale = m.out_shell + 4 * m.S;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const int s = (int)(i / (size_t)m.L);
    m.jblue[i] = scale[s] * m.jblue[i];
  }
}

#undef ENTRY

size_t transport_lds_bytes(bool multi, int n_models) {
  size_t b = sizeof(LaneTally) * kBlock;
  if (multi) b += sizeof(uint64_t) * ((size_t)n_models + 1);
  return b;
}

}  // namespace

int transport_block_threads() { return kBlock; }
int long_block_threads() { return kLongBlock; }

hipError_t launch_geometry(const DevModel& m, const double* v_bounds, hipStream_t s) {
  const int n = m.S + 1 > 8 ? m.S + 1 : 8;
  hipLaunchKernelGGL(geometry_kernel, dim3((n + 255) / 256), dim3(256), 0, s, m, v_bounds);
  return hipGetLastError();
}

hipError_t transport_occupancy(bool multi, int* blocks_per_cu) {
  const size_t lds = transport_lds_bytes(multi, kMaxBatchModels);
  return multi ? hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu,
                                                              transport_kernel<true>, kBlock, lds)
               : hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu,
                                                              transport_kernel<false>, kBlock,
                                                              transport_lds_bytes(false, 1));
}

template <bool kMulti, bool kExt>
static hipError_t long_occupancy_of(int lanes, int* blocks_per_cu) {
  switch (lanes) {
    case 16:
      return hipOccupancyMaxActiveBlocksPerMultiprocessor(
          blocks_per_cu, long_kernel<kMulti, 16, kExt>, kLongBlock, 0);
    case 32:
      return hipOccupancyMaxActiveBlocksPerMultiprocessor(
          blocks_per_cu, long_kernel<kMulti, 32, kExt>, kLongBlock, 0);
    case 64:
      if constexpr (!kExt)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, solo_kernel<kMulti>,
                                                            kLongBlock, 0);
      return hipOccupancyMaxActiveBlocksPerMultiprocessor(
          blocks_per_cu, long_kernel<kMulti, 64, kExt>, kLongBlock, 0);
  }
  return hipErrorInvalidValue;
}

hipError_t long_occupancy(bool multi, int lanes, bool ext, int* blocks_per_cu) {
  if (multi)
    return ext ? long_occupancy_of<true, true>(lanes, blocks_per_cu)
               : long_occupancy_of<true, false>(lanes, blocks_per_cu);
  return ext ? long_occupancy_of<false, true>(lanes, blocks_per_cu)
             : long_occupancy_of<false, false>(lanes, blocks_per_cu);
}

template <bool kMulti, bool kExt>
static hipError_t launch_long(int lanes, dim3 grid, dim3 block, const LaunchArgs& a,
                              hipStream_t s) {
  switch (lanes) {
    case 16:
      hipLaunchKernelGGL((long_kernel<kMulti, 16, kExt>), grid, block, 0, s, a);
      break;
    case 32:
      hipLaunchKernelGGL((long_kernel<kMulti, 32, kExt>), grid, block, 0, s, a);
      break;
    case 64:
      if constexpr (!kExt)
        hipLaunchKernelGGL(solo_kernel<kMulti>, grid, block, 0, s, a);
      else
        hipLaunchKernelGGL((long_kernel<kMulti, 64, kExt>), grid, block, 0, s, a);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <bool kMulti>
static hipError_t launch_all(const LaunchArgs& a, const Shape& shape, uint64_t max_jblue,
                             hipEvent_t ev_start, hipEvent_t ev_stop, hipStream_t s) {
  const unsigned ny = kMulti ? (unsigned)a.n_models : 1u;
  // reset: enough blocks to zero the largest J_blue array
  uint64_t nz = max_jblue > 4096 ? max_jblue : 4096;
  uint64_t bx = (nz + 255) / 256;
  if (bx > 2048) bx = 2048;
  if (kMulti && bx * ny > 65536) bx = (65536 + ny - 1) / ny;
  if (bx < 1) bx = 1;
  hipLaunchKernelGGL(reset_kernel<kMulti>, dim3((unsigned)bx, ny), dim3(256), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (ev_start) {
    e = hipEventRecord(ev_start, s);
    if (e != hipSuccess) return e;
  }
  if (shape.transport_grid > 0) {
    hipLaunchKernelGGL(transport_kernel<kMulti>, dim3(shape.transport_grid), dim3(kBlock),
                       transport_lds_bytes(kMulti, a.n_models), s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (shape.long_grid > 0) {
      if (kMulti) {
        hipLaunchKernelGGL(long_prefix_kernel, dim3(1), dim3(64), 0, s, a,
                           const_cast<BatchEntry*>(a.table));
        if ((e = hipGetLastError()) != hipSuccess) return e;
      }
      const unsigned og = (unsigned)(shape.long_grid < 1024 ? shape.long_grid : 1024);
      hipLaunchKernelGGL(order_count_kernel<kMulti>, dim3(og), dim3(256), 0, s, a);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      hipLaunchKernelGGL(order_scan_kernel, dim3(1), dim3(kOrderBuckets), 0, s, a);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      hipLaunchKernelGGL(order_place_kernel<kMulti>, dim3(og), dim3(256), 0, s, a);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      const dim3 grid(shape.long_grid), block(kLongBlock);
      if (shape.long_ext)
        e = launch_long<kMulti, true>(shape.long_lanes, grid, block, a, s);
      else
        e = launch_long<kMulti, false>(shape.long_lanes, grid, block, a, s);
      if (e != hipSuccess) return e;
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  if (ev_stop) {
    e = hipEventRecord(ev_stop, s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(finalise_kernel<kMulti>, dim3(ny), dim3(256), 0, s, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (max_jblue > 0) {
    uint64_t jx = (max_jblue + 255) / 256;
    if (jx > 2048) jx = 2048;
    if (kMulti && jx * ny > 65536) jx = (65536 + ny - 1) / ny;
    if (jx < 1) jx = 1;
    hipLaunchKernelGGL(jblue_scale_kernel<kMulti>, dim3((unsigned)jx, ny), dim3(256), 0, s, a);
    e = hipGetLastError();
  }
  return e;
}

hipError_t launch_iteration(const LaunchArgs& a, bool multi, const Shape& shape,
                            uint64_t max_jblue, hipEvent_t ev_start, hipEvent_t ev_stop,
                            hipStream_t s) {
  return multi ? launch_all<true>(a, shape, max_jblue, ev_start, ev_stop, s)
               : launch_all<false>(a, shape, max_jblue, ev_start, ev_stop, s);
}

}  // namespace smc
