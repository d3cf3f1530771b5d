// smc_kernels.hip -- gfx950 kernels of the r-packet Monte Carlo transport
// (Kerzendorf & Sim 2014, sections 2.1-2.9).
//
// One packet per lane.  A persistent grid pulls packets from a work queue
// (one atomic per wavefront per refill), so a lane whose packet ends picks up
// the next one while its neighbours are still marching through lines.  All
// arithmetic on positions, directions, frequencies and energies is FP64.
// Shell tallies (J, nu-bar) accumulate in registers while a packet stays in a
// shell and are flushed to LDS copies private to the workgroup; the spectrum
// is an LDS histogram; both are merged into HBM once per workgroup.  J_blue
// (one entry per line and shell) is accumulated with hardware FP64 atomics.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

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
// Philox4x64-10 (Salmon et al. 2011).  Packet p of iteration i draws its d-th
// number from word d%4 of the block with counter {d/4, p, i, 0} and key
// {seed, 0}; the four words of the current block stay in registers.
// ---------------------------------------------------------------------------
struct Stream {
  uint64_t seed, pid, iter;
  uint64_t next;   // index of the next draw
  uint64_t block;  // block held in w0..w3
  uint64_t w0, w1, w2, w3;
};

__device__ __forceinline__ void philox_block(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                             uint64_t k0, uint64_t k1, uint64_t& o0,
                                             uint64_t& o1, uint64_t& o2, uint64_t& o3) {
  constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint64_t lo0 = M0 * c0, hi0 = __umul64hi(M0, c0);
    const uint64_t lo1 = M1 * c2, hi1 = __umul64hi(M1, c2);
    const uint64_t n0 = hi1 ^ c1 ^ k0;
    const uint64_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  o0 = c0;
  o1 = c1;
  o2 = c2;
  o3 = c3;
}

__device__ __forceinline__ void stream_init(Stream& g, uint64_t seed, uint64_t pid,
                                            uint64_t iter) {
  g.seed = seed;
  g.pid = pid;
  g.iter = iter;
  g.next = 0;
  g.block = ~0ull;
}

// uniform in (0,1): 52 random bits plus one half, times 2^-52 (exact)
__device__ __forceinline__ double draw(Stream& g) {
  const uint64_t b = g.next >> 2;
  if (b != g.block) {
    philox_block(b, g.pid, g.iter, 0, g.seed, 0, g.w0, g.w1, g.w2, g.w3);
    g.block = b;
  }
  const uint32_t sel = (uint32_t)(g.next & 3);
  const uint64_t w = sel == 0 ? g.w0 : sel == 1 ? g.w1 : sel == 2 ? g.w2 : g.w3;
  g.next += 1;
  return ((double)(w >> 12) + 0.5) * 0x1p-52;
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

// Planck sampling in x = h nu / k T: pick the mixture term l with weight
// l^-4 / zeta(4), then x ~ Gamma(4, l) from four uniforms.
__device__ __forceinline__ double planck_x(Stream& g) {
  const double target = draw(g) * kZeta4;
  double acc = 0.0;
  int l = 1;
  for (; l <= kPlanckTerms; ++l) {
    const double dl = (double)l;
    acc += 1.0 / (dl * dl * dl * dl);
    if (acc >= target) break;
  }
  if (l > kPlanckTerms) l = kPlanckTerms;
  const double u1 = draw(g);
  const double u2 = draw(g);
  const double u3 = draw(g);
  const double u4 = draw(g);
  return -log(((u1 * u2) * u3) * u4) / (double)l;
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

struct Packet {
  uint64_t slot, pid;
  double r, mu, nu, E;
  double mu0, nu_cmf0;
  int32_t shell;
  int32_t next_line;
  uint64_t n_seg, n_esc, n_line, n_pass, hash;
  int32_t last_line;
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

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

// zero every tally of the iteration and fix T_inner (graph-safe: no memset)
__global__ void reset_kernel(DevModel m, DevIter it) {
  const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const size_t n_raw = 2 * (size_t)m.S + (size_t)m.n_bins + 2;
  for (size_t i = tid; i < n_raw; i += stride) m.raw[i] = 0.0;
  if (tid < 4) m.lsum[tid] = 0.0;
  if (tid < SMC_N_COUNTERS + 1) m.counters[tid] = 0ull;
  if (m.jblue && (it.flags & SMC_F_JBLUE)) {
    const size_t n = (size_t)m.S * (size_t)m.L;
    for (size_t i = tid; i < n; i += stride) m.jblue[i] = 0.0;
  }
  if (tid == 0) {
    m.scalars[SC_T_USED] = it.T_param > 0.0 ? it.T_param : m.scalars[SC_T_NEXT];
  }
}

// ---------------------------------------------------------------------------
// the transport kernel (sections 2.4-2.7, 2.9)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void transport_kernel(DevModel m, DevIter it) {
  extern __shared__ double lds[];  // J[S], nubar[S], spectrum[NB+2]
  const int S = m.S;
  const int32_t L = m.L;
  const int n_lds = 2 * S + m.n_bins + 2;
  for (int i = threadIdx.x; i < n_lds; i += blockDim.x) lds[i] = 0.0;
  __syncthreads();
  double* lds_J = lds;
  double* lds_nb = lds + S;
  double* lds_spec = lds + 2 * S;

  const int lane = threadIdx.x & (kWave - 1);
  const double ct = m.ct;
  const double T_inner = m.scalars[SC_T_USED];
  const double r_inner = m.r_bounds[0];
  const double e_packet = 1.0 / (double)it.n_packets;
  const double dnu_bin = (m.nu_max - m.nu_min) / (double)m.n_bins;
  const bool want_jblue = m.jblue != nullptr && (it.flags & SMC_F_JBLUE);
  const bool want_packets = m.packets != nullptr && (it.flags & SMC_F_PACKETS);
  unsigned long long* queue = m.counters + SMC_N_COUNTERS;

  // per-lane tallies
  double l_esc = 0.0, l_reab = 0.0, l_cap = 0.0;
  unsigned long long c_seg = 0, c_pass = 0, c_line = 0, c_escat = 0, c_out = 0, c_reab = 0,
                     c_cap = 0, c_cross = 0;
  double acc_J = 0.0, acc_nb = 0.0;
  int acc_shell = -1;

  Packet p;
  Stream g;
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
        const uint64_t idx = base + (uint64_t)__popcll(below);
        if (idx < it.n_work) {
          // ---- injection at the inner boundary (section 2.4)
          p.slot = idx;
          p.pid = it.ids ? it.ids[idx] : idx;
          stream_init(g, m.seed, p.pid, it.iteration);
          p.mu = sqrt(draw(g));  // zero limb darkening
          const double x = planck_x(g);
          const double nu_cmf = x * kKB * T_inner / kH;
          const double D0 = doppler(r_inner, p.mu, ct);
          p.nu = nu_cmf / D0;
          p.E = e_packet / D0;
          p.r = r_inner;
          p.mu0 = p.mu;
          p.nu_cmf0 = nu_cmf;
          p.shell = 0;
          p.next_line = L > 0 ? first_below(m.line_nu, L, nu_cmf) : 0;
          p.n_seg = p.n_esc = p.n_line = p.n_pass = 0;
          p.hash = 0xcbf29ce484222325ull;
          p.last_line = -1;
          active = true;
        } else {
          exhausted = true;
        }
      }
    }
    if (__ballot(active) == 0ull) break;
    if (!active) continue;

    // ---- one flight segment (section 2.6)
    int status = SMC_LIVE;
    if (p.n_seg >= it.max_segments) {
      status = SMC_CAPPED;
    } else {
      p.n_seg += 1;
      c_seg += 1;
      const int sh = p.shell;
      const double r_in = m.r_bounds[sh];
      const double r_out = m.r_bounds[sh + 1];
      double tau_event = -log(draw(g));

      const double r = p.r, mu = p.mu, nu = p.nu, E = p.E;
      const double D = doppler(r, mu, ct);
      const double nu_cmf = nu * D;
      const double e_cmf = E * D;
      // distance to the shell boundary met first (ray-sphere intersection)
      const double b = r * r * ((1.0 - mu) * (1.0 + mu));
      const bool inward = mu < 0.0 && b < r_in * r_in;
      double d_shell;
      if (inward) {
        d_shell = -r * mu - sqrt(r_in * r_in - b);
      } else {
        double q = r_out * r_out - b;
        q = q < 0.0 ? 0.0 : q;
        d_shell = sqrt(q) - r * mu;
      }
      d_shell = d_shell < 0.0 ? 0.0 : d_shell;
      const double kappa = kSigmaT * m.n_e[sh] * D;  // Thomson opacity with D
      double d_electron = kappa > 0.0 ? tau_event / kappa : INFINITY;

      // line march: pass redward lines while d_line is the shortest distance
      const double* __restrict__ tau_row = m.tau + (size_t)sh * (size_t)L;
      const double ct_over_nu = ct / nu;
      int32_t k = p.next_line;
      bool line_hit = false;
      double d_line = 0.0;
      while (k < L) {
        const double nu_k = m.line_nu[k];
        d_line = (nu_cmf - nu_k) * ct_over_nu;
        d_line = d_line < 0.0 ? 0.0 : d_line;
        if (!(d_line < d_electron && d_line < d_shell)) break;
        p.n_pass += 1;
        c_pass += 1;
        if (want_jblue) unsafeAtomicAdd(&m.jblue[(size_t)sh * (size_t)L + k], E * nu_k / (nu * nu));
        const double tau_line = tau_row[k];
        if (tau_line + kappa * d_line > tau_event) {
          line_hit = true;
          break;
        }
        tau_event -= tau_line;
        if (kappa > 0.0) d_electron = tau_event / kappa;
        k += 1;
      }
      p.next_line = k;

      int kind;
      double d;
      if (line_hit) {
        kind = EV_LINE;
        d = d_line;
      } else if (d_electron < d_shell) {
        kind = EV_ESCATTER;
        d = d_electron;
      } else {
        kind = inward ? EV_SHELL_IN : EV_SHELL_OUT;
        d = d_shell;
      }

      // J and nu-bar estimators (section 2.7), register-accumulated per shell
      if (acc_shell != sh) {
        if (acc_shell >= 0) {
          atomicAdd(&lds_J[acc_shell], acc_J);
          atomicAdd(&lds_nb[acc_shell], acc_nb);
        }
        acc_shell = sh;
        acc_J = 0.0;
        acc_nb = 0.0;
      }
      const double jc = e_cmf * d * D;
      acc_J += jc;
      acc_nb += jc * nu_cmf;

      // move
      const double r_new = sqrt(r * r + d * d + 2.0 * r * d * mu);
      double mu_new = (r * mu + d) / r_new;
      mu_new = mu_new > 1.0 ? 1.0 : (mu_new < -1.0 ? -1.0 : mu_new);

      if (kind == EV_SHELL_OUT || kind == EV_SHELL_IN) {
        p.r = kind == EV_SHELL_OUT ? r_out : r_in;
        p.mu = mu_new;
        c_cross += 1;
        p.hash = fnv_event(p.hash, kind, sh, -1, -1);
        p.shell = sh + (kind == EV_SHELL_OUT ? 1 : -1);
        if (p.shell >= S)
          status = SMC_ESCAPED;
        else if (p.shell < 0)
          status = SMC_REABSORBED;
      } else {
        p.r = r_new;
        const double D_old = doppler(r_new, mu_new, ct);
        const double e_cmf_ev = E * D_old;
        if (kind == EV_ESCATTER) {
          // coherent isotropic Thomson scattering in the comoving frame
          const double nu_cmf_ev = nu * D_old;
          const double mu_out = 2.0 * draw(g) - 1.0;
          const double D_new = doppler(r_new, mu_out, ct);
          p.mu = mu_out;
          p.nu = nu_cmf_ev / D_new;
          p.E = e_cmf_ev / D_new;
          p.n_esc += 1;
          c_escat += 1;
          p.hash = fnv_event(p.hash, kind, sh, -1, -1);
        } else {
          // line interaction: branch draw (used by downbranch), then direction
          const double u_branch = draw(g);
          const double u_mu = draw(g);
          int32_t emit = k;
          if (m.mode == SMC_DOWNBRANCH) {
            const int32_t up = m.line_upper[k];
            const int64_t a = m.level_ptr[up], e = m.level_ptr[up + 1];
            int64_t j = a;
            while (j < e - 1 && !(m.em_cum[j] > u_branch)) ++j;
            emit = m.em_line[j];
          }
          const double mu_out = 2.0 * u_mu - 1.0;
          const double D_new = doppler(r_new, mu_out, ct);
          p.mu = mu_out;
          p.nu = m.line_nu[emit] / D_new;
          p.E = e_cmf_ev / D_new;
          p.next_line = emit + 1;
          p.n_line += 1;
          p.last_line = k;
          c_line += 1;
          p.hash = fnv_event(p.hash, kind, sh, k, emit);
        }
      }
    }

    if (status != SMC_LIVE) {
      // end of the history: spectrum and luminosity tallies (section 2.9)
      if (status == SMC_ESCAPED) {
        c_out += 1;
        l_esc += p.E;
        int bin;
        if (!(p.nu >= m.nu_min)) {
          bin = m.n_bins;  // underflow (a NaN would land here too, never out of range)
        } else {
          const double f = floor((p.nu - m.nu_min) / dnu_bin);
          bin = f >= (double)m.n_bins ? m.n_bins + 1 : (int)f;
        }
        atomicAdd(&lds_spec[bin], p.E);
      } else if (status == SMC_REABSORBED) {
        c_reab += 1;
        l_reab += p.E;
      } else {
        c_cap += 1;
        l_cap += p.E;
      }
      if (want_packets) {
        smc_packet_out rec;
        rec.id = p.pid;
        rec.status = status;
        rec.shell = p.shell;
        rec.nu = p.nu;
        rec.energy = p.E;
        rec.mu = p.mu;
        rec.r = p.r;
        rec.mu0 = p.mu0;
        rec.nu_cmf0 = p.nu_cmf0;
        rec.n_segments = p.n_seg;
        rec.n_escatter = p.n_esc;
        rec.n_line = p.n_line;
        rec.n_passes = p.n_pass;
        rec.hash = p.hash;
        rec.last_line = p.last_line;
        static_cast<smc_packet_out*>(m.packets)[p.slot] = rec;
      }
      active = false;
    }
  }

  if (acc_shell >= 0) {
    atomicAdd(&lds_J[acc_shell], acc_J);
    atomicAdd(&lds_nb[acc_shell], acc_nb);
  }
  // wave reductions of the scalar tallies, one global atomic per wave each
  l_esc = wave_sum(l_esc);
  l_reab = wave_sum(l_reab);
  l_cap = wave_sum(l_cap);
  c_seg = wave_sum_u64(c_seg);
  c_pass = wave_sum_u64(c_pass);
  c_line = wave_sum_u64(c_line);
  c_escat = wave_sum_u64(c_escat);
  c_out = wave_sum_u64(c_out);
  c_reab = wave_sum_u64(c_reab);
  c_cap = wave_sum_u64(c_cap);
  c_cross = wave_sum_u64(c_cross);
  if (lane == 0) {
    if (l_esc != 0.0) unsafeAtomicAdd(&m.lsum[0], l_esc);
    if (l_reab != 0.0) unsafeAtomicAdd(&m.lsum[1], l_reab);
    if (l_cap != 0.0) unsafeAtomicAdd(&m.lsum[2], l_cap);
    atomicAdd(&m.counters[SMC_C_SEGMENTS], c_seg);
    atomicAdd(&m.counters[SMC_C_LINE_PASSES], c_pass);
    atomicAdd(&m.counters[SMC_C_LINE_EVENTS], c_line);
    atomicAdd(&m.counters[SMC_C_ESCATTERS], c_escat);
    atomicAdd(&m.counters[SMC_C_ESCAPED], c_out);
    atomicAdd(&m.counters[SMC_C_REABSORBED], c_reab);
    atomicAdd(&m.counters[SMC_C_CAPPED], c_cap);
    atomicAdd(&m.counters[SMC_C_CROSSINGS], c_cross);
  }
  __syncthreads();
  // merge the workgroup's LDS tallies into HBM
  for (int i = threadIdx.x; i < n_lds; i += blockDim.x) {
    const double v = lds[i];
    if (v != 0.0) unsafeAtomicAdd(&m.raw[i], v);
  }
}

// ---------------------------------------------------------------------------
// estimator normalisation and radiation-field update (sections 2.7, 2.8)
// ---------------------------------------------------------------------------
__global__ void finalise_kernel(DevModel m, DevIter it) {
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
  if (threadIdx.x == 0) {
    const double L_emit = L_inner * m.lsum[0];
    m.scalars[SC_L_EMITTED] = L_emit;
    m.scalars[SC_L_REABSORBED] = L_inner * m.lsum[1];
    m.scalars[SC_L_CAPPED] = L_inner * m.lsum[2];
    m.scalars[SC_L_INNER] = L_inner;
    // raise T_inner when the emergent luminosity is short of the request
    m.scalars[SC_T_NEXT] = (it.L_requested > 0.0 && L_emit > 0.0)
                               ? T * pow(it.L_requested / L_emit, 0.25 * it.damping)
                               : T;
  }
}

__global__ void jblue_scale_kernel(DevModel m) {
  const size_t n = (size_t)m.S * (size_t)m.L;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const double* scale = m.out_shell + 4 * m.S;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const int s = (int)(i / (size_t)m.L);
    m.jblue[i] = scale[s] * m.jblue[i];
  }
}

}  // namespace

int transport_block_threads() { return kBlock; }

size_t transport_lds_bytes(const DevModel& m) {
  return sizeof(double) * (2 * (size_t)m.S + (size_t)m.n_bins + 2);
}

hipError_t launch_geometry(const DevModel& m, const double* v_bounds, hipStream_t s) {
  const int n = m.S + 1 > 8 ? m.S + 1 : 8;
  hipLaunchKernelGGL(geometry_kernel, dim3((n + 255) / 256), dim3(256), 0, s, m, v_bounds);
  return hipGetLastError();
}

hipError_t launch_reset(const DevModel& m, const DevIter& it, hipStream_t s) {
  size_t n = 2 * (size_t)m.S + (size_t)m.n_bins + 2;
  if (m.jblue && (it.flags & SMC_F_JBLUE)) {
    const size_t nj = (size_t)m.S * (size_t)m.L;
    if (nj > n) n = nj;
  }
  size_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(reset_kernel, dim3((unsigned)blocks), dim3(256), 0, s, m, it);
  return hipGetLastError();
}

hipError_t launch_transport(const DevModel& m, const DevIter& it, int grid, hipStream_t s) {
  hipLaunchKernelGGL(transport_kernel, dim3(grid), dim3(kBlock), transport_lds_bytes(m), s, m,
                     it);
  return hipGetLastError();
}

hipError_t launch_finalise(const DevModel& m, const DevIter& it, hipStream_t s) {
  hipLaunchKernelGGL(finalise_kernel, dim3(1), dim3(256), 0, s, m, it);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (m.jblue && (it.flags & SMC_F_JBLUE) && m.L > 0) {
    const size_t n = (size_t)m.S * (size_t)m.L;
    size_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(jblue_scale_kernel, dim3((unsigned)blocks), dim3(256), 0, s, m);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace smc
