// smc_plasma.hip -- plasma state (Kerzendorf & Sim 2014, section 2.3) and
// Sobolev optical depths (section 2.5) on the device.
//
// Two launches per update (one more with NLTE ions, one more for derived
// macro-atom tables):
//   plasma_state_kernel  one workgroup per shell: partition functions (one
//                        wavefront per ion, lanes over its levels), the log
//                        ionization ratios, n_e from charge conservation
//                        (one wavefront, lanes over elements, safeguarded
//                        Newton in ln n_e), ion densities and level
//                        populations.  Latency-bound and small: S workgroups
//                        of 16 wavefronts.
//   plasma_tau_kernel    one workgroup per (shell, 8192 lines): the shell's
//                        table of populations per statistical weight staged
//                        in LDS, then per line a 16-byte record, two LDS
//                        gathers and one coalesced 8-byte store.  HBM-bound
//                        on the tau_S stores.
//   plasma_nlte_kernel   (NLTE ions only, between the two) one wavefront per
//                        (ion, shell): rate matrix in LDS, LU solve.
//   macroatom_table_kernel (macroatom models whose tables derive from the
//                        plasma, after the depths) one lane per (level,
//                        shell): the row's transition weights and their
//                        cumulative sums.
// plasma_lines_kernel runs once at load and folds the oscillator strength,
// the wavelength and t_exp into one coefficient per line, and derives the
// Einstein coefficients of the macro-atom rates;
// plasma_nlte_lines_kernel derives the Einstein coefficients and collision
// constants of the NLTE ions' lines.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "../../include/smc.h"
#include "smc_internal.h"

namespace smc {
namespace {

// CGS, CODATA 2018
constexpr double kC = 2.99792458e10;
constexpr double kH = 6.62607015e-27;
constexpr double kKB = 1.380649e-16;
constexpr double kME = 9.1093837015e-28;
constexpr double kECharge = 1.602176634e-19 * 2.99792458e9;  // statcoulomb
constexpr double kPi = 3.14159265358979323846;
// pi e^2 / (m_e c): the classical line-strength constant [cm^2 s^-1]
constexpr double kLineConst = kPi * (kECharge * kECharge) / (kME * kC);
// the nebular mode takes the electron temperature as 0.9 T_R
constexpr double kTeOverTr = 0.9;
// n_e is searched in [x_max e^-600, x_max], x_max the largest possible
// charge density of the shell
constexpr double kLogNeRange = 600.0;
constexpr int kNewtonMax = 200;

constexpr int kWave = 64;
// one workgroup per shell: 16 wavefronts keep many level loads in flight
constexpr int kStateThreads = 1024;
constexpr int kTauThreads = 256;
// lines per workgroup of the depth kernel (32 per lane, in batches of 8)
constexpr int kTauChunk = 8192;
constexpr int kTauBatch = 8;
// independent loads a lane issues before using any of them
constexpr int kBatch = 4;
// NLTE solve: one wavefront per (ion, shell); rates of this many lines are
// staged in LDS at a time
constexpr int kNlteChunk = 256;
// the depth kernel stages a shell's n / g table in LDS up to this many levels
constexpr int kTauLdsLevels = 8192;

__device__ inline double wave_sum(double v) {
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ inline unsigned long long wave_sum_u64(unsigned long long v) {
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Charge moments of one element at ln n_e = u: stage j has log weight
// sum_{m<j} (lphi[a+m] - u) relative to stage 0.  Returns the mean charge and
// its variance (minus the derivative of the mean in u).
__device__ inline void element_moments(const double* lphi, int a, int b, double u, double* q,
                                       double* var) {
  double lr = 0.0, m = 0.0;
  for (int i = a; i < b - 1; ++i) {
    lr += lphi[i] - u;
    m = fmax(m, lr);
  }
  double s0 = exp(-m), s1 = 0.0, s2 = 0.0;
  lr = 0.0;
  for (int i = a; i < b - 1; ++i) {
    lr += lphi[i] - u;
    const double w = exp(lr - m);
    const double j = (double)(i - a + 1);
    s0 += w;
    s1 += j * w;
    s2 += j * j * w;
  }
  *q = s1 / s0;
  *var = fmax(s2 / s0 - *q * *q, 0.0);
}

__global__ __launch_bounds__(kStateThreads) void plasma_state_kernel(DevPlasma p) {
  extern __shared__ double sh[];
  double* Z = sh;                     // [n_ions] partition functions
  double* lphi = sh + p.n_ions;       // [n_ions] log ionization ratios (stage j -> j+1)
  double* N = sh + 2 * p.n_ions;      // [n_ions] ion densities
  __shared__ double s_ne;
  const int s = blockIdx.x;
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const double T = p.T_R[s], W = p.W[s];
  const double kT = kKB * T;
  const bool dilute = p.excitation == SMC_EXC_DILUTE_LTE;
  const double* dens = p.density + (size_t)s * p.E;

  // step 1: partition functions, one wavefront per ion; a lane's levels are
  // loaded kBatch at a time so that their latencies overlap
  for (int i = wave; i < p.n_ions; i += kStateThreads / kWave) {
    const int l0 = p.ion_level_ptr[i], l1 = p.ion_level_ptr[i + 1];
    double z = 0.0;
    for (int lb = l0 + lane; lb < l1; lb += kBatch * kWave) {
      double g[kBatch], en[kBatch];
      uint8_t meta[kBatch];
#pragma unroll
      for (int j = 0; j < kBatch; ++j) {
        const int l = lb + j * kWave;
        const bool in = l < l1;
        g[j] = in ? p.level_g[l] : 0.0;
        en[j] = in ? p.level_energy[l] : 0.0;
        meta[j] = in ? p.level_meta[l] : 1;
      }
#pragma unroll
      for (int j = 0; j < kBatch; ++j) {
        double b = g[j] * exp(-en[j] / kT);
        if (dilute && !meta[j]) b = W * b;
        z += b;
      }
    }
    z = wave_sum(z);
    if (lane == 0) Z[i] = z;
  }
  __syncthreads();

  // step 2: log of N_{j+1} n_e / N_j (Saha, or the nebular form)
  const double log_thermal = 1.5 * log(2.0 * kPi * kME * kT / (kH * kH));
  for (int e = threadIdx.x; e < p.E; e += kStateThreads) {
    const int a = p.elem_ion_ptr[e], b = p.elem_ion_ptr[e + 1];
    for (int i = a; i < b - 1; ++i) {
      double l = log(2.0) + log(Z[i + 1]) - log(Z[i]) + log_thermal - p.ion_chi[i] / kT;
      if (p.ionization == SMC_ION_NEBULAR) {
        const double z = p.ion_zeta[i];
        l = l + log(W * (p.delta * z + W * (1.0 - z))) + 0.5 * log(kTeOverTr);
      }
      lphi[i] = l;
    }
    lphi[b - 1] = -INFINITY;
  }
  __syncthreads();

  // step 3: n_e from charge conservation; g(u) = sum_e N_e q_e(u) - e^u is
  // strictly decreasing in u = ln n_e, so Newton steps are kept inside a
  // bracket that every evaluation narrows
  if (wave == 0) {
    double xmax = 0.0;
    for (int e = lane; e < p.E; e += kWave)
      xmax += dens[e] * (double)(p.elem_ion_ptr[e + 1] - p.elem_ion_ptr[e] - 1);
    xmax = wave_sum(xmax);
    double x = 0.0;
    if (xmax > 0.0) {
      double hi = log(xmax), lo = hi - kLogNeRange, u = hi;
      for (int it = 0; it < kNewtonMax; ++it) {
        double sq = 0.0, sv = 0.0;
        for (int e = lane; e < p.E; e += kWave) {
          const double Ne = dens[e];
          if (Ne > 0.0) {
            double q, var;
            element_moments(lphi, p.elem_ion_ptr[e], p.elem_ion_ptr[e + 1], u, &q, &var);
            sq += Ne * q;
            sv += Ne * var;
          }
        }
        sq = wave_sum(sq);
        sv = wave_sum(sv);
        const double xu = exp(u);
        const double g = sq - xu;
        if (g > 0.0) lo = u;
        else hi = u;
        // a Newton step that no longer moves u ends the search (it may touch
        // the bracket end it converges to); otherwise a step leaving the
        // bracket is replaced by bisection
        double un = u - g / (-sv - xu);
        const bool done = fabs(un - u) <= 1e-15 * fmax(1.0, fabs(u));
        if (!done && !(un > lo && un < hi)) un = 0.5 * (lo + hi);
        u = un;
        if (done || !(hi > lo)) break;
      }
      x = exp(u);
    }
    // ion densities at that n_e
    const double lx = x > 0.0 ? log(x) : 0.0;
    for (int e = lane; e < p.E; e += kWave) {
      const int a = p.elem_ion_ptr[e], b = p.elem_ion_ptr[e + 1];
      const double Ne = dens[e];
      if (x > 0.0) {
        double lr = 0.0, m = 0.0;
        for (int i = a; i < b - 1; ++i) {
          lr += lphi[i] - lx;
          m = fmax(m, lr);
        }
        double s0 = exp(-m);
        lr = 0.0;
        for (int i = a; i < b - 1; ++i) {
          lr += lphi[i] - lx;
          s0 += exp(lr - m);
        }
        N[a] = Ne * (exp(-m) / s0);
        lr = 0.0;
        for (int i = a; i < b - 1; ++i) {
          lr += lphi[i] - lx;
          N[i + 1] = Ne * (exp(lr - m) / s0);
        }
      } else {
        // no charge is possible: every element sits in its only stage
        for (int i = a; i < b; ++i) N[i] = i == a ? Ne : 0.0;
      }
    }
    if (lane == 0) s_ne = x;
  }
  __syncthreads();

  for (int i = threadIdx.x; i < p.n_ions; i += kStateThreads) {
    p.partition[(size_t)s * p.n_ions + i] = Z[i];
    p.ion_density[(size_t)s * p.n_ions + i] = N[i];
  }
  if (threadIdx.x == 0) {
    p.n_e[s] = s_ne;
    if (s == 0) {  // the NLTE and depth kernels run after this one
      p.clamped[0] = 0ull;
      p.clamped[1] = 0ull;
    }
  }
  // step 4: level populations n, and n / g, the form the depth kernel uses
  double* pop = p.level_pop + (size_t)s * p.n_levels;
  double* xg = p.level_x + (size_t)s * p.n_levels;
  for (int lb = threadIdx.x; lb < p.n_levels; lb += kBatch * kStateThreads) {
    int ion[kBatch];
    double g[kBatch], en[kBatch];
    uint8_t meta[kBatch];
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const int l = lb + j * kStateThreads;
      const bool in = l < p.n_levels;
      ion[j] = in ? p.level_ion[l] : 0;
      g[j] = in ? p.level_g[l] : 0.0;
      en[j] = in ? p.level_energy[l] : 0.0;
      meta[j] = in ? p.level_meta[l] : 1;
    }
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const int l = lb + j * kStateThreads;
      if (l < p.n_levels) {
        const double nz = N[ion[j]] / Z[ion[j]];
        double e = exp(-en[j] / kT);
        if (dilute && !meta[j]) e = W * e;
        pop[l] = nz * (g[j] * e);
        xg[l] = nz * e;
      }
    }
  }
}

// step 5: Sobolev depths.  With x = n / g per level,
//   n_l (1 - g_l n_u / (g_u n_l)) = g_l (x_l - x_u),
// so tau_S = (coef g_l) (x_l - x_u): two gathers and one store per (shell,
// line).  One workgroup takes one shell and kTauChunk lines; with kLds the
// shell's x table is staged in LDS first, so the gathers are LDS reads
// instead of divergent cache-line fetches.
template <bool kLds>
__global__ __launch_bounds__(kTauThreads) void plasma_tau_kernel(DevPlasma p) {
  extern __shared__ double xs[];
  const int s = blockIdx.y;
  const double* x = p.level_x + (size_t)s * p.n_levels;
  if (kLds) {
    for (int lb = threadIdx.x; lb < p.n_levels; lb += kBatch * kTauThreads) {
      double v[kBatch];
#pragma unroll
      for (int j = 0; j < kBatch; ++j) {
        const int l = lb + j * kTauThreads;
        v[j] = l < p.n_levels ? x[l] : 0.0;
      }
#pragma unroll
      for (int j = 0; j < kBatch; ++j) {
        const int l = lb + j * kTauThreads;
        if (l < p.n_levels) xs[l] = v[j];
      }
    }
    __syncthreads();
    x = xs;
  }
  const int k0 = blockIdx.x * kTauChunk;
  const int k1 = min(k0 + kTauChunk, p.L);
  double* tau = p.tau + (size_t)s * p.Lp;
  unsigned long long neg = 0;
  // kTauBatch records are loaded before any of them is used, so their
  // latencies overlap
  for (int kb = k0 + threadIdx.x; kb < k1; kb += kTauBatch * kTauThreads) {
    PlasmaLine ln[kTauBatch];
#pragma unroll
    for (int j = 0; j < kTauBatch; ++j) {
      const int k = kb + j * kTauThreads;
      if (k < k1) ln[j] = p.lines[k];
    }
#pragma unroll
    for (int j = 0; j < kTauBatch; ++j) {
      const int k = kb + j * kTauThreads;
      if (k < k1) {
        double t = ln[j].coef_g * (x[ln[j].lower] - x[ln[j].upper]);
        if (t < 0.0) {
          t = 0.0;
          ++neg;
        }
        tau[k] = t;
      }
    }
  }
  neg = wave_sum_u64(neg);
  if ((threadIdx.x % kWave) == 0 && neg) atomicAdd(p.clamped, neg);
}

// NLTE statistical equilibrium of one ion in one shell, one wavefront:
// rates of kNlteChunk lines at a time in LDS (lanes over lines); lane r
// assembles row r from the lines of level r only (a per-level list staged in
// LDS, in line order, so every sum has a fixed order, the diagonal in a
// register); equation 0 is replaced by the ion's total; then Gaussian
// elimination with partial pivoting (the pivot is the first row of largest
// magnitude; lane r eliminates row r) and back substitution.  A single
// wavefront needs no workgroup barriers; the barriers below only order its
// LDS accesses.
__global__ __launch_bounds__(kWave) void plasma_nlte_kernel(DevPlasma p) {
  extern __shared__ double sm[];
  __shared__ double r_ul[kNlteChunk], r_lu[kNlteChunk];
  const int j = blockIdx.x, s = blockIdx.y, t = threadIdx.x;
  const int ion = p.nlte_ions[j];
  const int l0 = p.ion_level_ptr[ion], n = p.ion_level_ptr[ion + 1] - l0;
  const int ld = n + 1;
  double* M = sm;  // [n][n+1]: rates, then the right-hand side in column n
  int32_t* ent = (int32_t*)(sm + kNlteMaxLevels * (kNlteMaxLevels + 1));
  const double T = p.T_R[s], W = p.W[s], ne = p.n_e[s];
  const double Te = kTeOverTr * T;
  const double sqrt_te = sqrt(Te);
  const int e0 = p.nlte_line_ptr[j], e1 = p.nlte_line_ptr[j + 1];
  for (int i = t; i < n * ld; i += kWave) M[i] = 0.0;
  for (int i = t; i < 2 * (e1 - e0); i += kWave) ent[i] = p.nlte_ent[2 * e0 + i];
  int cur = 0, end = 0;
  if (t < n) {
    cur = p.nlte_lev_ptr[j * (kNlteMaxLevels + 1) + t];
    end = p.nlte_lev_ptr[j * (kNlteMaxLevels + 1) + t + 1];
  }
  double diag = 0.0;
  __syncthreads();

  for (int c0 = e0; c0 < e1; c0 += kNlteChunk) {
    const int c1 = min(c0 + kNlteChunk, e1);
    for (int e = c0 + t; e < c1; e += kWave) {
      const NlteLine ln = p.nlte_lines[e];
      const double tau = p.tau[(size_t)s * p.Lp + ln.line];
      const double b = tau > 0.0 ? -expm1(-tau) / tau : 1.0;
      double J;
      if (p.jb_detailed) {
        J = p.jblue[(size_t)s * p.L + ln.line];
      } else {
        const double nu = ln.nu;
        J = W * (2.0 * kH * (nu * nu * nu) / (kC * kC) / expm1(kH * nu / (kKB * T)));
      }
      const double C_ul = ln.c_ul / sqrt_te;
      const double C_lu = C_ul * ln.g_ratio * exp(-kH * ln.nu / (kKB * Te));
      r_ul[e - c0] = b * ln.A_ul + b * ln.B_ul * J + C_ul * ne;
      r_lu[e - c0] = b * ln.B_lu * J + C_lu * ne;
    }
    __syncthreads();
    // row t: a line where t is the lower level sends r_lu out of t and
    // brings r_ul in from the upper level; where t is the upper level, r_ul
    // out and r_lu in
    for (; cur < end; ++cur) {
      const int32_t v = ent[cur];
      const int e = (v >> 16) + e0;
      if (e >= c1) break;
      const int other = (v >> 1) & 0x7fff;
      if (v & 1) {
        M[t * ld + other] += r_ul[e - c0];
        diag -= r_lu[e - c0];
      } else {
        M[t * ld + other] += r_lu[e - c0];
        diag -= r_ul[e - c0];
      }
    }
    __syncthreads();
  }
  if (t < n) M[t * ld + t] = diag;
  __syncthreads();
  if (t < n) M[t] = 1.0;
  if (t == 0) M[n] = p.ion_density[(size_t)s * p.n_ions + ion];
  __syncthreads();

  bool singular = false;
  for (int k = 0; k < n; ++k) {
    // pivot: largest |M[r][k]| over r >= k.  The bits of a non-negative
    // double order like the value, so one 64-bit maximum finds it; the low
    // 6 mantissa bits carry 63 - r instead, which picks the first row among
    // magnitudes equal to 2^-46 relative
    unsigned long long key = 0ull;
    if (t >= k && t < n)
      key = ((unsigned long long)__double_as_longlong(fabs(M[t * ld + k])) & ~63ull) |
            (unsigned long long)(63 - t);
    for (int o = kWave / 2; o > 0; o >>= 1) {
      const unsigned long long ok = __shfl_xor(key, o, kWave);
      key = ok > key ? ok : key;
    }
    const int bi = 63 - (int)(key & 63ull);
    if ((key >> 6) == 0ull) {
      singular = true;  // the same on every lane
      break;
    }
    if (bi != k) {
      for (int c = k + t; c <= n; c += kWave) {
        const double a = M[k * ld + c];
        M[k * ld + c] = M[bi * ld + c];
        M[bi * ld + c] = a;
      }
      __syncthreads();
    }
    if (t > k && t < n) {
      double* __restrict__ row = M + t * ld;
      const double* __restrict__ prow = M + k * ld;
      const double l = row[k] * (1.0 / prow[k]);
#pragma unroll 8
      for (int c = k + 1; c <= n; ++c) row[c] -= l * prow[c];
    }
    __syncthreads();
  }
  if (singular) {
    if (t == 0) atomicAdd(&p.clamped[1], 1ull);
    return;
  }
  for (int k = n - 1; k >= 0; --k) {
    const double xk = M[k * ld + n] / M[k * ld + k];
    __syncthreads();
    if (t == k) M[k * ld + n] = xk;
    if (t < k) M[t * ld + n] -= M[t * ld + k] * xk;
    __syncthreads();
  }
  double* pop = p.level_pop + (size_t)s * p.n_levels + l0;
  double* xg = p.level_x + (size_t)s * p.n_levels + l0;
  for (int r = t; r < n; r += kWave) {
    const double v = fmax(M[r * ld + n], 0.0);
    pop[r] = v;
    xg[r] = v / p.level_g[l0 + r];
  }
}

// Per-line constants of the NLTE rates, once at load.
__global__ void plasma_nlte_lines_kernel(DevPlasma p, int count) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  NlteLine& r = p.nlte_lines[e];
  const int k = r.line;
  const double g_l = p.level_g[p.lines[k].lower], g_u = p.level_g[p.lines[k].upper];
  const double nu = p.line_nu[k];
  const double coll = kH * kH / (pow(2.0 * kPi * kME, 1.5) * sqrt(kKB));
  r.B_lu = 4.0 * (kPi * kPi) * (kECharge * kECharge) * p.line_f[k] / (kME * kC * kH * nu);
  r.B_ul = g_l / g_u * r.B_lu;
  r.A_ul = 2.0 * kH * (nu * nu * nu) / (kC * kC) * r.B_ul;
  r.c_ul = coll * p.line_upsilon[k] / g_u;
  r.g_ratio = g_u / g_l;
  r.nu = nu;
}

__global__ void plasma_lines_kernel(DevPlasma p) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= p.L) return;
  const double nu = p.line_nu[k];
  const double coef = kLineConst * p.line_f[k] * (kC / nu) * p.t_exp;
  const double g_l = p.level_g[p.lines[k].lower], g_u = p.level_g[p.lines[k].upper];
  p.lines[k].coef_g = coef * g_l;
  // Einstein coefficients of the macro-atom rates (as the NLTE lines')
  MacroLine m;
  m.B_lu = 4.0 * (kPi * kPi) * (kECharge * kECharge) * p.line_f[k] / (kME * kC * kH * nu);
  m.B_ul = g_l / g_u * m.B_lu;
  m.A_ul = 2.0 * kH * (nu * nu * nu) / (kC * kC) * m.B_ul;
  m.pad = 0.0;
  p.macro_lines[k] = m;
}

// Macro-atom transition tables of a shell from its new plasma state
// (section 2.5: the macro atom of Lucy 2002, 2003 with bound-bound radiative
// transitions).  A line's radiative rates are R_ul = beta (A_ul + B_ul J_b)
// per upper-level atom and R_lu = beta B_lu J_b per lower-level atom, beta =
// (1 - e^-tau) / tau of the tau_S just computed; J_b = W B_nu(T_R), or the
// J_blue estimator in the detailed mode.  From level i (energy e_i) the
// weights are R_il (e_i - e_l) for deactivation in a line i -> l, R_il e_l
// for an internal jump down to l and R_iu e_i for a jump up along i -> u;
// the cumulative sums over the row are divided by the row's total (equal
// steps when it is 0) and the last entry is set to 1.  One lane per
// (level, shell) row, entries in row order: the sums are sequential, so they
// never decrease along a row.
__global__ __launch_bounds__(kWave) void macroatom_table_kernel(DevPlasma p) {
  const int lev = blockIdx.x * kWave + threadIdx.x;
  const int s = blockIdx.y;
  if (lev >= p.n_levels) return;
  const int64_t a = p.level_ptr[lev], b = p.level_ptr[lev + 1];
  if (b <= a) return;
  double* cum = p.em_cum + (size_t)s * (size_t)p.n_em;
  const double* tau = p.tau + (size_t)s * (size_t)p.Lp;
  const double e_i = p.level_energy[lev];
  const double T = p.T_R[s], Wd = p.W[s];
  double run = 0.0;
  for (int64_t j = a; j < b; ++j) {
    const int32_t k = p.em_via[j];
    const uint8_t kind = p.em_kind[j];
    const double t = tau[k];
    const double beta = t > 0.0 ? -expm1(-t) / t : 1.0;
    double J;
    if (p.macro_detailed) {
      J = p.jblue[(size_t)s * (size_t)p.L + (size_t)k];
    } else {
      const double nu = p.line_nu[k];
      J = Wd * (2.0 * kH * (nu * nu * nu) / (kC * kC) / expm1(kH * nu / (kKB * T)));
    }
    const MacroLine m = p.macro_lines[k];
    double w;
    if (kind == kMacroUp) {
      w = beta * m.B_lu * J * e_i;
    } else {
      const double e_l = p.level_energy[p.lines[k].lower];
      w = beta * (m.A_ul + m.B_ul * J) * (kind == kMacroEmit ? e_i - e_l : e_l);
    }
    run += w;
    cum[j] = run;
  }
  const double total = run;
  const double n = (double)(b - a);
  for (int64_t j = a; j < b - 1; ++j)
    cum[j] = total > 0.0 ? cum[j] / total : (double)(j - a + 1) / n;
  cum[b - 1] = 1.0;
}

}  // namespace

hipError_t launch_plasma_lines(const DevPlasma& p, int n_nlte_lines, hipStream_t s) {
  if (p.L == 0) return hipSuccess;
  hipLaunchKernelGGL(plasma_lines_kernel, dim3((p.L + 255) / 256), dim3(256), 0, s, p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || n_nlte_lines == 0) return e;
  hipLaunchKernelGGL(plasma_nlte_lines_kernel, dim3((n_nlte_lines + 255) / 256), dim3(256), 0,
                     s, p, n_nlte_lines);
  return hipGetLastError();
}

hipError_t launch_plasma_update(const DevPlasma& p, hipStream_t s) {
  const size_t lds = 3 * (size_t)p.n_ions * sizeof(double);
  hipLaunchKernelGGL(plasma_state_kernel, dim3(p.S), dim3(kStateThreads), lds, s, p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (p.n_nlte > 0) {
    const size_t lds = (size_t)kNlteMaxLevels * (kNlteMaxLevels + 1) * sizeof(double) +
                       2 * (size_t)kNlteMaxLines * sizeof(int32_t);
    hipLaunchKernelGGL(plasma_nlte_kernel, dim3(p.n_nlte, p.S), dim3(kWave), lds, s, p);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (p.L == 0) return hipSuccess;
  const dim3 grid((p.L + kTauChunk - 1) / kTauChunk, p.S);
  if (p.n_levels <= kTauLdsLevels)
    hipLaunchKernelGGL(plasma_tau_kernel<true>, grid, dim3(kTauThreads),
                       (size_t)p.n_levels * sizeof(double), s, p);
  else
    hipLaunchKernelGGL(plasma_tau_kernel<false>, grid, dim3(kTauThreads), 0, s, p);
  if ((e = hipGetLastError()) != hipSuccess || !p.macro) return e;
  hipLaunchKernelGGL(macroatom_table_kernel, dim3((p.n_levels + kWave - 1) / kWave, p.S),
                     dim3(kWave), 0, s, p);
  return hipGetLastError();
}

}  // namespace smc
