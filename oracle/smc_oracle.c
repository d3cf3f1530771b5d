/*
 * smc_oracle.c -- plain, slow, single-threaded FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the CPU
 * baseline leg of the benchmark.  It shares no code with the HIP path.
 *
 * What it computes (Kerzendorf & Sim 2014):
 *   - packet injection at the inner boundary            (section 2.4)
 *   - Thomson scattering with the first-order Doppler   (section 2.5)
 *   - Sobolev line interactions, scatter and downbranch  (section 2.5, Table 1)
 *   - the three-distance propagation scheme             (section 2.6)
 *   - the J, nu-bar and J_blue estimators               (section 2.7)
 *   - the radiation-field and T_inner update            (sections 2.7, 2.8)
 *   - the emergent spectrum from escaping packets       (section 2.9)
 *
 * Readings taken where the paper is silent or garbled are marked READING.
 * Random numbers come from Philox4x32-10 (Salmon et al. 2011), a
 * counter-based generator, in place of the Mersenne Twister named in
 * section 2; the draw schedule is fixed so that a second implementation can
 * reproduce every history.
 *
 * Compiled with -O2 -ffp-contract=off so that no multiply-add is fused.
 * All tallies use Neumaier-compensated sums.
 */
#include "smc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* CGS constants (CODATA 2018; the paper takes them from astropy) */
static const double ORC_C = 2.99792458e10;          /* speed of light [cm/s] */
static const double ORC_H = 6.62607015e-27;         /* Planck [erg s] */
static const double ORC_KB = 1.380649e-16;          /* Boltzmann [erg/K] */
static const double ORC_SIGMA_SB = 5.670374419e-5;  /* Stefan-Boltzmann [erg/cm^2/s/K^4] */
static const double ORC_SIGMA_T = 6.6524587321e-25; /* Thomson cross section [cm^2] */
static const double ORC_ZETA5 = 1.0369277551433699263;
static const double ORC_PI = 3.14159265358979323846;
static const double ORC_PI4_OVER_90 = 1.0823232337111381915; /* zeta(4) = sum of l^-4 */
static const int ORC_PLANCK_LMAX = 1000;

const char* oracle_version(void) { return "smc-oracle 2"; }

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror & Shaw 2011, "Parallel random numbers: */
/* as easy as 1, 2, 3").  Multipliers and Weyl key increments as published.  */
/* ------------------------------------------------------------------------ */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t p0 = (uint64_t)M0 * (uint64_t)x0;
    uint64_t p1 = (uint64_t)M1 * (uint64_t)x2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    uint32_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    k0 += W0;
    k1 += W1;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Uniform deviate in the open interval (0,1): the top 52 bits of a 64-bit
 * word plus one half, scaled by 2^-52.  Exact in FP64, never 0 or 1, so it
 * serves both the (0,1] and [0,1] draws of sections 2.4-2.6. */
double oracle_uniform(uint64_t word) {
  return ((double)(word >> 12) + 0.5) * 0x1p-52;
}

/* Per-packet random stream.  Draw d of packet p in iteration i is the 64-bit
 * word (x[2j+1] << 32) | x[2j], j = d%2, of the Philox4x32-10 block x with
 * counter {d/2, p_lo, p_hi, i} and key {seed_lo, seed_hi}. */
typedef struct {
  uint32_t key[2];
  uint64_t packet;
  uint32_t iteration;
  uint64_t draw;
} orc_stream;

static double orc_next_uniform(orc_stream* s) {
  uint32_t ctr[4] = {(uint32_t)(s->draw / 2), (uint32_t)s->packet,
                     (uint32_t)(s->packet >> 32), s->iteration};
  uint32_t out[4];
  oracle_philox4x32_10(ctr, s->key, out);
  int j = (int)(s->draw % 2);
  uint64_t w = ((uint64_t)out[2 * j + 1] << 32) | (uint64_t)out[2 * j];
  s->draw += 1;
  return oracle_uniform(w);
}

static void orc_stream_init(orc_stream* s, uint64_t seed, uint64_t packet, uint32_t iteration) {
  s->key[0] = (uint32_t)seed;
  s->key[1] = (uint32_t)(seed >> 32);
  s->packet = packet;
  s->iteration = iteration;
  s->draw = 0;
}

/* Direction draws of the v-packets of packet p in iteration i come from a
 * second stream: draw dv is word dv%2 of the block with counter
 * {dv/2, p_lo, p_hi, i} and key {seed_lo ^ 0x56504B54, seed_hi}.  The v-packet
 * j of the e-th launch of the packet (e = 0 at injection, then one per
 * interaction) takes draw dv = e * N_v + j, so v-packets never disturb the
 * r-packet's own draws. */
static double orc_virtual_uniform(uint64_t seed, uint64_t packet, uint32_t iteration,
                                  uint64_t dv) {
  uint32_t key[2] = {(uint32_t)seed ^ 0x56504B54u, (uint32_t)(seed >> 32)};
  uint32_t ctr[4] = {(uint32_t)(dv / 2), (uint32_t)packet, (uint32_t)(packet >> 32), iteration};
  uint32_t out[4];
  oracle_philox4x32_10(ctr, key, out);
  int j = (int)(dv % 2);
  return oracle_uniform(((uint64_t)out[2 * j + 1] << 32) | (uint64_t)out[2 * j]);
}

/* ------------------------------------------------------------------------ */
/* Compensated (Neumaier) accumulation                                      */
/* ------------------------------------------------------------------------ */
static void nsum_add(double* sum, double* comp, double x) {
  double t = *sum + x;
  if (fabs(*sum) >= fabs(x))
    *comp += (*sum - t) + x;
  else
    *comp += (x - t) + *sum;
  *sum = t;
}

/* Word-wise FNV-1a over (kind, shell, line, emitted line) of every event. */
static uint64_t hash_word(uint64_t h, uint64_t w) {
  return (h ^ w) * 0x100000001b3ULL;
}
static uint64_t hash_event(uint64_t h, int kind, int shell, int64_t line, int64_t emit) {
  h = hash_word(h, (uint64_t)(int64_t)kind);
  h = hash_word(h, (uint64_t)(int64_t)shell);
  h = hash_word(h, (uint64_t)line);
  h = hash_word(h, (uint64_t)emit);
  return h;
}

/* ------------------------------------------------------------------------ */
/* Geometry                                                                  */
/* ------------------------------------------------------------------------ */

/* First-order Doppler factor D = 1 - mu v / c with v = r / t_exp for
 * homologous flow (section 2.5). */
static double doppler(double r, double mu, double ct) {
  return 1.0 - (mu * r) / ct;
}

/* Distance along the ray (r, mu) to the shell boundary it meets first.
 * Textbook ray-sphere intersection (the paper gives no formula).  b is the
 * squared impact parameter.  READING: a tangent ray (b == r_in^2) misses the
 * inner sphere; round-off negatives are clamped to zero. */
double oracle_distance_to_shell(double r, double mu, double r_in, double r_out) {
  double b = r * r * ((1.0 - mu) * (1.0 + mu));
  double d;
  if (mu < 0.0 && b < r_in * r_in) {
    d = -r * mu - sqrt(r_in * r_in - b);
  } else {
    double q = r_out * r_out - b;
    if (q < 0.0) q = 0.0;
    d = sqrt(q) - r * mu;
  }
  if (d < 0.0) d = 0.0;
  return d;
}

/* Is the ray (r, mu) heading for the inner sphere? (same test as above) */
static int heads_inward(double r, double mu, double r_in) {
  double b = r * r * ((1.0 - mu) * (1.0 + mu));
  return mu < 0.0 && b < r_in * r_in;
}

/* Index of the closest redward line: the first k with nu_k < nu_cmf in the
 * non-increasing line list (section 2.6).  Plain bisection. */
static int64_t first_line_below(const double* nu, int64_t n, double nu_cmf) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (nu[mid] < nu_cmf)
      hi = mid;
    else
      lo = mid + 1;
  }
  return lo;
}

/* ------------------------------------------------------------------------ */
/* Injection (section 2.4)                                                   */
/* ------------------------------------------------------------------------ */

/* Planck-distributed x = h nu / k T by the exact mixture method of Carter &
 * Cashwell (1975), as in Bjorkman & Wood (2001): x^3/(e^x-1) is a sum over l
 * of l^-4-weighted Gamma(4, l) densities.  READING: the paper does not say how
 * it samples the Planck function.  l is capped at 1000 (tail mass < 1e-9). */
static double sample_planck_x(orc_stream* s) {
  double u_l = orc_next_uniform(s);
  double target = u_l * ORC_PI4_OVER_90;
  double acc = 0.0;
  int l = 1;
  for (; l <= ORC_PLANCK_LMAX; ++l) {
    double dl = (double)l;
    acc += 1.0 / (dl * dl * dl * dl);
    if (acc >= target) break;
  }
  if (l > ORC_PLANCK_LMAX) l = ORC_PLANCK_LMAX;
  double u1 = orc_next_uniform(s);
  double u2 = orc_next_uniform(s);
  double u3 = orc_next_uniform(s);
  double u4 = orc_next_uniform(s);
  return -log(((u1 * u2) * u3) * u4) / (double)l;
}

static void inject(const oracle_model* m, double T_inner, uint64_t n_packets, orc_stream* s,
                   double* mu, double* nu_cmf, double* nu_lab, double* e_lab,
                   int64_t* next_line) {
  double ct = ORC_C * m->t_exp;
  double r0 = m->v_bounds[0] * m->t_exp;
  /* zero limb darkening: mu = sqrt(z) */
  double u_mu = orc_next_uniform(s);
  *mu = sqrt(u_mu);
  double x = sample_planck_x(s);
  *nu_cmf = x * ORC_KB * T_inner / ORC_H;
  /* equal comoving energies 1/N (fraction of L_i * dt) */
  double e_cmf = 1.0 / (double)n_packets;
  /* READING: lab = comoving / D, the inverse of the first-order transform */
  double D = doppler(r0, *mu, ct);
  *nu_lab = *nu_cmf / D;
  *e_lab = e_cmf / D;
  *next_line = first_line_below(m->line_nu, m->n_lines, *nu_cmf);
}

void oracle_inject(const oracle_model* m, double T_inner, uint64_t n_packets, uint32_t iteration,
                   uint64_t packet_id, double* mu, double* nu_cmf, double* nu_lab,
                   double* e_lab, int64_t* next_line) {
  orc_stream s;
  orc_stream_init(&s, m->seed, packet_id, iteration);
  inject(m, T_inner, n_packets, &s, mu, nu_cmf, nu_lab, e_lab, next_line);
}

/* ------------------------------------------------------------------------ */
/* One packet history (sections 2.5-2.7, 2.9)                               */
/* ------------------------------------------------------------------------ */

typedef struct {
  double *J, *Jc, *nb, *nbc, *jb, *jbc, *sp, *spc, *L, *Lc, *vs, *vsc;
} orc_tally;

static size_t spectrum_bin(const oracle_model* m, double nu) {
  const int nb = m->n_bins;
  const double dnu = (m->nu_max - m->nu_min) / (double)nb;
  if (nu < m->nu_min) return (size_t)nb;
  double f = floor((nu - m->nu_min) / dnu);
  return (f >= (double)nb) ? (size_t)nb + 1 : (size_t)f;
}

/* Section 2.9: follow one v-packet from (r, mu) in `shell`, lines from
 * index k on, along its straight path to the outer boundary, adding the
 * Sobolev depth of every resonance it reaches and the Thomson depth of every
 * shell piece, with the conventions of the r-packet flight (quantities at the
 * start of each shell piece, a line counts when its resonance lies before the
 * shell boundary).  Returns 1 with *tau when the v-packet leaves the outer
 * boundary with tau_v <= ORACLE_TAU_VIRTUAL_MAX, else 0.  This is exactly the
 * probability exp(-tau_v) that an r-packet launched on that path escapes
 * without interacting, segment by segment. */
static int virtual_path(const oracle_model* m, double r, double mu, int shell, int64_t k,
                        double nu_lab, double* tau, uint64_t* passes) {
  const int S = m->n_shells;
  const int64_t L = m->n_lines;
  const double ct = ORC_C * m->t_exp;
  double t = 0.0;
  for (;;) {
    const double r_in = m->v_bounds[shell] * m->t_exp;
    const double r_out = m->v_bounds[shell + 1] * m->t_exp;
    const double D = doppler(r, mu, ct);
    const double nu_cmf = nu_lab * D;
    const double d_shell = oracle_distance_to_shell(r, mu, r_in, r_out);
    const double kappa = ORC_SIGMA_T * m->n_e[shell] * D;
    const double ct_over_nu = ct / nu_lab;
    while (k < L) {
      double d_line = (nu_cmf - m->line_nu[k]) * ct_over_nu;
      if (d_line < 0.0) d_line = 0.0;
      if (!(d_line < d_shell)) break;
      t += m->tau_sobolev[(size_t)shell * (size_t)L + (size_t)k];
      *passes += 1;
      if (t > ORACLE_TAU_VIRTUAL_MAX) return 0;
      k += 1;
    }
    t += kappa * d_shell;
    if (t > ORACLE_TAU_VIRTUAL_MAX) return 0;
    const int inward = heads_inward(r, mu, r_in);
    const double r_new = sqrt(r * r + d_shell * d_shell + 2.0 * r * d_shell * mu);
    double mu_new = (r * mu + d_shell) / r_new;
    if (mu_new > 1.0) mu_new = 1.0;
    if (mu_new < -1.0) mu_new = -1.0;
    r = inward ? r_in : r_out;
    mu = mu_new;
    shell += inward ? -1 : 1;
    if (shell >= S) {
      *tau = t;
      return 1;
    }
    if (shell < 0) return 0; /* only a ray grazing the inner boundary by rounding */
  }
}

/* Section 2.9: the v-packets of one packet launch.  They share the launching
 * r-packet's position, comoving frequency and next redward line, take
 * directions mu_v uniform in (mu_min, 1) with mu_min = -sqrt(1 - (r_i/r)^2)
 * (so that no v-packet meets the inner boundary), and comoving energies
 * E 2 mu_v / N_v at injection or E (1 - mu_min) / (2 N_v) after an
 * interaction.  READING: a v-packet's energy and frequency enter the
 * spectrum in the lab frame (E_v / D, nu_cmf / D at launch), as those of an
 * escaping r-packet do; this makes the v-packet spectrum an unbiased
 * estimate of the r-packet one. */
static void launch_virtual(const oracle_model* m, const oracle_iter* it, uint64_t pid,
                           uint64_t e, int injection, double r, int shell, int64_t next_line,
                           double nu_cmf, double e_cmf, orc_tally* t, oracle_out* out) {
  const double ct = ORC_C * m->t_exp;
  const double r_inner = m->v_bounds[0] * m->t_exp;
  const uint32_t nv = it->n_virtual;
  double q = 1.0 - (r_inner / r) * (r_inner / r);
  if (q < 0.0) q = 0.0;
  const double mu_min = -sqrt(q);
  for (uint32_t j = 0; j < nv; ++j) {
    const double u = orc_virtual_uniform(m->seed, pid, it->iteration, e * nv + j);
    const double mu_v = mu_min + (1.0 - mu_min) * u;
    const double w = injection ? 2.0 * mu_v / (double)nv : (1.0 - mu_min) / (2.0 * (double)nv);
    const double D = doppler(r, mu_v, ct);
    const double nu_lab = nu_cmf / D;
    const double e_lab = e_cmf * w / D;
    double tau = 0.0;
    out->vcounts[0] += 1;
    if (virtual_path(m, r, mu_v, shell, next_line, nu_lab, &tau, &out->vcounts[2])) {
      out->vcounts[1] += 1;
      const size_t bin = spectrum_bin(m, nu_lab);
      nsum_add(&t->vs[bin], &t->vsc[bin], e_lab * exp(-tau));
    }
  }
}

static void record_event(oracle_out* out, uint64_t pid, int kind, int shell, int64_t line,
                         int64_t emit, double r, double d, double mu_in, double mu_out,
                         double nu_in, double nu_out, double e_in, double e_out) {
  if (!out->trace) return;
  if (out->trace_len < out->trace_cap) {
    oracle_event* ev = &out->trace[out->trace_len];
    ev->packet_id = pid;
    ev->kind = kind;
    ev->shell = shell;
    ev->line = line;
    ev->emit_line = emit;
    ev->r = r;
    ev->d = d;
    ev->mu_in = mu_in;
    ev->mu_out = mu_out;
    ev->nu_in = nu_in;
    ev->nu_out = nu_out;
    ev->e_in = e_in;
    ev->e_out = e_out;
  }
  out->trace_len += 1;
}

static void run_packet(const oracle_model* m, const oracle_iter* it, uint64_t pid,
                       orc_tally* t, oracle_out* out, oracle_packet* rec) {
  const int S = m->n_shells;
  const int64_t L = m->n_lines;
  const double ct = ORC_C * m->t_exp;

  orc_stream s;
  orc_stream_init(&s, m->seed, pid, it->iteration);

  double mu, nu_cmf0, nu, E;
  int64_t next_line;
  inject(m, it->T_inner, it->n_packets, &s, &mu, &nu_cmf0, &nu, &E, &next_line);
  double r = m->v_bounds[0] * m->t_exp;
  int shell = 0;
  double mu0 = mu;

  uint64_t hash = 0xcbf29ce484222325ULL;
  uint64_t n_seg = 0, n_esc = 0, n_line = 0, n_pass = 0;
  int64_t last_line = -1;
  int status = ORACLE_LIVE;
  record_event(out, pid, ORACLE_EV_INJECT, 0, -1, -1, r, 0.0, mu, mu, nu, nu, E, E);
  if (t->vs)
    launch_virtual(m, it, pid, 0, 1, r, 0, next_line, nu_cmf0, 1.0 / (double)it->n_packets, t,
                   out);

  for (;;) {
    if (n_seg >= it->max_segments) {
      status = ORACLE_CAPPED;
      break;
    }
    n_seg += 1;
    out->counters[ORACLE_C_SEGMENTS] += 1;

    const double r_in = m->v_bounds[shell] * m->t_exp;
    const double r_out = m->v_bounds[shell + 1] * m->t_exp;

    /* section 2.6: optical depth to the next event.  The paper prints
     * tau = ln z; READING: the attenuation law needs tau = -ln z. */
    double tau_event = -log(orc_next_uniform(&s));

    /* quantities at the segment start */
    double D = doppler(r, mu, ct);
    double nu_cmf = nu * D;
    double e_cmf = E * D;
    double d_shell = oracle_distance_to_shell(r, mu, r_in, r_out);
    /* section 2.5: observer-frame Thomson opacity kappa_e = sigma_T n_e D */
    double kappa = ORC_SIGMA_T * m->n_e[shell] * D;
    double d_electron = kappa > 0.0 ? tau_event / kappa : INFINITY;

    /* section 2.6: march through the redward lines while d_line is the
     * shortest distance.  READING: the combined optical depth uses kappa_e
     * (with D) so that tau accumulates as integral(kappa ds) + sum(tau_S). */
    int line_hit = 0;
    int64_t k = next_line;
    double d_line = 0.0;
    const double ct_over_nu = ct / nu;
    while (k < L) {
      d_line = (nu_cmf - m->line_nu[k]) * ct_over_nu;
      if (d_line < 0.0) d_line = 0.0;
      if (!(d_line < d_electron && d_line < d_shell)) break;
      /* section 2.7: J_blue over every resonance passage (READING: the
       * interacting passage included).  (E/nu)_cmf * D at resonance equals
       * E * nu_k / nu^2 in lab quantities, because D_res = nu_k / nu. */
      n_pass += 1;
      out->counters[ORACLE_C_LINE_PASSES] += 1;
      if (t->jb) {
        size_t idx = (size_t)shell * (size_t)L + (size_t)k;
        nsum_add(&t->jb[idx], &t->jbc[idx], E * m->line_nu[k] / (nu * nu));
      }
      double tau_line = m->tau_sobolev[(size_t)shell * (size_t)L + (size_t)k];
      if (tau_line + kappa * d_line > tau_event) {
        line_hit = 1;
        break;
      }
      tau_event -= tau_line;
      if (kappa > 0.0) d_electron = tau_event / kappa;
      k += 1;
    }
    next_line = k;

    int kind;
    double d;
    if (line_hit) {
      kind = ORACLE_EV_LINE;
      d = d_line;
    } else if (d_electron < d_shell) {
      kind = ORACLE_EV_ESCATTER;
      d = d_electron;
    } else {
      kind = heads_inward(r, mu, r_in) ? ORACLE_EV_SHELL_IN : ORACLE_EV_SHELL_OUT;
      d = d_shell;
    }

    /* section 2.7: J and nu-bar with comoving E and nu, observer-frame path
     * length l and D, all at the segment start. */
    double jc = e_cmf * d * D;
    nsum_add(&t->J[shell], &t->Jc[shell], jc);
    nsum_add(&t->nb[shell], &t->nbc[shell], jc * nu_cmf);

    /* move along the straight flight path */
    double r_new = sqrt(r * r + d * d + 2.0 * r * d * mu);
    double mu_new = (r * mu + d) / r_new;
    if (mu_new > 1.0) mu_new = 1.0;
    if (mu_new < -1.0) mu_new = -1.0;
    double mu_before = mu_new, nu_before = nu, e_before = E;

    if (kind == ORACLE_EV_SHELL_OUT || kind == ORACLE_EV_SHELL_IN) {
      /* section 2.6: cross into the neighbouring shell; the domain edges end
       * the history (escape outside, reabsorption inside). */
      r = (kind == ORACLE_EV_SHELL_OUT) ? r_out : r_in;
      mu = mu_new;
      out->counters[ORACLE_C_CROSSINGS] += 1;
      hash = hash_event(hash, kind, shell, -1, -1);
      record_event(out, pid, kind, shell, -1, -1, r, d, mu, mu, nu, nu, E, E);
      shell += (kind == ORACLE_EV_SHELL_OUT) ? 1 : -1;
      if (shell >= S) {
        status = ORACLE_ESCAPED;
        break;
      }
      if (shell < 0) {
        status = ORACLE_REABSORBED;
        break;
      }
      continue;
    }

    r = r_new;
    double D_old = doppler(r, mu_new, ct);
    double e_cmf_ev = E * D_old;

    if (kind == ORACLE_EV_ESCATTER) {
      /* section 2.5: coherent, isotropic Thomson scattering in the comoving
       * frame: nu_cmf and E_cmf kept, mu = 2z - 1. */
      double nu_cmf_ev = nu * D_old;
      double u_mu = orc_next_uniform(&s);
      mu = 2.0 * u_mu - 1.0;
      double D_new = doppler(r, mu, ct);
      nu = nu_cmf_ev / D_new;
      E = e_cmf_ev / D_new;
      n_esc += 1;
      out->counters[ORACLE_C_ESCATTERS] += 1;
      hash = hash_event(hash, kind, shell, -1, -1);
      record_event(out, pid, kind, shell, -1, -1, r, d, mu_before, mu, nu_before, nu, e_before, E);
      if (t->vs)
        launch_virtual(m, it, pid, n_esc + n_line, 0, r, shell, next_line, nu_cmf_ev, e_cmf_ev, t,
                       out);
      continue;
    }

    /* line interaction with line k (section 2.5).  Draws: the branch draw
     * (unused in scatter mode), one more per internal macro-atom jump, then
     * the new direction. */
    double u_branch = orc_next_uniform(&s);
    int64_t emit = k;
    if (m->line_mode == ORACLE_DOWNBRANCH) {
      /* downbranch: the macro atom activated in the upper level of line k
       * deactivates directly, choosing a downward line by its branching
       * probability (Table 1; macro atom without internal jumps). */
      int32_t up = m->line_upper[k];
      int64_t a = m->level_ptr[up], b = m->level_ptr[up + 1];
      int64_t j = a;
      while (j < b - 1 && !(m->em_cum[j] > u_branch)) j += 1;
      emit = m->em_line[j];
    } else if (m->line_mode == ORACLE_MACROATOM) {
      /* macroatom: the macro atom activated in the upper level of line k
       * makes internal jumps between levels until it deactivates by
       * emission in one of the current level's downward lines (section 2.5,
       * after Lucy 2002, 2003); each step draws from the level's row of this
       * shell's transition probabilities. */
      const int64_t n_em = m->level_ptr[m->n_levels];
      const double* cum = m->em_cum + (size_t)shell * (size_t)n_em;
      int32_t level = m->line_upper[k];
      double u = u_branch;
      uint64_t steps = 0;
      for (;;) {
        int64_t a = m->level_ptr[level], b = m->level_ptr[level + 1];
        int64_t j = a;
        while (j < b - 1 && !(cum[j] > u)) j += 1;
        int32_t target = m->em_line[j];
        if (target >= 0) {
          emit = target;
          break;
        }
        level = -target - 1;
        steps += 1;
        if (steps >= ORACLE_MACRO_MAX_STEPS) {
          emit = -1;
          break;
        }
        u = orc_next_uniform(&s);
      }
      if (emit < 0) {
        /* never deactivated: the packet ends at the interaction point */
        mu = mu_new;
        status = ORACLE_CAPPED;
        break;
      }
    }
    double u_mu = orc_next_uniform(&s);
    mu = 2.0 * u_mu - 1.0;
    double D_new = doppler(r, mu, ct);
    nu = m->line_nu[emit] / D_new;
    E = e_cmf_ev / D_new;
    next_line = emit + 1;
    n_line += 1;
    last_line = k;
    out->counters[ORACLE_C_LINE_EVENTS] += 1;
    hash = hash_event(hash, kind, shell, k, emit);
    record_event(out, pid, kind, shell, k, emit, r, d, mu_before, mu, nu_before, nu, e_before, E);
    if (t->vs)
      launch_virtual(m, it, pid, n_esc + n_line, 0, r, shell, next_line, m->line_nu[emit],
                     e_cmf_ev, t, out);
  }

  if (status == ORACLE_ESCAPED) {
    out->counters[ORACLE_C_ESCAPED] += 1;
    nsum_add(&t->L[0], &t->Lc[0], E);
    /* section 2.9: bin the escaping packet in lab-frame frequency */
    const size_t bin = spectrum_bin(m, nu);
    nsum_add(&t->sp[bin], &t->spc[bin], E);
  } else if (status == ORACLE_REABSORBED) {
    out->counters[ORACLE_C_REABSORBED] += 1;
    nsum_add(&t->L[1], &t->Lc[1], E);
  } else {
    out->counters[ORACLE_C_CAPPED] += 1;
    nsum_add(&t->L[2], &t->Lc[2], E);
  }

  if (rec) {
    rec->id = pid;
    rec->status = status;
    rec->shell = shell;
    rec->nu = nu;
    rec->energy = E;
    rec->mu = mu;
    rec->r = r;
    rec->mu0 = mu0;
    rec->nu_cmf0 = nu_cmf0;
    rec->n_segments = n_seg;
    rec->n_escatter = n_esc;
    rec->n_line = n_line;
    rec->n_passes = n_pass;
    rec->hash = hash;
    rec->last_line = last_line;
  }
}

static int validate(const oracle_model* m) {
  if (m->n_shells < 1 || m->n_lines < 0 || m->n_bins < 1) return -1;
  if (!(m->t_exp > 0.0)) return -1;
  for (int i = 0; i < m->n_shells; ++i)
    if (!(m->v_bounds[i + 1] > m->v_bounds[i]) || !(m->v_bounds[i] > 0.0)) return -1;
  for (int i = 0; i < m->n_shells; ++i)
    if (!(m->n_e[i] >= 0.0)) return -1;
  for (int64_t k = 1; k < m->n_lines; ++k)
    if (!(m->line_nu[k] <= m->line_nu[k - 1])) return -1;
  if (!(m->nu_max > m->nu_min)) return -1;
  if (m->line_mode == ORACLE_DOWNBRANCH || m->line_mode == ORACLE_MACROATOM) {
    for (int64_t k = 0; k < m->n_lines; ++k) {
      int32_t up = m->line_upper[k];
      if (up < 0 || up >= m->n_levels) return -1;
      if (!(m->level_ptr[up + 1] > m->level_ptr[up])) return -1;
    }
    const int64_t n_em = m->level_ptr[m->n_levels];
    for (int64_t j = 0; j < n_em; ++j) {
      int32_t t = m->em_line[j];
      if (t >= m->n_lines) return -1;
      if (t < 0) {
        if (m->line_mode != ORACLE_MACROATOM) return -1;
        int32_t lv = -t - 1;
        if (lv >= m->n_levels || !(m->level_ptr[lv + 1] > m->level_ptr[lv])) return -1;
      }
    }
  } else if (m->line_mode != ORACLE_SCATTER) {
    return -1;
  }
  return 0;
}

int oracle_run(const oracle_model* m, const oracle_iter* it, oracle_out* out) {
  if (validate(m) != 0) return -1;
  if (it->n_packets == 0 || !(it->T_inner > 0.0)) return -1;
  const size_t S = (size_t)m->n_shells, L = (size_t)m->n_lines;
  const size_t NB = (size_t)m->n_bins + 2;

  orc_tally t;
  memset(&t, 0, sizeof t);
  t.J = out->J_raw;
  t.nb = out->nubar_raw;
  t.sp = out->spec_raw;
  t.L = out->L_raw;
  memset(t.J, 0, S * sizeof(double));
  memset(t.nb, 0, S * sizeof(double));
  memset(t.sp, 0, NB * sizeof(double));
  memset(t.L, 0, 3 * sizeof(double));
  memset(out->counters, 0, ORACLE_N_COUNTERS * sizeof(uint64_t));
  t.Jc = calloc(S, sizeof(double));
  t.nbc = calloc(S, sizeof(double));
  t.spc = calloc(NB, sizeof(double));
  t.Lc = calloc(3, sizeof(double));
  if (it->want_jblue && out->jblue_raw) {
    t.jb = out->jblue_raw;
    memset(t.jb, 0, S * L * sizeof(double));
    t.jbc = calloc(S * L > 0 ? S * L : 1, sizeof(double));
  }
  out->trace_len = 0;
  memset(out->vcounts, 0, sizeof out->vcounts);
  if (it->n_virtual > 0 && out->vspec_raw) {
    t.vs = out->vspec_raw;
    memset(t.vs, 0, NB * sizeof(double));
    t.vsc = calloc(NB, sizeof(double));
  }

  uint64_t n = it->packet_ids ? it->n_ids : it->n_packets;
  for (uint64_t i = 0; i < n; ++i) {
    uint64_t pid = it->packet_ids ? it->packet_ids[i] : i;
    run_packet(m, it, pid, &t, out, out->packets ? &out->packets[i] : NULL);
  }

  for (size_t i = 0; i < S; ++i) {
    t.J[i] += t.Jc[i];
    t.nb[i] += t.nbc[i];
  }
  for (size_t i = 0; i < NB; ++i) t.sp[i] += t.spc[i];
  if (t.vs)
    for (size_t i = 0; i < NB; ++i) t.vs[i] += t.vsc[i];
  for (size_t i = 0; i < 3; ++i) t.L[i] += t.Lc[i];
  if (t.jb)
    for (size_t i = 0; i < S * L; ++i) t.jb[i] += t.jbc[i];
  free(t.Jc);
  free(t.nbc);
  free(t.spc);
  free(t.Lc);
  free(t.jbc);
  free(t.vsc);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Finalise (sections 2.7 and 2.8)                                           */
/* ------------------------------------------------------------------------ */
void oracle_initial_radiation_field(const oracle_model* m, double* T_R, double* W) {
  double r_inner = m->v_bounds[0] * m->t_exp;
  for (int i = 0; i < m->n_shells; ++i) {
    double r_c = 0.5 * (m->v_bounds[i] + m->v_bounds[i + 1]) * m->t_exp;
    double q = r_inner / r_c;
    T_R[i] = 10000.0;
    W[i] = 0.5 * (1.0 - sqrt(1.0 - q * q));
  }
}

int oracle_finalise(const oracle_model* m, double T_inner, double L_requested, double damping,
                    const oracle_out* raw, oracle_final* fin) {
  const int S = m->n_shells;
  const int64_t L = m->n_lines;
  const double r_inner = m->v_bounds[0] * m->t_exp;
  /* section 2.4: L_i = 4 pi r_i^2 sigma T_i^4; packet energies are in units
   * of L_i dt, so every estimator carries one factor L_i and no dt. */
  const double L_inner = 4.0 * ORC_PI * r_inner * r_inner * ORC_SIGMA_SB *
                         (T_inner * T_inner) * (T_inner * T_inner);
  fin->L_inner = L_inner;
  for (int i = 0; i < S; ++i) {
    double ri = m->v_bounds[i] * m->t_exp, ro = m->v_bounds[i + 1] * m->t_exp;
    double V = 4.0 * ORC_PI / 3.0 * (ro * ro * ro - ri * ri * ri);
    double f = L_inner / (4.0 * ORC_PI * V);
    fin->J[i] = f * raw->J_raw[i];
    fin->nubar[i] = f * raw->nubar_raw[i];
    if (fin->jblue && raw->jblue_raw) {
      double fb = f * m->t_exp / ORC_C;
      for (int64_t k = 0; k < L; ++k)
        fin->jblue[(size_t)i * (size_t)L + (size_t)k] =
            fb * raw->jblue_raw[(size_t)i * (size_t)L + (size_t)k];
    }
    /* section 2.7: T_R from the mean frequency, W from the energy density.
     * READING: a shell with no flight path keeps its previous T_R and W. */
    if (fin->J[i] > 0.0) {
      double T_R = (ORC_H / ORC_KB) * (ORC_PI * ORC_PI * ORC_PI * ORC_PI / (360.0 * ORC_ZETA5)) *
                   fin->nubar[i] / fin->J[i];
      fin->T_R[i] = T_R;
      fin->W[i] = ORC_PI * fin->J[i] / (ORC_SIGMA_SB * (T_R * T_R) * (T_R * T_R));
    }
  }
  const double dnu = (m->nu_max - m->nu_min) / (double)m->n_bins;
  for (int b = 0; b < m->n_bins + 2; ++b) fin->L_nu[b] = L_inner * raw->spec_raw[b] / dnu;
  /* section 2.9: L_v = E_v exp(-tau_v) / (dt dnu), summed per bin */
  fin->L_virtual = 0.0;
  if (fin->L_nu_virtual && raw->vspec_raw) {
    double sum = 0.0, comp = 0.0;
    for (int b = 0; b < m->n_bins + 2; ++b) {
      fin->L_nu_virtual[b] = L_inner * raw->vspec_raw[b] / dnu;
      nsum_add(&sum, &comp, raw->vspec_raw[b]);
    }
    fin->L_virtual = L_inner * (sum + comp);
  }
  fin->L_emitted = L_inner * raw->L_raw[0];
  fin->L_reabsorbed = L_inner * raw->L_raw[1];
  fin->L_capped = L_inner * raw->L_raw[2];
  /* section 2.8: raise T_inner when the emergent luminosity is below the
   * requested one and lower it otherwise.  READING: L_i scales as T_i^4, so
   * T_i <- T_i (L_requested / L_emitted)^(damping/4), applied every
   * iteration; damping = 1 is the undamped law. */
  if (L_requested > 0.0 && fin->L_emitted > 0.0)
    fin->T_inner_next = T_inner * pow(L_requested / fin->L_emitted, 0.25 * damping);
  else
    fin->T_inner_next = T_inner;
  return 0;
}
