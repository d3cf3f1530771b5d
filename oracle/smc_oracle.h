/*
 * smc_oracle.h -- plain, slow, single-threaded FP64 CPU oracle for the
 * r-packet Monte Carlo transport of Kerzendorf & Sim (2014), sections 2.4-2.9.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP
 * implementation; the product path never links, loads or calls it.  It shares
 * no code, header, constant or helper with the HIP path.
 *
 * Units are CGS throughout.  Packet energies are dimensionless: every packet
 * starts with comoving energy 1/N, i.e. energies are fractions of L_i * dt
 * (section 2.4, the packet-energy equation), and the finaliser multiplies by
 * the inner-boundary luminosity L_i.
 */
#ifndef SMC_ORACLE_H
#define SMC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORACLE_SCATTER = 0, ORACLE_DOWNBRANCH = 1, ORACLE_MACROATOM = 2 };

/* A macro atom that has made this many internal jumps without deactivating
 * ends its packet as CAPPED. */
#define ORACLE_MACRO_MAX_STEPS 100000

enum { ORACLE_LIVE = 0, ORACLE_ESCAPED = 1, ORACLE_REABSORBED = 2, ORACLE_CAPPED = 3 };

/* event kinds, also the first word hashed into the per-packet event hash */
enum {
  ORACLE_EV_INJECT = 0,
  ORACLE_EV_SHELL_OUT = 1,
  ORACLE_EV_SHELL_IN = 2,
  ORACLE_EV_ESCATTER = 3,
  ORACLE_EV_LINE = 4
};

/* counters[] indices */
enum {
  ORACLE_C_SEGMENTS = 0,
  ORACLE_C_LINE_PASSES = 1,
  ORACLE_C_LINE_EVENTS = 2,
  ORACLE_C_ESCATTERS = 3,
  ORACLE_C_ESCAPED = 4,
  ORACLE_C_REABSORBED = 5,
  ORACLE_C_CAPPED = 6,
  ORACLE_C_CROSSINGS = 7,
  ORACLE_N_COUNTERS = 8
};

typedef struct {
  int32_t n_shells;            /* S */
  const double* v_bounds;      /* S+1 shell boundary velocities [cm/s], increasing */
  double t_exp;                /* time since explosion [s] */
  const double* n_e;           /* S free-electron densities [cm^-3] */
  int64_t n_lines;             /* L */
  const double* line_nu;       /* L line frequencies [Hz], non-increasing */
  const double* tau_sobolev;   /* S*L Sobolev optical depths, shell-major */
  int32_t line_mode;           /* ORACLE_SCATTER, ORACLE_DOWNBRANCH or ORACLE_MACROATOM */
  /* macro-atom tables (ignored in scatter mode): one row per level.  In
   * downbranch mode every entry is an emission line and em_cum holds one
   * row set; in macroatom mode an entry em_line = -(j+1) is an internal jump
   * to level j, and em_cum holds one row set per shell (shell-major,
   * S * level_ptr[n_levels] entries). */
  const int32_t* line_upper;   /* L: upper level of each line (the activated level) */
  int32_t n_levels;
  const int64_t* level_ptr;    /* n_levels+1 row offsets */
  const int32_t* em_line;      /* emission line index (>= 0) or internal jump (< 0) */
  const double* em_cum;        /* cumulative probability, last entry of a row is 1 */
  /* emergent spectrum grid, linear in lab-frame frequency */
  double nu_min, nu_max;
  int32_t n_bins;
  uint64_t seed;               /* Philox key (low word, high word) */
} oracle_model;

typedef struct {
  uint64_t n_packets;          /* N of the iteration: energy unit 1/N, ids in [0,N) */
  uint32_t iteration;          /* Philox counter word 3 */
  double T_inner;              /* inner boundary temperature [K] */
  uint64_t max_segments;       /* flight segments before a packet is CAPPED */
  const uint64_t* packet_ids;  /* subset of ids to run, NULL = all of [0,N) */
  uint64_t n_ids;
  int32_t want_jblue;
  uint32_t n_virtual;          /* v-packets per packet launch (section 2.9), 0 = none */
} oracle_iter;

typedef struct {
  uint64_t id;
  int32_t status;
  int32_t shell;               /* shell at termination (-1 or S at the domain edges) */
  double nu, energy, mu, r;    /* final lab-frame state */
  double mu0, nu_cmf0;         /* injection direction and comoving frequency */
  uint64_t n_segments, n_escatter, n_line, n_passes;
  uint64_t hash;               /* event-sequence hash */
  int64_t last_line;           /* last absorbing line, -1 if none */
} oracle_packet;

typedef struct {
  uint64_t packet_id;
  int32_t kind;                /* ORACLE_EV_* */
  int32_t shell;               /* shell the event happened in */
  int64_t line;                /* absorbing line (line events), else -1 */
  int64_t emit_line;           /* emitted line (line events), else -1 */
  double r, d;                 /* position after the move, flight distance */
  double mu_in, mu_out;        /* direction before / after the event */
  double nu_in, nu_out;        /* lab frequency before / after */
  double e_in, e_out;          /* lab energy before / after */
} oracle_event;

typedef struct {
  double* J_raw;               /* S:  sum of E_cmf * l * D */
  double* nubar_raw;           /* S:  sum of E_cmf * nu_cmf * l * D */
  double* jblue_raw;           /* S*L: sum of (E/nu)_cmf * D at resonance, or NULL */
  double* spec_raw;            /* n_bins+2: lab energy per bin, then under, over */
  double* L_raw;               /* 3: escaped, reabsorbed, capped lab energy */
  uint64_t* counters;          /* ORACLE_N_COUNTERS */
  double* vspec_raw;           /* n_bins+2: v-packet lab energy * exp(-tau_v) per bin, then
                                  under, over; NULL when no v-packets are run */
  uint64_t vcounts[3];         /* v-packets launched, v-packets counted, resonances they swept */
  oracle_packet* packets;      /* n_ids (or N) records, or NULL */
  oracle_event* trace;         /* event trace, or NULL */
  uint64_t trace_cap;
  uint64_t trace_len;          /* written by the oracle (may exceed cap: then truncated) */
} oracle_out;

typedef struct {
  double* J;                   /* S  mean intensity estimator [erg s^-1 cm^-2] */
  double* nubar;               /* S  frequency-weighted estimator */
  double* jblue;               /* S*L or NULL */
  double* T_R;                 /* S  in: previous value, out: new value */
  double* W;                   /* S  in: previous value, out: new value */
  double* L_nu;                /* n_bins+2 [erg s^-1 Hz^-1] (under/over as luminosity) */
  double* L_nu_virtual;        /* n_bins+2 v-packet spectrum, or NULL */
  double L_virtual;            /* v-packet estimate of the emergent luminosity [erg/s] */
  double L_emitted, L_reabsorbed, L_capped;
  double L_inner;
  double T_inner_next;
} oracle_final;

/* One Monte Carlo iteration over the chosen packets (sections 2.4-2.7, 2.9). */
int oracle_run(const oracle_model* m, const oracle_iter* it, oracle_out* out);

/* Estimator normalisation and radiation-field update (sections 2.7 and 2.8). */
int oracle_finalise(const oracle_model* m, double T_inner, double L_requested, double damping,
                    const oracle_out* raw, oracle_final* fin);

/* Initial radiation-field guess of section 2.8: T_R = 10^4 K, geometric W. */
void oracle_initial_radiation_field(const oracle_model* m, double* T_R, double* W);

/* v-packets whose accumulated optical depth exceeds this are not counted
 * (their weight exp(-tau_v) would be below 1e-13). */
#define ORACLE_TAU_VIRTUAL_MAX 30.0

/* Helpers exposed so that the pins can test each step on its own. */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double oracle_uniform(uint64_t word);
double oracle_distance_to_shell(double r, double mu, double r_in, double r_out);
void oracle_inject(const oracle_model* m, double T_inner, uint64_t n_packets, uint32_t iteration,
                   uint64_t packet_id, double* mu, double* nu_cmf, double* nu_lab,
                   double* e_lab, int64_t* next_line);
const char* oracle_version(void);

#ifdef __cplusplus
}
#endif
#endif
