/*
 * smc.h -- C ABI of libsmc, Monte Carlo r-packet transport through
 * homologously expanding spherical ejecta on AMD Instinct MI355X (gfx950).
 *
 * The method is the indivisible energy-packet scheme of Kerzendorf & Sim
 * (2014), "A spectral synthesis code for rapid modelling of supernovae":
 * packets are injected at the inner boundary (section 2.4), propagate through
 * shells with Thomson and Sobolev line opacity (sections 2.5, 2.6), and build
 * the J, nu-bar and J_blue estimators (section 2.7) and the emergent spectrum
 * (section 2.9); each iteration ends with the radiation-field and T_inner
 * update (sections 2.7, 2.8).
 *
 * Conventions for every entry point
 *   - Return value: SMC_OK (0) on success, a negative SMC_E* code otherwise;
 *     smc_last_error() then describes the failure (thread-local string, valid
 *     until the next call on the same thread).  On error nothing is written
 *     to the caller's output buffers.
 *   - "host" pointers are ordinary CPU memory; "device" pointers are HIP
 *     device memory of the context's GPU.  The caller owns every buffer it
 *     passes; the library only borrows them for the duration of the call,
 *     except the model workspace, which it borrows until smc_model_free().
 *   - Streams are hipStream_t passed as void* (NULL = the null stream).
 *     Launches are asynchronous on that stream; smc_read_* synchronise it.
 *   - Units are CGS.  Packet energies are fractions of L_i * dt: each packet
 *     carries comoving energy 1/N at injection.
 *   - Calls on one model must not overlap; distinct models may run
 *     concurrently on distinct streams.
 */
#ifndef SMC_H
#define SMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SMC_OK 0
#define SMC_EINVAL (-1)  /* invalid argument or model (ordering, sizes, signs, CSR) */
#define SMC_ENOMEM (-2)  /* workspace too small, or over the admitted budget */
#define SMC_EDEVICE (-3) /* HIP runtime error (text in smc_last_error) */
#define SMC_EBUSY (-4)   /* the object is in use */

#define SMC_SCATTER 0    /* resonance scattering (Table 1, "scatter") */
#define SMC_DOWNBRANCH 1 /* macro atom without internal jumps (Table 1, "downbranch") */
#define SMC_MACROATOM 2  /* macro atom with internal jumps (Table 1, "macroatom"; section 2.5) */

/* packet status */
#define SMC_LIVE 0
#define SMC_ESCAPED 1    /* left through the outer boundary (section 2.6) */
#define SMC_REABSORBED 2 /* crossed the inner boundary (section 2.6) */
#define SMC_CAPPED 3     /* reached max_segments flight segments */

/* capability / iteration flags */
#define SMC_F_JBLUE 1u   /* tally J_blue per line and shell ("detailed" rates, section 2.7) */
#define SMC_F_PACKETS 2u /* write one smc_packet_out per packet (parity and debugging) */
#define SMC_F_TIMING 4u  /* time the transport kernel with HIP events (smc_read_timing) */

/* counters returned by smc_read_counters, in this order */
#define SMC_C_SEGMENTS 0    /* flight segments (one per distance comparison) */
#define SMC_C_LINE_PASSES 1 /* Sobolev resonances reached (J_blue contributions) */
#define SMC_C_LINE_EVENTS 2 /* line interactions */
#define SMC_C_ESCATTERS 3   /* Thomson scatterings */
#define SMC_C_ESCAPED 4
#define SMC_C_REABSORBED 5
#define SMC_C_CAPPED 6
#define SMC_C_CROSSINGS 7   /* shell-boundary crossings */
#define SMC_N_COUNTERS 8

typedef struct smc_ctx smc_ctx;
typedef struct smc_model smc_model;

/* Model description (section 2.1 shells, section 2.5 lines).  All arrays are
 * host pointers read during smc_model_load only. */
typedef struct {
  int32_t n_shells;          /* S in 1 .. 4096 */
  const double* v_bounds;    /* [S+1] boundary velocities [cm/s], > 0, strictly increasing,
                                below c/2 */
  double t_exp;              /* time since explosion [s], > 0; radii are v * t_exp */
  const double* n_e;         /* [S] free-electron density [cm^-3], >= 0 */
  int64_t n_lines;           /* L >= 0 */
  const double* line_nu;     /* [L] line frequencies [Hz], non-increasing */
  const double* tau_sobolev; /* [S*L] Sobolev optical depth, shell-major (shell s at s*L), >= 0 */
  int32_t line_mode;         /* SMC_SCATTER, SMC_DOWNBRANCH or SMC_MACROATOM */
  /* macro-atom tables (ignored for SMC_SCATTER): the upper level of each line
   * (where an absorption activates the macro atom) and, per level, a CSR row
   * of transitions with cumulative probabilities (the last entry of each
   * used row is 1).  Downbranch: every entry is a downward line to emit in,
   * one probability set for all shells.  Macroatom: an entry em_line >= 0
   * deactivates by emission in that line, em_line = -(j+1) jumps to level j
   * (which then draws from its own row), and em_cum holds one probability
   * set per shell (shell-major).  A macro atom that makes 100000 internal
   * jumps without deactivating ends its packet as CAPPED.
   * Macroatom with level_ptr, em_line and em_cum all NULL (and n_em = 0):
   * the tables are derived on the device from the plasma state (section
   * 2.5 with 2.3): smc_plasma_load lays out the rows from the atom's lines
   * and every smc_plasma_update recomputes em_cum (see the plasma section);
   * iterations are refused until the first update. */
  const int32_t* line_upper; /* [L] in [0, n_levels) */
  int32_t n_levels;
  const int64_t* level_ptr;  /* [n_levels+1] row offsets into em_line / em_cum */
  int64_t n_em;              /* level_ptr[n_levels] */
  const int32_t* em_line;    /* [n_em] emitted line in [0, L), or -(level+1) (macroatom) */
  const double* em_cum;      /* [n_em] (downbranch) or [S*n_em] (macroatom) cumulative
                                probabilities in [0, 1], non-decreasing within a row
                                (SMC_EINVAL otherwise) */
  /* emergent spectrum: n_bins bins linear in lab frequency over
   * [nu_min, nu_max), plus underflow and overflow (section 2.9) */
  double nu_min, nu_max;
  int32_t n_bins;            /* 1 .. 8192 */
  uint64_t seed;             /* key of the model's Philox4x32-10 streams (low, high word) */
} smc_model_desc;

/* One Monte Carlo iteration (section 2.8). */
typedef struct {
  uint64_t n_packets;        /* N: sets the packet energy 1/N and the id range [0, N) */
  uint32_t iteration;        /* enters every packet's random-number counter */
  uint32_t flags;            /* SMC_F_* bits; JBLUE and PACKETS must also be load flags */
  double T_inner;            /* > 0: inner-boundary temperature [K]; <= 0: use the value
                                the previous iteration's update left on the device */
  double L_requested;        /* > 0: update T_inner toward this emergent luminosity [erg/s] */
  double damping;            /* exponent scale of the T_inner update, in (0, 1] */
  uint64_t max_segments;     /* flight segments before a packet is CAPPED, 1 .. 2^30 */
  const uint64_t* packet_ids;/* device [n_ids] subset of ids in [0, N), or NULL for all N */
  uint64_t n_ids;
  /* section 2.9: virtual packets per packet launch (injection and every
   * interaction), 0 .. 16; 0 = none.  With v-packets every history runs in
   * the group-per-packet kernel (the hand-off budget is ignored), and the
   * v-packet spectrum is read with smc_read_virtual_spectrum. */
  uint32_t n_virtual;
  uint32_t reserved;         /* must be 0 */
} smc_iter_params;

/* Per-packet record (SMC_F_PACKETS), in work-list order.  hash is a
 * word-wise FNV-1a over (kind, shell, line, emitted line) of every event,
 * with kind 1 = outward crossing, 2 = inward crossing, 3 = Thomson, 4 = line. */
typedef struct {
  uint64_t id;
  int32_t status;            /* SMC_ESCAPED / SMC_REABSORBED / SMC_CAPPED */
  int32_t shell;             /* S after escape, -1 after reabsorption */
  double nu, energy, mu, r;  /* final lab-frame frequency, energy, direction, radius */
  double mu0, nu_cmf0;       /* injection direction and comoving frequency */
  uint64_t n_segments, n_escatter, n_line, n_passes;
  uint64_t hash;
  int64_t last_line;         /* last absorbing line, -1 if none */
} smc_packet_out;

/* Launch tuning of one model (0 in a field = the library default). */
typedef struct {
  int32_t blocks_per_cu;     /* lane-per-packet kernel: workgroups of 256 resident per CU */
  int32_t long_waves_per_cu; /* group-per-packet kernel: wavefronts resident per CU */
  uint32_t long_budget;      /* flight segments after which a history moves from the
                                lane-per-packet to the group-per-packet kernel;
                                UINT32_MAX keeps every history in the first kernel;
                                the default is 256 for one model in the scatter and
                                downbranch modes, 4096 for a multi-model launch of
                                them, 1024 with macro atoms */
  uint32_t long_lanes;       /* lanes that carry one handed-off history: 16, 32 or 64
                                (a wavefront carries 64 / long_lanes of them); the
                                default is 64 (the wavefront-per-history kernel) for one
                                model in the scatter and downbranch modes without
                                v-packets, 16 for a multi-model launch of them, 32 with
                                macro atoms or v-packets */
} smc_tune;

/* Create a context on HIP device `hip_device`.  The context owns a few small
 * device and pinned host buffers for multi-model launches (about 3 MB). */
int smc_ctx_create(smc_ctx** out, int hip_device);
/* Free a context's buffers once the multi-model launches that use them have
 * finished (NULL: no-op).  Models, plasmas and graphs made on it are freed
 * first by the caller. */
int smc_ctx_destroy(smc_ctx* ctx);
/* Message of the last failing call on this thread (empty after a success);
 * valid until the thread's next call into the library. */
const char* smc_last_error(void);

/* Device workspace a model needs for up to n_packets_max packets per
 * iteration with the given capability flags.  Writes *bytes. */
int smc_model_workspace_bytes(const smc_model_desc* desc, uint64_t n_packets_max,
                              uint32_t flags, uint64_t* bytes);

/* Validate the description, copy its arrays into the caller's device
 * workspace (`ws_bytes` bytes at `d_workspace`, 256-byte aligned, device
 * memory of the context's device from hipMalloc: coarse-grained, since the
 * tallies are FP64 atomic adds; host and managed memory are refused with
 * SMC_EINVAL, and fine-grained memory must not be passed) and derive
 * the shell geometry (radii r = v t_exp and volumes) on the device
 * (section 2.1).  Synchronises `stream` before returning, so the host arrays
 * may be released afterwards.  The radiation field starts at T_R = 10^4 K and
 * geometric dilution at the shell centres (section 2.8). */
int smc_model_load(smc_ctx* ctx, const smc_model_desc* desc, uint64_t n_packets_max,
                   uint32_t flags, void* d_workspace, uint64_t ws_bytes, void* stream,
                   smc_model** out);
/* Release the handle; never frees the caller's workspace. */
int smc_model_free(smc_model* model);

/* Enqueue one iteration on `stream`: reset the tallies, inject and propagate
 * every packet (sections 2.4-2.6, 2.9), normalise the estimators and update
 * T_R, W and T_inner (sections 2.7, 2.8).  Asynchronous. */
int smc_run_iteration(smc_model* model, const smc_iter_params* params, void* stream);

/* Copy the normalised estimators of the last iteration to host buffers:
 * J and nubar [S] (section 2.7), jblue [S*L] shell-major (NULL to skip;
 * requires SMC_F_JBLUE), T_R and W [S].  Any pointer may be NULL. */
int smc_read_estimators(smc_model* model, double* J, double* nubar, double* jblue,
                        double* T_R, double* W, void* stream);

/* Copy the spectrum L_nu [n_bins+2] in erg s^-1 Hz^-1 (bins, underflow,
 * overflow) and six scalars: L_emitted, L_reabsorbed, L_capped, L_inner,
 * T_inner used by the iteration and T_inner for the next one. */
int smc_read_spectrum(smc_model* model, double* L_nu, double* scalars6, void* stream);

/* Copy the SMC_N_COUNTERS event counters of the last iteration. */
int smc_read_counters(smc_model* model, uint64_t* counters, void* stream);

/* The virtual-packet spectrum of the last iteration (section 2.9): each
 * v-packet leaves from the launching packet's position with a direction
 * uniform in (mu_min, 1), mu_min = -sqrt(1 - (r_inner/r)^2), comoving
 * energy E 2 mu_v / N_v (injection) or E (1 - mu_min) / (2 N_v)
 * (interaction), and adds its lab energy times exp(-tau_v) to the bin of its
 * lab frequency, tau_v being the Thomson and Sobolev depth of its straight
 * path to the outer boundary; v-packets with tau_v > 30 are not counted.
 * L_nu [n_bins + 2] in erg/s/Hz as smc_read_spectrum; *L_total the summed
 * luminosity [erg/s]; counts[3] (may be NULL): v-packets launched, counted,
 * and line resonances they swept.  Directions come from a second Philox
 * stream of the packet (key {seed_lo ^ 0x56504B54, seed_hi}, draw e*N_v + j
 * for v-packet j of the e-th launch).  Synchronises `stream`. */
int smc_read_virtual_spectrum(smc_model* model, double* L_nu, double* L_total, uint64_t* counts,
                              void* stream);

/* Copy the first n per-packet records of the last iteration
 * (requires SMC_F_PACKETS in both the load and the iteration flags). */
int smc_read_packets(smc_model* model, smc_packet_out* out, uint64_t n, void* stream);

/* Enqueue one iteration of each of n_models models (1 .. 1024, distinct, all
 * of this context) as ONE set of launches on `stream`: every kernel of the
 * iteration covers all models, and the lane-per-packet kernel pulls packets
 * of any model from one launch-wide queue, so models of uneven size and the
 * long histories of one overlap the bulk of the others.  params[k] is model
 * k's iteration (as for smc_run_iteration); `tune` (NULL: defaults) shapes
 * the launches; flags may hold SMC_F_TIMING (smc_batch_read_timing).
 * Results per model are those of smc_run_iteration up to the summation order
 * of the tallies.  The context stages the model table in a ring of pinned
 * and device buffers it owns, so calls may follow one another without
 * waiting for the GPU.  Asynchronous. */
int smc_batch_run(smc_ctx* ctx, smc_model* const* models, const smc_iter_params* params,
                  int n_models, const smc_tune* tune, uint32_t flags, void* stream);

/* smc_batch_run for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops): the launch-wide scratch (queue heads,
 * hand-off order histogram, device model table) lives in a static array of
 * 128 KiB on each device instead of the context's buffers, and the call
 * makes no allocation of any kind.  At most SMC_STATIC_MAX_MODELS models;
 * more is SMC_EINVAL.  Arguments, results and errors are those of
 * smc_batch_run.  All calls on one device share that array and keep its last
 * contents (each launch clears what it needs cleared), so two such calls on
 * one device must not overlap: issue them on one stream, or wait for one
 * before issuing the next.  Asynchronous. */
#define SMC_STATIC_MAX_MODELS 64
int smc_batch_run_static(smc_ctx* ctx, smc_model* const* models, const smc_iter_params* params,
                         int n_models, const smc_tune* tune, uint32_t flags, void* stream);

/* Measurement: the device's throughput of FP64 atomic adds in the patterns the
 * estimator tallies use: scattered = 0, each wavefront adds to 64 consecutive
 * doubles of a table (a J_blue window), at a new pseudo-random place each
 * round; scattered != 0, every lane adds at a pseudo-random place of its own
 * (the lane-per-packet tallies).  `d_table` is caller-owned device memory of
 * n_doubles (>= 64) doubles, which the call overwrites; 8 * n_cu workgroups of
 * 256 lanes make n_rounds adds per lane; the rate of the second of two
 * launches goes to *atomics_per_s.  Synchronises `stream`.  Returns
 * SMC_EINVAL for a null pointer, n_doubles < 64, n_rounds = 0 or n_cu < 1,
 * SMC_EDEVICE on a HIP error. */
int smc_measure_atomic_rate(double* d_table, uint64_t n_doubles, uint32_t n_rounds, int scattered,
                            int n_cu, void* stream, double* atomics_per_s);

/* Duration in milliseconds of the transport kernels of the last timed batch
 * of this context.  Waits for them to end. */
int smc_batch_read_timing(smc_ctx* ctx, double* transport_ms);

/* Pick launch tuning for this batch by running it: each candidate (NULL:
 * the library's coordinate search over hand-off budget, lanes per handed-off
 * history, waves per CU and workgroups per CU) runs two timed iterations of
 * the whole batch, the faster counting; a candidate of the search replaces
 * the current choice only when at least 2 % faster (runs of one batch vary
 * by a few per cent).  The choice goes to *best (its time to *best_ms, may
 * be NULL).  Every
 * params[k].T_inner must be > 0 so that all trials see the same inputs; the
 * models' tallies hold the last trial's results afterwards.  Synchronises
 * `stream`. */
int smc_batch_autotune(smc_ctx* ctx, smc_model* const* models, const smc_iter_params* params,
                       int n_models, const smc_tune* candidates, int n_candidates,
                       smc_tune* best, double* best_ms, void* stream);

/* A captured sequence of iterations: n_iter iterations of the same
 * n_models models (params[i*n_models + k] is iteration i of model k;
 * T_inner <= 0 carries the device-side update between iterations), recorded
 * once into a HIP graph and replayed by smc_graph_launch with no host work
 * per iteration.  n_models = 1 records the single-model kernels.  The graph
 * owns copies of the model tables; the models' workspaces and any
 * packet_ids arrays must outlive it.  Recording uses a private stream (so
 * `stream` may be the null stream) and enqueues nothing; launches must not
 * overlap with other work on the same models. */
typedef struct smc_graph smc_graph;
int smc_graph_capture(smc_ctx* ctx, smc_model* const* models, const smc_iter_params* params,
                      int n_models, int n_iter, const smc_tune* tune, void* stream,
                      smc_graph** out);
/* Replay a captured graph on `stream` (asynchronous). */
int smc_graph_launch(smc_graph* graph, void* stream);
/* Free a graph (NULL: no-op); waits for the device's outstanding work, so a
 * replay still in flight finishes first. */
int smc_graph_destroy(smc_graph* graph);

/* Set (NULL: reset to defaults) or read the launch tuning of a model.  Tuning
 * changes launch shapes only: results are identical up to the summation
 * order of the tallies. */
int smc_model_set_tune(smc_model* model, const smc_tune* tune);
int smc_model_get_tune(smc_model* model, smc_tune* tune);

/* Duration in milliseconds of the last iteration's transport kernels, from
 * HIP events recorded around them on the iteration's stream (requires
 * SMC_F_TIMING in that iteration's flags).  Waits for the kernel to end. */
int smc_read_timing(smc_model* model, double* transport_ms);

/* ---------------------------------------------------------------------------
 * Plasma state (section 2.3) and Sobolev optical depths (section 2.5)
 *
 * A plasma object recomputes a model's tau_sobolev and n_e on the device from
 * a radiation field (T_R, W per shell), closing the loop of section 2.8: the
 * estimators of one iteration set the opacities of the next.  Per shell:
 *   1. partition functions Z of every ion: the sum over its levels of
 *      g exp(-e / k T_R), with the factor W on every level that is not
 *      metastable in dilute-LTE excitation;
 *   2. ionization ratios N_{j+1} n_e / N_j: the Saha factor
 *      Phi = 2 Z_{j+1} / Z_j (2 pi m_e k T_R / h^2)^{3/2} exp(-chi_j / k T_R),
 *      times W [delta zeta_j + W (1 - zeta_j)] (T_e / T_R)^{1/2} with
 *      T_e = 0.9 T_R in the nebular mode;
 *   3. ion densities from the ratios, each element's total density and
 *      charge conservation, which fixes n_e (the unique root of the charge
 *      balance; an n_e below 1e-260 of the largest possible charge density
 *      is returned as that floor);
 *   4. level populations g / Z N exp(-e / k T_R), times W for levels that
 *      are not metastable in dilute-LTE excitation;
 *   5. tau_S = (pi e^2 / m_e c) f lambda t_exp n_l (1 - g_l n_u / (g_u n_l))
 *      with lambda = c / nu of the model's line list; a negative value
 *      (population inversion) is stored as 0 and counted.
 * NLTE excitation (section 2.3): the ions listed in the description may
 * instead take their level populations from statistical equilibrium.  For
 * every line l -> u of such an ion the downward rate per upper-level atom is
 * beta A_ul + beta B_ul J_b + C_ul n_e and the upward rate per lower-level
 * atom beta B_lu J_b + C_lu n_e, with beta = (1 - e^-tau) / tau of the line's
 * tau_S in the model when the update starts (1 at tau = 0), J_b = W B_nu(T_R)
 * or the model's J_blue estimator, A and B from f, and
 * C_ul = 8.629e-6 Upsilon / (g_u T_e^{1/2}), C_lu = C_ul (g_u / g_l)
 * exp(-h nu / k T_e), T_e = 0.9 T_R.  Inflow equals outflow for every level
 * and the populations sum to the ion density; the system is solved by LU
 * decomposition with partial pivoting, one workgroup per (ion, shell).
 * Populations below zero from rounding are stored as 0; a singular system
 * leaves that ion's populations from step 4 and is counted.
 * Macro-atom tables (a macroatom model loaded without tables): after step 5
 * the update recomputes the model's em_cum for every shell from the new
 * tau_S, with the macro atom of Lucy (2002, 2003) for bound-bound radiative
 * transitions.  A line's rates are R_ul = beta (A_ul + B_ul J_b) per
 * upper-level atom and R_lu = beta B_lu J_b per lower-level atom, beta from
 * the new tau_S, A and B from f, J_b = W B_nu(T_R) of the update's field or,
 * with SMC_JB_DETAILED, the model's J_blue estimator.  From level i (energy
 * e_i above its ion's ground state) the weights are R_il (e_i - e_l) for
 * deactivation in a line i -> l, R_il e_l for an internal jump down to l and
 * R_iu e_i for a jump up along i -> u.  Row i (laid out by smc_plasma_load)
 * holds the lines with upper level i as deactivations (in line order), the
 * same lines as jumps down, then the lines with lower level i as jumps up;
 * its cumulative sums are divided by the row's total (equal steps when the
 * total is 0) and its last entry is 1.  Downbranch tables and caller-given
 * macroatom tables are never changed.  Calls on a plasma and on its model
 * must not overlap.
 * ------------------------------------------------------------------------- */
#define SMC_ION_LTE 0        /* Saha ionization balance at T_R */
#define SMC_ION_NEBULAR 1    /* modified nebular approximation */
#define SMC_EXC_LTE 0        /* Boltzmann level populations at T_R */
#define SMC_EXC_DILUTE_LTE 1 /* Boltzmann, times W for levels that are not metastable */
#define SMC_JB_DILUTE_BLACKBODY 0 /* NLTE rates with J_b = W B_nu(T_R) */
#define SMC_JB_DETAILED 1         /* NLTE rates with the J_blue estimator of the model's last
                                     iteration (W B_nu(T_R) before its first iteration) */

typedef struct smc_plasma smc_plasma;

/* Atomic data and composition; host pointers read during smc_plasma_load
 * only.  S and L are the model's shells and lines. */
typedef struct {
  int32_t n_elements;              /* E, 1 .. 256 */
  int32_t n_ions;                  /* ion stages of all elements, E .. 2048 */
  int32_t n_levels;                /* levels of all ions, >= n_ions */
  int32_t n_nlte_ions;             /* ions that may take NLTE populations, 0 .. 64 */
  const int32_t* element_ion_ptr;  /* [E+1] the stages of element e are ions ptr[e] .. ptr[e+1]-1,
                                      stage j (charge j) at ptr[e] + j; ptr[0] = 0, increasing,
                                      ptr[E] = n_ions */
  const double* ion_chi;           /* [n_ions] energy to ionize stage j to j+1 [erg], > 0
                                      (the last stage of an element: unused) */
  const double* ion_zeta;          /* [n_ions] in [0, 1]: fraction of recombinations from stage
                                      j+1 that go to stage j's ground state (nebular mode) */
  const int32_t* ion_level_ptr;    /* [n_ions+1] the levels of ion i are ptr[i] .. ptr[i+1]-1,
                                      at least one; ptr[0] = 0, ptr[n_ions] = n_levels */
  const double* level_energy;      /* [n_levels] above the ion's ground state [erg], finite,
                                      >= 0; each ion's first level is its ground state
                                      (energy 0, metastable) */
  const double* level_g;           /* [n_levels] statistical weight, > 0 */
  const uint8_t* level_metastable; /* [n_levels] nonzero = metastable */
  const int32_t* line_lower;       /* [L] lower level of line k */
  const int32_t* line_upper;       /* [L] upper level of line k: same ion, higher energy */
  const double* line_f;            /* [L] absorption oscillator strength, >= 0 */
  const double* number_density;    /* [S*E] element number densities [cm^-3], >= 0,
                                      shell-major */
  const int32_t* nlte_ions;        /* [n_nlte_ions] distinct ion indices, each with 1 .. 64
                                      levels all joined to its ground state by its lines
                                      (NULL when n_nlte_ions = 0) */
  const double* line_upsilon;      /* [L] thermally averaged collision strength of each line,
                                      >= 0; read for the lines of NLTE ions only (NULL when
                                      n_nlte_ions = 0) */
} smc_plasma_desc;

typedef struct {
  int32_t ionization;  /* SMC_ION_LTE or SMC_ION_NEBULAR */
  int32_t excitation;  /* SMC_EXC_LTE or SMC_EXC_DILUTE_LTE */
  double delta;        /* nebular-mode correction factor, finite, >= 0 (unused in LTE) */
  const double* T_R;   /* host [S] radiation temperatures [K] > 0, or NULL (and W NULL):
                          the model's current T_R and W on the device (the last
                          iteration's, or the initial field of smc_model_load) */
  const double* W;     /* host [S] dilution factors > 0, or NULL */
  int32_t nlte;        /* 1: statistical equilibrium for the description's NLTE ions;
                          0: they follow `excitation` like every other ion */
  int32_t jblue_mode;  /* SMC_JB_DILUTE_BLACKBODY or SMC_JB_DETAILED: J_b of the NLTE rates
                          and of derived macro-atom tables (detailed needs a model loaded
                          with SMC_F_JBLUE whose last iteration, if any, tallied J_blue) */
} smc_plasma_params;

/* Device workspace of a plasma object for a model of n_shells shells and
 * n_lines lines (including 47 bytes per line for derived macro-atom tables).
 * Writes *bytes. */
int smc_plasma_workspace_bytes(const smc_plasma_desc* desc, int32_t n_shells, int64_t n_lines,
                               uint64_t* bytes);
/* Validate the description against the model, copy it into the caller's
 * device workspace (256-byte aligned device memory from hipMalloc, as for
 * smc_model_load; borrowed until smc_plasma_free) and derive the per-line
 * constants on the device.  The model must outlive the plasma object.  For a
 * macroatom model loaded without tables, the atom's n_levels and line_upper
 * must be the model's, and the call writes the model's rows (level_ptr,
 * em_line); otherwise it changes nothing in the model.  Synchronises
 * `stream`. */
int smc_plasma_load(smc_model* model, const smc_plasma_desc* desc, void* d_workspace,
                    uint64_t ws_bytes, void* stream, smc_plasma** out);
/* Enqueue steps 1-5 on `stream`, overwriting the model's tau_sobolev [S*L]
 * and n_e [S] on the device.  Host T_R / W arrays are copied before the call
 * returns; otherwise asynchronous. */
int smc_plasma_update(smc_plasma* plasma, const smc_plasma_params* params, void* stream);
/* Copy the state of the last update to host buffers (any may be NULL):
 * n_e [S], ion densities and partition functions [S*n_ions], level
 * populations [S*n_levels], tau_sobolev [S*L] (all shell-major) and
 * counts[2]: inverted (shell, line) pairs stored as 0, and singular NLTE
 * systems.  Synchronises `stream`. */
int smc_plasma_read(smc_plasma* plasma, double* n_e, double* ion_density, double* partition,
                    double* level_pop, double* tau_sobolev, uint64_t* counts, void* stream);
/* Release the handle; never frees the caller's workspace. */
int smc_plasma_free(smc_plasma* plasma);

/* Copy a downbranch or macroatom model's tables to host buffers (any may be
 * NULL): level_ptr [n_levels+1], em_line [n_em] and em_cum ([n_em], or
 * [S*n_em] shell-major in macroatom mode), where n_em = 3 L for derived
 * tables.  SMC_EINVAL for a scatter-mode model, or derived tables before
 * the first plasma update.  Synchronises `stream`. */
int smc_model_read_macroatom(smc_model* model, int64_t* level_ptr, int32_t* em_line,
                             double* em_cum, void* stream);

/* A captured sequence as smc_graph_capture in which every iteration of model
 * k is followed by the plasma update of plasmas[k] (NULL: none; the plasma
 * must belong to models[k]) with plasma_params[k], from the model's own
 * radiation field (its T_R and W must be NULL), so that the whole loop of
 * section 2.8 (transport, estimators, plasma state, opacities) replays with
 * no host work.  With detailed J_b every captured iteration of the model must
 * tally J_blue.  The plasma objects and their workspaces must outlive the
 * graph. */
int smc_graph_capture_plasma(smc_ctx* ctx, smc_model* const* models,
                             const smc_iter_params* params, int n_models, int n_iter,
                             const smc_tune* tune, smc_plasma* const* plasmas,
                             const smc_plasma_params* plasma_params, void* stream,
                             smc_graph** out);

#ifdef __cplusplus
}
#endif
#endif
