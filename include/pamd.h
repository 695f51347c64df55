/*
 * pamd.h -- C ABI of the MI355X (gfx950) population-annealing MD library (libpamd.so).
 *
 * The calls follow the numbered population-annealing MD (PAMD) scheme of
 * Christiansen, Weigel & Janke, "Accelerating molecular dynamics simulations
 * with population annealing" (arXiv:1806.06016):
 *
 *   step 1  set up R independent copies at a high temperature T0  -> pamd_init
 *                                                                     (+ pamd_md_steps at T0)
 *   step 2  resample to T_i < T_{i-1} with weights
 *           tau_j = exp(-(1/kB T_i - 1/kB T_{i-1}) E_j) / Q,
 *           Q = (1/R) sum_j exp(-(1/kB T_i - 1/kB T_{i-1}) E_j),
 *           velocities rescaled by sqrt(T_i / T_{i-1})             -> pamd_resample
 *   step 3  theta MD steps per copy                                 -> pamd_md_steps
 *   step 4  observables as population averages                     -> pamd_observables
 *   step 5  loop until T_i <= T_N                                    (the caller)
 *
 * The free energy follows from the recorded normalisers: ln Q_i estimates
 * ln Z(T_i) - ln Z(T_{i-1}) (the paragraph on the recorded Q values); the
 * library accumulates sum_i ln Q_i in FP64 on the device.
 *
 * Conventions for every call
 *  - Returns a pamd_status; PAMD_OK == 0.  Nothing aborts or prints.  After an
 *    error the context's message is available from pamd_last_error(); device
 *    detected errors (non-finite energies, population over capacity) are
 *    sticky in device memory and surface at the next synchronising call
 *    (pamd_observables, pamd_get_*), after which the context refuses further
 *    work until pamd_destroy().
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    pamd_md_steps and pamd_resample only enqueue work (asynchronous, no host
 *    synchronisation, capturable into a HIP graph); pamd_init, pamd_observables
 *    and the pamd_get_* / pamd_set_* calls synchronise `stream`.
 *  - Host arrays passed in are only read during the call (copied).
 *  - Device memory is always the caller's: `d_state` and `d_work` of a
 *    context (sizes from pamd_query_sizes), the surrogate's parameters and
 *    workspace (pamd_nn_query_sizes) and the r-RESPA buffers
 *    (pamd_mts_query_sizes), each 256-byte aligned and kept alive until the
 *    object that uses it is destroyed.  The library allocates no device memory
 *    at run time; the only device memory it owns is the fixed staging array of
 *    pamd_nn_forces_static, part of the loaded code object.
 */
#ifndef PAMD_H
#define PAMD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pamd_status;
enum {
    PAMD_OK = 0,
    PAMD_ERR_ARG = 1,        /* null pointer, size mismatch, index out of range, unsupported size */
    PAMD_ERR_HIP = 2,        /* a HIP runtime call failed; message holds hipGetErrorString */
    PAMD_ERR_CAPACITY = 3,   /* resampled population larger than R_cap (or extinct) */
    PAMD_ERR_NONFINITE = 4,  /* NaN / Inf potential energy */
    PAMD_ERR_STATE = 5,      /* call-order violation or context already failed */
    PAMD_ERR_INTERNAL = 6    /* bounds-checked build only (libpamd_check.so): a resampling index
                                (destination offset of the scan, source slot of the gather) was
                                out of range; nothing out of range was written */
};

enum { PAMD_FP64 = 0, PAMD_FP32 = 1 };
/* Copy-number rule of PAMD step 2 (pamd_params.resampling):
 *   NEAREST      c_j = floor(tau_j) + [u_j < frac(tau_j)]: random rounding of the
 *                expected copy numbers; the population size fluctuates around R.
 *   MULTINOMIAL  R independent draws from p_j = tau_j / R (the rule the paper states
 *                after the scheme); the population size stays R.
 *   NONE         c_j = 1: resampling switched off (the paper's "anneal" ablation);
 *                the rescale, recentring and ln Q bookkeeping still run. */
enum { PAMD_RESAMPLE_NEAREST = 0, PAMD_RESAMPLE_MULTINOMIAL = 1, PAMD_RESAMPLE_NONE = 2 };
/* Heat bath of the MD steps (pamd_params.thermostat):
 *   ANDERSEN  velocity Verlet; after each step every atom collides with
 *             probability 1 - exp(-nu dt) and takes a Maxwell-Boltzmann velocity.
 *   LANGEVIN  the paper's stochastic bath (friction gamma = nu, a distinct random
 *             stream per replica) in the B-A-O-A-B velocity-Verlet splitting
 *             (Leimkuhler & Matthews 2013): v += dt/2 F/m; x += dt/2 v;
 *             v = c1 v + sqrt(1 - c1^2) sqrt(kB T/m) xi with c1 = exp(-gamma dt) and
 *             xi from Philox stream 5, counter (slot, step, atom, 5); x += dt/2 v;
 *             F = F(x); v += dt/2 F/m.  Not combined with pamd_set_mts. */
enum { PAMD_THERMOSTAT_ANDERSEN = 0, PAMD_THERMOSTAT_LANGEVIN = 1 };
enum { PAMD_DIELECTRIC_VACUUM = 0, PAMD_DIELECTRIC_4R = 1 };
/* MD layout of a run (pamd_params.layout):
 *   AUTO  register tile when every molecule of the context has at most
 *         PAMD_TILE_ATOMS atoms, else wide;
 *   TILE  register tile: one replica per 16-lane row, four per wavefront, one
 *         persistent launch per run (molecules up to PAMD_TILE_ATOMS atoms);
 *   WIDE  one replica per wavefront; every wide run of a context shares one
 *         persistent launch (FP32 only).  Its LJ coefficients come from a
 *         table over the molecule's distinct (sigma, epsilon) pairs, at most
 *         PAMD_WIDE_LJ_CLASSES of them per molecule.
 * A context may mix both (an autotuner picks per run). */
enum { PAMD_LAYOUT_AUTO = 0, PAMD_LAYOUT_TILE = 1, PAMD_LAYOUT_WIDE = 2 };

#define PAMD_MAX_ATOMS 320   /* FP32; FP64 runs take at most 32 atoms */
#define PAMD_TILE_ATOMS 80   /* the largest molecule of the register-tile layout (PAMD_LAYOUT_*) */
#define PAMD_FORCE_CHUNK 256 /* replicas per pamd_get_forces call */
#define PAMD_WIDE_LJ_CLASSES 25  /* distinct per-atom (sigma, epsilon) pairs of a wide-layout molecule */

/*
 * One molecule (host pointers; all arrays row-major).  Functional form:
 *   bonds      U = 1/2 k (r - r0)^2
 *   angles     U = 1/2 k (theta - theta0)^2                        (theta0 in radians)
 *   dihedrals  U = k (1 + cos(n phi - delta)), delta in {0, pi} (within 1e-9 rad)
 *   LJ         U = s 4 eps_ij ((sigma_ij / r)^12 - (sigma_ij / r)^6),
 *              sigma_ij = (sigma_i + sigma_j) / 2, eps_ij = sqrt(eps_i eps_j)
 *   Coulomb    U = s k_e q_i q_j / r          (dielectric PAMD_DIELECTRIC_VACUUM)
 *              U = s k_e q_i q_j / (4 r^2)    (PAMD_DIELECTRIC_4R: eps(r) = 4 r)
 * Nonbonded pairs: every i < j except 1-2 and 1-3 pairs of the bond graph;
 * 1-4 pairs (three bonds apart) take s = scale14_lj / scale14_coul, others s = 1.
 * Units are the caller's (kB and coulomb_k set them).
 */
typedef struct pamd_system {
    int32_t n_atoms;               /* 1 .. PAMD_MAX_ATOMS */
    int32_t n_bonds, n_angles, n_dihedrals;
    const double* mass;            /* [n_atoms] > 0 */
    const double* charge;          /* [n_atoms] */
    const double* sigma;           /* [n_atoms] */
    const double* epsilon;         /* [n_atoms] >= 0 */
    const int32_t* bond_idx;       /* [n_bonds][2] */
    const double* bond_k;          /* [n_bonds] */
    const double* bond_r0;         /* [n_bonds] */
    const int32_t* angle_idx;      /* [n_angles][3]  (i, centre, k) */
    const double* angle_k;
    const double* angle_theta0;
    const int32_t* dih_idx;        /* [n_dihedrals][4] */
    const double* dih_k;
    const int32_t* dih_n;          /* multiplicity 1..6 */
    const double* dih_delta;
    double scale14_lj, scale14_coul;
    double coulomb_k;
    int32_t dielectric;            /* PAMD_DIELECTRIC_* */
    int32_t reserved;
    double kB;                     /* Boltzmann constant in the caller's units */
    const double* x_init;          /* [n_atoms][3] start configuration of every copy */
} pamd_system;

/* Run parameters. */
typedef struct pamd_params {
    int64_t R_target;              /* population size R (expected copies sum to it) */
    int64_t R_cap;                 /* slots per buffer, >= R_target (fluctuation headroom) */
    double T0;                     /* initial temperature */
    double dt;                     /* MD time step */
    double nu;                     /* Andersen collision frequency, or Langevin friction gamma
                                      (1/time; 0: NVE) */
    uint64_t seed;                 /* Philox key = (seed_lo, seed_hi + run) */
    int32_t precision;             /* PAMD_FP32 (positions, velocities, forces FP32) or PAMD_FP64 */
    int32_t waves_per_block;       /* register-tile kernel: 0 automatic, else 1..16 (from run 0) */
    double V_target;               /* adaptive schedule: normalised weight variance per step */
    double T_final;                /* adaptive schedule: lowest temperature T_N */
    int32_t resampling;            /* PAMD_RESAMPLE_*: how pamd_resample draws the copy numbers */
    int32_t thermostat;            /* PAMD_THERMOSTAT_*: the same for every run of a context */
    int32_t layout;                /* PAMD_LAYOUT_* of this run */
    int32_t wide_waves_per_block;  /* batched wide launch: 0 automatic (4), else 1..4 (from run 0) */
} pamd_params;

/* Population observables of one run (PAMD step 4), all FP64. */
typedef struct pamd_obs {
    double T;                      /* current bath temperature T_i */
    double T_prev;                 /* previous temperature T_{i-1} */
    double lnQ_last;               /* ln Q_i of the last resampling */
    double sum_lnQ;                /* sum_i ln Q_i = estimate of ln Z(T_i) - ln Z(T_0) */
    double V_last;                 /* normalised weight variance R sum p_j^2 - 1 of the last step */
    double E_mean;                 /* <E_pot> */
    double E2_mean;                /* <E_pot^2> */
    double K_mean;                 /* <E_kin> */
    double T_measured;             /* 2 <E_kin> / (3 N kB) */
    double Cv;                     /* (<E^2> - <E>^2) / (kB T)^2 = heat capacity / kB */
    int64_t R;                     /* current population size R_i */
    int64_t families;              /* distinct ancestors among the R_i copies */
    int64_t temp_index;            /* i */
    int64_t step;                  /* MD steps done since pamd_init */
    int32_t error;                 /* sticky device error code (PAMD_ERR_*) or 0 */
    int32_t reserved;
} pamd_obs;

typedef struct pamd_ctx pamd_ctx;

/* Device bytes needed for `n_runs` independent runs (sys[n_runs], p[n_runs]).
 * Pure host function.  PAMD_ERR_ARG for a descriptor out of range, runs of
 * different precision or bath, or a molecule of the wide layout with more
 * than PAMD_WIDE_LJ_CLASSES distinct (sigma, epsilon) pairs (pamd_init
 * returns the same). */
pamd_status pamd_query_sizes(const pamd_system* sys, int32_t n_runs, const pamd_params* p,
                             size_t* state_bytes, size_t* work_bytes);

/* PAMD step 1.  Copies topology and parameters to the device, derives the
 * exclusion / 1-4 lists from the bonds, builds the pair-parameter tables,
 * fills R_target slots per run with x_init and Maxwell-Boltzmann(T0)
 * velocities (Philox stream 3), ancestor = slot.  Equilibration at T0 is the
 * caller's pamd_md_steps.  Synchronises `stream`. */
pamd_status pamd_init(const pamd_system* sys, int32_t n_runs, const pamd_params* p,
                      void* d_state, size_t state_bytes, void* d_work, size_t work_bytes,
                      void* stream, pamd_ctx** out);

/* PAMD step 3.  n_steps >= 0 NVT steps of every copy of every run at the
 * run's current T with the context's bath (velocity Verlet with Andersen
 * collisions after each step, or the Langevin B-A-O-A-B step); leaves E_pot
 * and E_kin of the final configurations (n_steps = 0 only evaluates them).
 * With a surrogate attached (pamd_set_mts) the same time span is covered by
 * r-RESPA outer steps.  A run whose sticky device error is set when the call's
 * work starts keeps its state (positions, velocities, energies, step counter).
 * Asynchronous. */
pamd_status pamd_md_steps(pamd_ctx* ctx, int32_t n_steps, void* stream);

/* PAMD step 2.  T_next: host [n_runs]; T_next[r] > 0 is the next temperature
 * of run r, T_next[r] == 0 (or T_next == NULL) chooses it adaptively (largest
 * step with normalised weight variance <= V_target, not below T_final), and
 * T_next[r] < 0 takes the next entry of the run's device schedule
 * (pamd_set_schedule; the last entry repeats once it is reached).
 * d_uniforms: device [n_runs][R_cap] doubles in [0,1), or NULL to draw them
 * from Philox.  Copy numbers follow the run's pamd_params.resampling with
 * tau_j = R_target w_j / sum w, w_j = exp(-dbeta (E_j - min E)):
 *   NEAREST      c_j = floor(tau_j) + [u_j < frac(tau_j)]; u_j = d_uniforms[r][j]
 *                or Philox stream 2, counter (j, i, 0, 2);
 *   MULTINOMIAL  draw k = 0 .. R_target-1 picks the first j with W_j > u_k W_{R-1},
 *                W_j = w_0 + ... + w_j (FP64 running sums, in chunk order; if
 *                rounding leaves no such j, the first j with W_j == W_{R-1});
 *                u_k = d_uniforms[r][k] or Philox stream 4, counter (k, i, 0, 4);
 *   NONE         c_j = 1;
 * where i is the index of the new temperature.  Copies of source j take
 * consecutive new slots in increasing j; velocities
 * are scaled by sqrt(T_i / T_{i-1}) and each copy is translated so its centre
 * of mass sits at the origin.  Asynchronous; an over-capacity population
 * leaves the state unchanged and raises PAMD_ERR_CAPACITY at the next sync.
 * PAMD_ERR_STATE (the context stays usable) when no pamd_md_steps call, or
 * pamd_set_state with energies, has given the population its energies. */
pamd_status pamd_resample(pamd_ctx* ctx, const double* T_next, const double* d_uniforms,
                          void* stream);

/* PAMD steps 2 and 3 as HIP graphs.  Captures into graph `slot` (0..3), on
 * `stream` (must not be the null stream), the work selected by `parts`:
 * 1 = one resampling of every run (mode 0: adaptive temperature, mode 1: next
 * entry of the device schedule), 2 = n_steps MD steps of every run, 3 = both
 * in that order; then instantiates it (replacing that slot's previous graph).
 * Every value that changes between temperatures lives in device memory, so
 * one capture is replayed for the whole anneal.  The graphs hold kernels only. */
pamd_status pamd_graph_capture(pamd_ctx* ctx, int32_t slot, int32_t parts, int32_t n_steps, int32_t mode,
                               void* stream);

/* Replays graph `slot` on `stream` (any stream).  Asynchronous. */
pamd_status pamd_graph_launch(pamd_ctx* ctx, int32_t slot, void* stream);

/* Device temperature schedule of `run` (T[0] = T0 ... T[n-1] = T_N; n <= 4096),
 * used by pamd_resample with T_next[run] < 0 and by graphs of mode 1.
 * Synchronises `stream`. */
pamd_status pamd_set_schedule(pamd_ctx* ctx, int32_t run, const double* T, int32_t n, void* stream);

/* PAMD step 4.  out: host [n_runs].  Synchronises `stream`. */
pamd_status pamd_observables(pamd_ctx* ctx, pamd_obs* out, void* stream);

/* ---- inspection / checkpoint calls (synchronising) ---------------------- */

/* Forces and potential energies at the current positions of replicas
 * [r0, r0 + count) of `run`, count <= PAMD_FORCE_CHUNK.
 * host_F: [count][n_atoms][3], host_E: [count] (either may be NULL). */
pamd_status pamd_get_forces(pamd_ctx* ctx, int32_t run, int64_t r0, int32_t count,
                            double* host_F, double* host_E, void* stream);

/* Per-run scalars that travel with a checkpoint. */
typedef struct pamd_run_scalars {
    double T, T_prev, sum_lnQ, lnQ_last;
    int64_t R;
    uint32_t step, temp_index;
} pamd_run_scalars;

/* Copy the current population of `run` to the host.  Arrays have room for
 * R_cap replicas; x, v: [R][n_atoms][3]; E_pot, E_kin: [R]; ancestor: [R].
 * Any pointer may be NULL.  After a device-side error the outputs are still
 * filled and that error is returned: on PAMD_ERR_CAPACITY the population and
 * scalars the failed resampling step started from, on PAMD_ERR_NONFINITE the
 * population holding the non-finite energy; the context then accepts no
 * further step (PAMD_ERR_STATE), so a caller recovers by moving the state to a
 * new context. */
pamd_status pamd_get_state(pamd_ctx* ctx, int32_t run, double* x, double* v, double* E_pot,
                           double* E_kin, int32_t* ancestor, pamd_run_scalars* scalars,
                           void* stream);

/* Replace the population of `run` (R = scalars->R <= R_cap copies).  x, v
 * required; E_pot and ancestor optional (NULL: zeros / slot index). */
pamd_status pamd_set_state(pamd_ctx* ctx, int32_t run, const double* x, const double* v,
                           const double* E_pot, const int32_t* ancestor,
                           const pamd_run_scalars* scalars, void* stream);

/* Copy numbers c_j of the last resampling of `run` (host [R_{i-1}]). */
pamd_status pamd_get_counts(pamd_ctx* ctx, int32_t run, int32_t* host_c, int64_t* n, void* stream);

/* Launch shape chosen at init: waves per workgroup, workgroups and LDS bytes
 * of the batched wide launch if the context has one, else of the
 * register-tile kernel (informational). */
pamd_status pamd_launch_info(const pamd_ctx* ctx, int32_t* waves_per_block, int32_t* blocks,
                             int32_t* lds_bytes);

/* Layout (PAMD_LAYOUT_TILE or PAMD_LAYOUT_WIDE) and launch shape of the
 * kernel that advances `run`.  Host function. */
pamd_status pamd_run_launch(const pamd_ctx* ctx, int32_t run, int32_t* layout, int32_t* waves_per_block,
                            int32_t* blocks, int32_t* lds_bytes);

void pamd_destroy(pamd_ctx* ctx);
const char* pamd_last_error(const pamd_ctx* ctx);

/*
 * Population analysis (host, FP64, no context, no GPU; host pointers only).
 *
 * Copies made by resampling are correlated, which the errors of population
 * averages must respect (the paragraph on correlations after resampling:
 * binning over the population).  A family is all copies descending from one
 * initial replica (equal `ancestor`, as pamd_get_state returns it).
 *   mean        (1/R) sum_j O_j
 *   naive_se    sqrt( sum_j (O_j - mean)^2 / (R (R - 1)) )        (0 for R = 1)
 *   family_se   sqrt( sum_f (sum_{j in f} (O_j - mean))^2 / (R (R - 1)) )
 *   rho_t       R sum_f nu_f^2,  nu_f = n_f / R   (1 without resampling)
 *   family_entropy  -sum_f nu_f ln nu_f          (exp of it: effective families)
 * PAMD_ERR_ARG for null pointers or R < 1, PAMD_ERR_NONFINITE for a NaN/Inf value.
 */
typedef struct pamd_family_stats {
    double mean, naive_se, family_se, rho_t, family_entropy;
    int64_t families;
} pamd_family_stats;
pamd_status pamd_family_error(const double* O, const int32_t* ancestor, int64_t R, pamd_family_stats* out);

/* Standard error of the mean from bins of `bin` consecutive slots (copies of
 * one source occupy consecutive slots after each resampling): the first
 * floor(R / bin) complete bins, se^2 = sum_k (m_k - m)^2 / ((n_b - 1) n_b).
 * PAMD_ERR_ARG unless bin >= 1 and R / bin >= 2. */
pamd_status pamd_binning_error(const double* O, int64_t R, int64_t bin, double* se);

/*
 * Multiple-histogram (WHAM) self-consistency in per-sample form (the paragraph
 * on the recorded normalisers: sum ln Q gives ln Z(T_i) - ln Z(T_0) and the
 * starting values).  Samples: E[n_samples[0]] at beta[0], then E[n_samples[1]]
 * at beta[1], ... (e.g. the population's E_pot at each temperature).  With
 *   ln D(E) = logsumexp_l (ln N_l - beta_l E - ln Z_l),
 * each iteration sets ln Z_k = logsumexp_samples (-beta_k E - ln D(E)), shifted
 * so that ln Z_0 keeps its input value, until the largest change is < tol or
 * max_iter iterations.  lnZ[n_temps]: in = starting values (e.g. the running
 * sum of ln Q), out = refined.  *iterations (optional) = iterations done.
 * Deterministic for any thread count (fixed chunk order).
 */
pamd_status pamd_wham(int32_t n_temps, const double* beta, const int64_t* n_samples, const double* E,
                      double* lnZ, int32_t max_iter, double tol, int32_t* iterations);

/* <E> and <E^2> at inverse temperature beta_q by reweighting all samples with
 * exp(-beta_q E) / D(E), D from converged ln Z (same sample layout). */
pamd_status pamd_wham_average(int32_t n_temps, const double* beta, const int64_t* n_samples, const double* E,
                              const double* lnZ, double beta_q, double* E_mean, double* E2_mean);

/* Roofline calibration (no context): runs a kernel of independent FP32 FMAs
 * (v_fma_f32 with VGPR operands only; every kernel of this library is built
 * without packed FP32 instructions) over the whole GPU three times and returns
 * in *tflops the best rate in TFLOP/s (FMA = 2 flop): the ceiling of an FP32
 * VALU-bound kernel of this library.  d_sink: device pointer to one float the
 * kernel may write.  Synchronises `stream`. */
pamd_status pamd_fp32_fma_rate(float* d_sink, double* tflops, void* stream);

/* Issue cost of single VALU instruction forms (no context; measurement
 * infrastructure behind the roofline reading of the MD kernels): for each form
 * a kernel of eight independent chains per lane of that one instruction,
 * `waves_per_simd` (1, 2, 4 or 8) waves on every SIMD.  Returns in
 * cycles_per_instr[PAMD_VALU_FORMS] the shader cycles per wave64 instruction
 * per SIMD (issue time; lower is faster) and in *clock_ghz the shader clock
 * measured from one wave alone on its SIMD (s_memtime over the launch time).
 * d_sink: device buffer of at least 16 bytes the kernels may write.
 * Synchronises `stream`; about 10 ms. */
enum {
    PAMD_VALU_FMA_VGPR = 0,   /* v_fma_f32, all operands VGPRs */
    PAMD_VALU_FMA_SGPR = 1,   /* v_fma_f32 with one SGPR operand */
    PAMD_VALU_FMAC_VOP2 = 2,  /* v_fmac_f32_e32 */
    PAMD_VALU_MUL_VOP2 = 3,   /* v_mul_f32_e32 */
    PAMD_VALU_ADD_DPP = 4,    /* v_add_f32 with a DPP row-rotated source */
    PAMD_VALU_MOV_DPP = 5,    /* v_mov_b32 with DPP row rotation */
    PAMD_VALU_RCP = 6,        /* v_rcp_f32 (transcendental unit) */
    PAMD_VALU_FORMS = 7
};
pamd_status pamd_valu_issue_rates(float* d_sink, int32_t waves_per_simd, double* cycles_per_instr,
                                  double* clock_ghz, void* stream);

/* ---- learned multiple-time-step (MTS) surrogate --------------------------
 * Not part of the paper's scheme: an optional acceleration of the MD update
 * of step 3 by r-RESPA.  A network shared by all atoms maps Gaussian radial
 * features of an atom's nonbonded partners to an atomic energy,
 *   G_i[t][k] = sum over partners j of type t of exp(-(r_ij - mu_k)^2 / (2 s^2)),
 *   mu_k = 0.1 + k s, s = 1.1 / 31 (positions in nm), k = 0..31, t = 0..7,
 *   E_i = w3 . silu(W2^T silu(W1^T G_i + b1) + b2) + b3,  E_NN = sum_i E_i,
 *   F_NN = -grad E_NN,  silu(x) = x / (1 + exp(-x)),
 * where the partners are the nonbonded pair set (1-2 and 1-3 pairs excluded,
 * 1-4 pairs included unscaled).  Parameters are FP32 masters with BF16 copies
 * for the matrix cores (FP32 accumulation); features and hidden activations
 * are rounded to BF16, so forces agree with an exact evaluation to about 1e-2
 * relative.  All device arrays below are FP32 [n_conf][n_atoms][3] unless
 * stated; calls marked asynchronous only enqueue work on `stream`. */
#define PAMD_NN_TYPES 8
#define PAMD_NN_FEATURES 256
#define PAMD_NN_HIDDEN 128
/* flat parameter vector: W1 [256][128], b1 [128], W2 [128][128], b2 [128], w3 [128], b3 [1] */
#define PAMD_NN_PARAMS 49537

typedef struct pamd_nn pamd_nn;

/* Device bytes of a surrogate for molecules of n_atoms (1..80) atoms whose
 * inference, loss and training calls take at most max_conf configurations:
 * FP32 parameters, gradient and Adam moments, the BF16 weight copies, and a
 * workspace of about 7.3 KB per (configuration, atom) row plus 4.3 MB of
 * split-K partial sums.  Pure host function; PAMD_ERR_ARG for sizes out of range. */
pamd_status pamd_nn_query_sizes(int32_t n_atoms, int64_t max_conf, size_t* bytes);

/* Surrogate for molecule `sys` (its atom count and bonds are used) with
 * atom_type[n_atoms] in 0..7, living in the caller's device buffer d_mem
 * (mem_bytes >= pamd_nn_query_sizes(n_atoms, max_conf), 256-byte aligned,
 * kept alive until pamd_nn_destroy).  Parameters start at zero (F_NN = 0).
 * Synchronises `stream`.  PAMD_ERR_ARG for a bad type, bond index, size or
 * buffer; the calls below refuse batches larger than max_conf (PAMD_ERR_ARG). */
pamd_status pamd_nn_create(const pamd_system* sys, const int32_t* atom_type, int64_t max_conf, void* d_mem,
                           size_t mem_bytes, void* stream, pamd_nn** out);

/* Host params[PAMD_NN_PARAMS] -> device masters and BF16 copies; resets the
 * Adam state.  Synchronises `stream`. */
pamd_status pamd_nn_set_weights(pamd_nn* nn, const float* params, void* stream);

/* Device masters -> host params[PAMD_NN_PARAMS].  Synchronises `stream`. */
pamd_status pamd_nn_get_weights(pamd_nn* nn, float* params, void* stream);

/* E_NN (d_E [n_conf], may be NULL) and F_NN (d_F) of the configurations
 * d_x, n_conf <= max_conf.  Asynchronous. */
pamd_status pamd_nn_forces(pamd_nn* nn, int64_t n_conf, const float* d_x, float* d_F, float* d_E, void* stream);

/* pamd_nn_forces for callers that cannot allocate device memory or size a
 * workspace (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation): the same inputs, outputs and results (the same
 * kernels), but the features and dE/dG rows are staged in a fixed 16 MiB
 * device array of the library (one per GPU, set up by pamd_nn_create, held
 * until the process ends) instead of the surrogate's workspace.  Requires
 * n_conf * n_atoms <= PAMD_NN_STATIC_ROWS (PAMD_ERR_ARG beyond, with the
 * sizes in pamd_nn_last_error).  Every call on one GPU uses that one array:
 * calls that overlap in time on one GPU (several streams or threads) race.
 * Allocates nothing.  Asynchronous. */
#define PAMD_NN_STATIC_ROWS 16000
pamd_status pamd_nn_forces_static(pamd_nn* nn, int64_t n_conf, const float* d_x, float* d_F, float* d_E,
                                  void* stream);

/* Force-matching loss L = mean over configurations, atoms and components of
 * (F_NN - F_target)^2 into device float *d_loss, and its gradient with
 * respect to the FP32 parameters into d_grad (device [PAMD_NN_PARAMS]; NULL:
 * loss only).  The gradient is reverse mode through the forward-mode
 * derivative of the network along the features' derivative in the direction
 * dL/dF.  Asynchronous. */
pamd_status pamd_nn_loss_grad(pamd_nn* nn, int64_t n_conf, const float* d_x, const float* d_F_target,
                              float* d_loss, float* d_grad, void* stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, step size lr) on that
 * gradient of the batch; the batch loss before the step goes to *d_loss
 * (may be NULL).  Asynchronous. */
pamd_status pamd_nn_train_step(pamd_nn* nn, int64_t n_conf, const float* d_x, const float* d_F_target, float lr,
                               float* d_loss, void* stream);

/* Frees the host object; the caller's device buffer is untouched. */
void pamd_nn_destroy(pamd_nn* nn);
const char* pamd_nn_last_error(const pamd_nn* nn);

/* Positions and exact nonbonded (LJ + Coulomb) forces of replicas
 * [r0, r0 + count) of `run` of an FP32 context into device arrays d_x and
 * d_F_nb (training data of the surrogate).  Asynchronous. */
pamd_status pamd_export_configs(pamd_ctx* ctx, int32_t run, int64_t r0, int64_t count, float* d_x, float* d_F_nb,
                                void* stream);

/* Device bytes of the r-RESPA buffers of `ctx` (every run: features and
 * dE/dG rows of R_cap x n_atoms configurations-atoms in BF16, row energies
 * and F_NN), about 1 KB per replica-atom.  Host function. */
pamd_status pamd_mts_query_sizes(pamd_ctx* ctx, size_t* bytes);

/* Switch pamd_md_steps of an FP32 context to r-RESPA with surrogate `nn`
 * (every run must have nn's atom count): per outer step of Dt = outer_ratio dt
 *   v += Dt/2 (F_nb - F_NN) / m;
 *   outer_ratio velocity-Verlet steps of dt with the force F_bonded + F_NN;
 *   v += Dt/2 (F_nb - F_NN) / m;
 *   Andersen collisions with probability 1 - exp(-nu Dt) per atom, drawn
 *   with the MD step counter at the start of the outer step as Philox step word.
 * n_steps of pamd_md_steps must then be a multiple of outer_ratio; energies
 * for the resampling weights stay exact.  nn = NULL switches back to plain
 * velocity Verlet (d_mem ignored).  d_mem: the caller's device buffer of
 * mem_bytes >= pamd_mts_query_sizes bytes (256-byte aligned) for the per-run
 * buffers; it and nn must stay alive while attached.  Synchronises `stream`. */
pamd_status pamd_set_mts(pamd_ctx* ctx, pamd_nn* nn, int32_t outer_ratio, void* d_mem, size_t mem_bytes,
                         void* stream);

#ifdef __cplusplus
}
#endif
#endif /* PAMD_H */
