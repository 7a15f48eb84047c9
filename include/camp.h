/*
 * camp.h -- C ABI of the MI355X-native batched stiff multiphase chemistry solver.
 *
 * The operation: every grid cell's gas + aerosol-phase chemistry is an independent stiff
 * ODE system dy/dt = f(y) over one host time step dt. The host model creates one object
 * per mechanism, sets externally computed rates, passes temperature, pressure,
 * concentrations, aerosol state and dt, asks for a solve, and reads the state back
 * (paper Sect. 2.1 CampCore; Sect. 2.4.2 runtime workflow). Each cell is integrated with
 * variable-order BDF and Newton iteration over a sparse LU (Sect. 2.4.1). Here all cells
 * of a call are solved together on one GPU.
 *
 * Conventions
 *  - Every function returns camp_status (0 = OK, < 0 = error). No exception crosses the
 *    ABI. On error, camp_last_error() returns a thread-local message.
 *  - Concentrations are mol m^-3 of air. Arrays of per-cell data are row-major
 *    [cells][...] (one cell's values contiguous), double precision.
 *  - "host" pointers are ordinary CPU memory; "device" pointers are HIP device memory
 *    (e.g. torch.Tensor.data_ptr() of a CUDA tensor). Streams are hipStream_t passed as
 *    void* (NULL = the default stream).
 *  - The library never frees or retains caller memory after a call returns (the device
 *    calls are stream-ordered: inputs must stay valid until the stream reaches the call).
 *
 * State layout (n_state values per cell): gas species in the order given to
 * camp_mech_load, then for each phase in order, for each of its instances in order, the
 * phase's species in the order the phase lists them (paper Sect. 2.2.3: a phase's
 * species and chemistry are identical in every instance).
 */
#ifndef CAMP_H
#define CAMP_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CAMP_OK = 0,
  CAMP_EINVAL = -1,   /* invalid argument or mechanism description               */
  CAMP_ENOMEM = -2,   /* host or device allocation failed                         */
  CAMP_EDEVICE = -3,  /* HIP runtime error or no usable device                    */
  CAMP_ESOLVE = -4    /* at least one cell failed; see the per-cell status array  */
} camp_status;

/* Per-cell status codes written by the solve calls. A failed cell's state is restored
 * to its input values. */
enum {
  CAMP_CELL_OK = 0,
  CAMP_CELL_MAX_STEPS = 1,    /* more step attempts than opts.max_steps            */
  CAMP_CELL_H_MIN = 2,        /* step below opts.h_min or the roundoff floor of t  */
  CAMP_CELL_ERR_FAIL = 3,     /* 10 consecutive local error test failures          */
  CAMP_CELL_NEWTON_FAIL = 4,  /* 10 consecutive Newton convergence failures        */
  CAMP_CELL_NONFINITE = 5     /* non-finite rate constant, forcing or weight       */
};

/* Process types (paper Sect. 2.2.1, tables of Process-extending classes).
 * p[] meanings:
 *  ARRHENIUS            gas. k = A exp(-Ea/(kb T)) (T/D)^B (1 + E P).
 *                       p = {A [(molecule cm^-3)^-(n_r-1) s^-1], Ea/kb [K], B, D [K], E [Pa^-1]}.
 *  PHOTOLYSIS           gas, 1 reactant. p = {J0 [s^-1], sza_flag}. sza_flag != 0 scales
 *                       J0 by max(0, cos sza) of the cell. Externally settable.
 *  EMISSION             gas, 0 reactants, 1 product. p = {E [mol m^-3 s^-1]}. Settable.
 *  FIRST_ORDER_LOSS     gas, 1 reactant, 0 products. p = {k [s^-1]}. Settable.
 *  CONDENSED_ARRHENIUS  reactants/products in .phase, applied in every instance.
 *                       p = {A, Ea/kb, B, D, E, aqueous}. aqueous != 0: k in M^-(n_r-1) s^-1
 *                       acting on molarities (phase volume = mass / density); else in
 *                       (mol m^-3 air)^-(n_r-1) s^-1.
 *  HENRY_TRANSFER       react[0] gas species G, prod[0] species A of .phase.
 *                       p = {H298 [M Pa^-1], C [K]}; H(T) = H298 exp(C (1/T - 1/298)).
 *                       Condensation k_c = 4 pi r D_g f_FS(Kn, alpha) N (Fuchs-Sutugin);
 *                       evaporation k_c / (H 1000 V R T).
 *  SIMPOL_TRANSFER      as HENRY_TRANSFER; p = {B1, B2, B3, B4, raoult}, log10 p0[atm] =
 *                       B1/T + B2 + B3 T + B4 ln T; evaporation k_c p0 101325 / (R T n_abs),
 *                       n_abs = mass / mw_absorber of the instance. raoult = 1 takes the
 *                       full Raoult mole fraction instead (a Parameter, Sect. 2.2.2): the
 *                       evaporation rate is k_c p0 101325 / (R T) * y_A / n_tot with
 *                       n_tot = n_abs + the sum of every condensed species of the instance
 *                       (a state-dependent amount, whose derivative enters the Jacobian);
 *                       0 when n_tot = 0. raoult must be 0 or 1.
 *  TROE                 gas fall-off reaction: k = k0[M] / (1 + k0[M]/kinf)
 *                       Fc^(1 / (1 + (1/N) log10(k0[M]/kinf)^2)), with k0 and kinf of
 *                       Arrhenius form A exp(-Ea/(kb T)) (T/300)^B and [M] = P / (kb T) the
 *                       number density of air [molecule cm^-3].
 *                       p = {A0, Ea0/kb, B0, Ainf, Eainf/kb, Binf, Fc, N}.
 *  CUSTOM_H2O2          gas: k = k1 + k2[M] (k1, k2 of Arrhenius form as for TROE).
 *                       p = {A1, Ea1/kb, B1, A2, Ea2/kb, B2}.
 *  CUSTOM_OH_HNO3       gas: k = k0 + k3[M] / (1 + k3[M]/k2).
 *                       p = {A0, Ea0/kb, B0, A2, Ea2/kb, B2, A3, Ea3/kb, B3}.
 *  WENNBERG_TUNNELING   gas: k = A exp(-B/T) exp(C/T^3). p = {A, B [K], C [K^3]}.
 *                       The gas-phase forms above give k in (molecule cm^-3)^-(n_r-1) s^-1.
 *  AQUEOUS_REVERSIBLE   reactants <-> products in .phase (every instance), on molarities
 *                       (phase volume = mass / density): reverse k_r [M^-(n_p-1) s^-1],
 *                       equilibrium K = A exp(C (1/T - 1/298)) [M^(n_p-n_r)], forward
 *                       K k_r. Products distinct with yield 1. p = {A, C [K], k_r}. Expands to
 *                       a forward and a reverse reaction per instance.
 * A phase instance with zero mass has all its rate constants equal to 0.
 */
enum {
  CAMP_RXN_ARRHENIUS = 1,
  CAMP_RXN_PHOTOLYSIS = 2,
  CAMP_RXN_EMISSION = 3,
  CAMP_RXN_FIRST_ORDER_LOSS = 4,
  CAMP_RXN_CONDENSED_ARRHENIUS = 5,
  CAMP_RXN_HENRY_TRANSFER = 6,
  CAMP_RXN_SIMPOL_TRANSFER = 7,
  CAMP_RXN_TROE = 8,
  CAMP_RXN_CUSTOM_H2O2 = 9,
  CAMP_RXN_CUSTOM_OH_HNO3 = 10,
  CAMP_RXN_WENNBERG_TUNNELING = 11,
  CAMP_RXN_AQUEOUS_REVERSIBLE = 12
};

typedef struct {
  const char* name;      /* may be NULL                                              */
  int phase;             /* -1 gas, else index into the phase array                  */
  double mw_kg_mol;      /* gas species: molecular weight (used by phase transfer);  */
                         /* species of a phase whose radius follows the state: the   */
                         /* molecular weight that converts moles to particle volume   */
  double diff_m2_s;      /* gas species: gas-phase diffusion coefficient             */
  double accom;          /* gas species: mass accommodation coefficient              */
} camp_species;

typedef struct {
  const char* name;       /* may be NULL                                             */
  int n_species;          /* >= 1                                                    */
  const int* species;     /* [n_species] species ids, each with .phase == this index */
  int n_instances;        /* >= 1 (modes, sections or particles)                     */
  double density_kg_m3;   /* > 0                                                     */
  double mw_absorber_kg_mol; /* > 0, SIMPOL absorbing-mass molar mass                */
  int radius_from_state;  /* 0: particle radius from the environment. 1: the particles */
                          /* grow with the condensed species (an aerosol representation */
                          /* computing the radius from particle mass, Sect. 2.2.3): the */
                          /* environment's radius and mass give the particle core and   */
                          /* number concentration N_p = m / (rho 4/3 pi r^3), and a     */
                          /* transfer's rate is evaluated at r(y) = (3 V / (4 pi N_p))^  */
                          /* (1/3), V = m / rho + sum of y_j MW_j / rho over the phase's  */
                          /* species (which then need mw_kg_mol > 0). SIMPOL transfer   */
                          /* only (Henry transfer into such a phase is rejected).       */
} camp_phase;

typedef struct {
  int type;               /* CAMP_RXN_*                                              */
  int phase;              /* condensed/transfer: phase index; gas: ignored           */
  int n_react;            /* 0..3 (repeats allowed: 2A -> B lists A twice)           */
  int react[3];           /* species ids                                             */
  int n_prod;             /* 0..3, distinct                                          */
  int prod[3];
  double yield[3];        /* molar yields of the products                            */
  double p[10];           /* type-specific parameters, see above                     */
} camp_reaction;

typedef struct camp_mech camp_mech;

/* Compile a mechanism: validate it, expand phases over instances, assign state ids, take
 * the union of the Jacobian elements every process touches plus the diagonal (paper
 * table of Process functions: get_used_jacobian_elements, update_ids), choose a
 * fill-reducing elimination order, compute the LU fill symbolically once, and build the
 * level-scheduled elimination and solve tables. All inputs are deep-copied; the caller
 * may free them on return. Host-only work: no device is touched until the first solve.
 * Errors: CAMP_EINVAL (bad ids, counts, non-finite or negative parameters, transfer
 * partner not gas-phase, phase without species or instances), CAMP_ENOMEM. */
int camp_mech_load(const camp_reaction* rxns, int n_rxn, const camp_species* species,
                   int n_species, const camp_phase* phases, int n_phases, camp_mech** out);

/* Compile a mechanism from its JSON description (paper Sect. 2.3: run-time configuration of
 * species, phases and processes without recompiling). `text` is a NUL-terminated UTF-8 JSON
 * document: {"species": [...], "phases": [...], "aerosol representation": {"instances":
 * {phase: count}}, "processes": [...]}; the keys of every element and process type are
 * listed at the top of csrc/mech_json.cpp. Names are resolved to ids, then camp_mech_load
 * runs. Errors: CAMP_EINVAL with the offending element in camp_last_error (malformed JSON,
 * unknown species, phase or type, missing parameters, or any camp_mech_load validation). */
int camp_mech_load_json(const char* text, camp_mech** out);

/* Serialize a compiled mechanism (every table the engines read) into one buffer, so other
 * processes or ranks load it without the host compile (paper Sect. 2.1: the core object is
 * packed on one process and unpacked on others). With buf NULL only *size (bytes needed) is
 * written; else capacity must be at least that (CAMP_EINVAL otherwise). Host memory. */
int camp_mech_pack(const camp_mech* mech, void* buf, size_t capacity, size_t* size);

/* Rebuild a mechanism from camp_mech_pack's buffer (same library format version). The
 * buffer is checked for magic, version, length and checksum and its tables for internal
 * consistency; a buffer from any other source is rejected with CAMP_EINVAL. The checksum
 * guards against accidental damage, not against a buffer crafted to pass it: the contents
 * of the index tables are trusted. The caller may free buf on return. Device tables upload
 * on first use, as for camp_mech_load. */
int camp_mech_unpack(const void* buf, size_t size, camp_mech** out);

typedef struct {
  int n_state;          /* N: state values per cell                                  */
  int n_gas;
  int n_instances;      /* total phase instances                                     */
  int n_rxn_expanded;   /* R: generalized mass-action reactions after expansion      */
  int n_external;       /* externally settable processes (rate_override columns)     */
  int nnz_pattern;      /* Jacobian pattern incl. diagonal, before fill              */
  int nnz_fill;         /* Z: LU pattern after fill                                  */
  long long lu_pairs;   /* U: multiply-subtract pairs of one LU factorization        */
  int lu_levels;        /* dependency levels of the factorization                    */
  int fwd_levels;       /* dependency levels of the forward solve                    */
  int bwd_levels;       /* dependency levels of the backward solve                   */
  int n_partials;       /* sum over reactions of reactant occurrences                */
  int n_terms;          /* forcing terms (species x reaction with nonzero net coef)  */
  int n_jac_contrib;    /* Jacobian contributions                                    */
  int tail_k;           /* size of the dense trailing block of the filled pattern        */
  int nnz_lu;           /* entries of the symbolic LU fill (nnz_fill less the zeros the  */
                        /* dense trailing block adds)                                    */
} camp_mech_info_t;

int camp_mech_info(const camp_mech* mech, camp_mech_info_t* info);

/* Export the compiled structure (for validation). Any pointer may be NULL.
 *  perm[N]       : elimination position t holds state index perm[t]
 *  row_ptr[N+1], col[Z] : filled pattern, CSR in elimination order (cols in elimination
 *                  order, ascending); value slot s of the device matrices is CSR entry s.
 *  pattern0[Z]   : 1 if the slot is in the unfilled pattern, 0 if it is fill. */
int camp_mech_export(const camp_mech* mech, int* perm, int* row_ptr, int* col, int* pattern0);

/* The fused kernel's table layout for lanes_per_cell (64, 128 or 256): dense tail size,
 * dependency levels of the forward sweep, backward sweep and factorization it runs (the
 * Gauss-Jordan steps of the tail come on top of lu_levels), and bytes of its table block.
 * Any output pointer may be NULL. */
int camp_mech_layout_info(const camp_mech* mech, int lanes_per_cell, int* tail_k, int* fwd_levels,
                          int* bwd_levels, int* lu_levels, int* staged_bytes);

/* The autotuner's cached launch choice for (mechanism, current device, size bucket of
 * n_cells): engine, lanes per cell, launch mode (camp_opts.stage_tables), cells per
 * workgroup and persistent workgroups per CU (0: one workgroup per cell batch). CAMP_EINVAL
 * if no engine-AUTO solve of that size bucket has run on this device. Outputs may be NULL. */
int camp_tuned_launch(camp_mech* mech, int n_cells, int* engine, int* lanes_per_cell,
                      int* launch_mode, int* cells_per_wg, int* wg_per_cu);

/* Validation: runs the fused kernel's factor-and-solve table program on the host, in
 * order, for one matrix (paper Sect. 2.4.1: the sparse direct solve of each Newton
 * iteration). m[Z] holds a Newton matrix in the slot order of camp_mech_export and is
 * overwritten with the factors (the pivot reciprocals, row-scaled U and, with the dense
 * tail, the inverse of the trailing block's Schur complement); x[N] holds the right-hand
 * side in elimination order (position t is state perm[t]) and is overwritten with the
 * solution. lanes_per_cell (64, 128 or 256) selects the term-list layout; dense_tail = 0
 * selects the plain layout of the single-step entry points (64 only). Host memory only.
 * Returns CAMP_ESOLVE on a zero or non-finite pivot, CAMP_EINVAL on bad arguments. */
int camp_emulate_factor_solve(const camp_mech* mech, int lanes_per_cell, int dense_tail,
                              double* m, double* x);

void camp_mech_free(camp_mech* mech);

/* Per-cell environment. All arrays [cells] or [cells][n_instances] row-major.
 * radius_m / aer_mass_kg_m3 may be NULL when the mechanism has no phases.
 * cos_sza may be NULL (treated as 1). rate_override may be NULL; else [cells][n_external]
 * values that replace the configured rates of the photolysis, emission and loss
 * processes, in the order those processes appear in the reaction array (paper Sect. 2.4.2:
 * Process-connection objects). */
typedef struct {
  const double* T_K;
  const double* P_Pa;
  const double* cos_sza;
  const double* radius_m;
  const double* aer_mass_kg_m3;
  const double* rate_override;
} camp_env;

/* Solver engines. */
enum {
  CAMP_ENGINE_AUTO = 0,          /* the autotuner's choice for (mechanism, cell count)  */
  CAMP_ENGINE_PLAIN = 1,         /* one lane per cell, separate kernels per BDF phase   */
  CAMP_ENGINE_FUSED_WAVE = 2,    /* persistent fused kernel, one wavefront per cell,    */
                                 /* matrix and vectors resident in LDS                  */
  CAMP_ENGINE_FUSED_LANE = 3     /* persistent fused kernel, one lane per cell,         */
                                 /* cell-interleaved matrices streamed from HBM         */
};

typedef struct {
  int max_order;        /* 1..5 (default 5)                                           */
  int max_steps;        /* step attempts per cell per call (default 100000)           */
  int newton_max_iter;  /* default 4                                                  */
  double h_min;         /* absolute minimum step, s (default 0: only the roundoff floor,*/
                        /* a step too small to change the time reached)               */
  double h_init;        /* > 0: initial step, s (default: starting-step heuristic)    */
  int engine;           /* CAMP_ENGINE_*                                              */
  int wg_per_cu;        /* FUSED_WAVE persistent grid: workgroups per CU, 0 = auto     */
  int persistent;       /* FUSED_*: 1 = persistent grid with a cell queue, 0 = one    */
                        /* workgroup per cell batch, -1 = auto                        */
  int use_graph;        /* PLAIN: 1 = replay a captured hipGraph of each chunk of     */
                        /* step-attempt launches                                      */
  int waves_per_wg;     /* FUSED_WAVE, one wavefront per cell: cells per workgroup      */
                        /* 1..8 (1..12 in launch modes 3, 4 up to 128 state variables),*/
                        /* 0 = auto                                                    */
  int stage_tables;     /* FUSED_WAVE launch mode: 0 = tables read from global memory, */
                        /* 1 = sparse-index tables staged in LDS, 2 = all tables in    */
                        /* LDS (also forcing terms and Jacobian map), 3 / 4 = as 0 / 1 */
                        /* with the rate constants in a global per-cell-slot scratch   */
                        /* (persistent grid), -1 = auto                                */
  int lanes_per_cell;   /* FUSED_WAVE: 64 = one wavefront per cell, 128 or 256 = one     */
                        /* workgroup of 2 or 4 wavefronts per cell (more than 64 / 128  */
                        /* state variables), 0 = auto                                   */
  int full_newton;      /* 0 (default): Newton with Jacobian reuse; a cell that fails   */
                        /* (status 1-4) is integrated again from its input with full    */
                        /* Newton. 1: full Newton (fresh Jacobian and LU every iteration)*/
  const int* cell_order;/* NULL (default), or a permutation of 0..n_cells-1 giving the   */
                        /* order in which a persistent wavefront-engine launch takes     */
                        /* cells from its queue (for example costliest first, by the     */
                        /* per-cell counters of the previous host step, so the last      */
                        /* cells to start are short). Device memory for                  */
                        /* camp_solve_device and the server (it must stay valid until    */
                        /* the solve has run on the stream), host memory for camp_solve. */
                        /* camp_solve rejects a non-permutation with CAMP_EINVAL; on the */
                        /* device path it is checked on the stream and, if it is not a   */
                        /* permutation, ignored (cells run in index order). Other        */
                        /* engines and non-persistent launches ignore it. Results never  */
                        /* depend on the order: each cell is integrated alone.           */
  double lu_gamma_drift;/* Jacobian reuse: refactor when h / beta drifts from the value    */
                        /* of the last factorization by more than this fraction          */
                        /* (default 0.3; <= 0 = default)                                 */
  int lu_max_age;       /* ... or after this many accepted steps (default 20)            */
  double newton_tol;    /* Newton convergence: estimated remaining error in the weighted */
                        /* norm at most this (default 0.1)                               */
} camp_opts;

/* Per-cell counters (optional output). */
typedef struct {
  int steps, rejected, newton_fail, newton_iters, n_f, n_jac, n_lu, order;
} camp_cell_stats;

/* Solve n_cells cells with host arrays (paper Sect. 2.4.2, runtime workflow: the host
 * model hands over the environment and concentrations of each grid cell, the solver
 * integrates the chemistry over the host time step, the new state is read back; Sect.
 * 2.4.1: each cell by variable-order BDF with Newton iteration and error control).
 * state[cells][n_state] is read and overwritten in place. cell_status[cells] and
 * cell_stats[cells] may be NULL. opts may be NULL.
 * Returns CAMP_ESOLVE if any cell failed (its row is left at its input values). */
int camp_solve(camp_mech* mech, int n_cells, double* state, const camp_env* env, double dt,
               double rtol, double atol, const camp_opts* opts, int* cell_status,
               camp_cell_stats* cell_stats);

/* Same with device arrays (env fields are device pointers) on a stream. Stream-ordered:
 * results are ready when the stream reaches the end of the call. cell_status is required
 * (device, [cells]). The return value reports argument and launch errors only; per-cell
 * failures are reported through cell_status (use camp_count_failed). */
int camp_solve_device(camp_mech* mech, int n_cells, double* d_state, const camp_env* d_env,
                      double dt, double rtol, double atol, const camp_opts* opts,
                      int* d_cell_status, camp_cell_stats* d_cell_stats, void* stream);

/* --- Plans: one device solve captured once as a HIP graph and replayed. For a host model
 *     that calls the solver every time step on the same device arrays (paper Sect. 2.4.2:
 *     set the environment, solve, read the state back, every step): the launch sequence of
 *     the fused wavefront engine (queue reset, cell-order check, persistent kernel) is
 *     resolved (autotuner trials included), given its own scratch and captured once; each
 *     replay then costs one graph launch. --- */
typedef struct camp_plan camp_plan;

/* Same arguments as camp_solve_device; the pointers (device memory) are fixed in the plan
 * and read at every replay, so they must stay valid until camp_plan_free. Only the fused
 * wavefront engine is captured: engine AUTO (which must resolve to it) or FUSED_WAVE, else
 * CAMP_EINVAL. The plan owns its scratch: replays of different plans may overlap, replays of
 * one plan on several streams at once race. Errors: CAMP_EINVAL, CAMP_ENOMEM, CAMP_EDEVICE. */
int camp_plan_create(camp_mech* mech, int n_cells, double* d_state, const camp_env* d_env,
                     double dt, double rtol, double atol, const camp_opts* opts,
                     int* d_cell_status, camp_cell_stats* d_cell_stats, void* stream,
                     camp_plan** out);

/* Replays the captured solve on `stream` (stream-ordered; results as camp_solve_device).
 * The current device must be the plan's. */
int camp_plan_launch(camp_plan* plan, void* stream);

/* Waits for the plan's device, then releases the graph and its scratch. NULL is ignored. */
void camp_plan_free(camp_plan* plan);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): camp_solve_device without any device
 * allocation. Its scratch (queue counter and flags, rate-constant scratch, cell-order
 * check counters) is a fixed array of camp_noalloc_scratch_bytes() (32 MiB) per GPU, held
 * until the process ends. Requirements: the mechanism's tables already resident on the
 * current device (a camp_solve_device or camp_plan_create with it on this device), and the
 * fused wavefront engine (engine AUTO, which takes the autotuner's cached choice for this
 * size bucket or else the occupancy default and never runs trials, or FUSED_WAVE). A solve
 * that needs more scratch than the array holds is rejected with CAMP_EINVAL, as are the
 * other engines. Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (other streams, other threads) race; serialize them. Results equal camp_solve_device's
 * with the same launch choice. */
int camp_solve_device_noalloc(camp_mech* mech, int n_cells, double* d_state,
                              const camp_env* d_env, double dt, double rtol, double atol,
                              const camp_opts* opts, int* d_cell_status,
                              camp_cell_stats* d_cell_stats, void* stream);
size_t camp_noalloc_scratch_bytes(void);

/* --- Individual hot-path steps on device arrays (validation and composition). All
 *     per-cell arrays are row-major [cells][...] device memory. --- */

/* Rate constants k[cells][R] in expanded-reaction order (camp_mech_info.n_rxn_expanded).
 * Expansion order: processes in input order; a gas process gives one reaction; a
 * condensed-phase process one per instance of its phase; a transfer process two per
 * instance (condensation G -> A, then evaporation A -> G). */
int camp_rate_constants_device(camp_mech* mech, int n_cells, const camp_env* d_env,
                               double* d_k, void* stream);

/* Forcing f[cells][N] = sum over reactions of net stoichiometry times
 * k * product of reactant concentrations (paper Sect. 2.4.2), state layout as above. */
int camp_forcing_device(camp_mech* mech, int n_cells, const double* d_k, const double* d_y,
                        double* d_f, void* stream);

/* Newton matrix M = I - gamma * J(y) in the filled pattern: m[cells][Z], slot order of
 * camp_mech_export (fill slots hold 0 off the diagonal). */
int camp_newton_matrix_device(camp_mech* mech, int n_cells, const double* d_k,
                              const double* d_y, double gamma, double* d_m, void* stream);

/* In-place LU factorization of m[cells][Z] (static order, no pivoting): afterwards the
 * strictly lower slots hold L (unit diagonal implied) and the rest U. */
int camp_lu_factor_device(camp_mech* mech, int n_cells, double* d_m, void* stream);

/* Solve (L U) x = b for each cell; b[cells][N] in state layout is overwritten by x. */
int camp_lu_solve_device(camp_mech* mech, int n_cells, const double* d_lu, double* d_b,
                         void* stream);

/* Number of cells with nonzero status (device status array), written to *n_failed. */
int camp_count_failed(int n_cells, const int* d_cell_status, int* n_failed, void* stream);

/* --- Measurement probes: what the device sustains, as denominators beside the published
 *     peaks of a roofline. Both synchronize on `stream` and return the rate. --- */

/* Device copy d_dst[i] = d_src[i] of n doubles (n even, 16-byte aligned buffers owned by
 * the caller), `reps` timed launches after one warm-up: *gb_per_s = 16 n reps / time
 * (bytes read plus written). */
int camp_probe_copy(const double* d_src, double* d_dst, size_t n, int reps, void* stream,
                    double* gb_per_s);

/* FP64 FMA rate: `blocks` workgroups of 256 threads, each thread 16 independent FMA chains
 * of `iters` steps; d_sink (caller-owned, blocks * 256 doubles) receives the sums.
 * *tflop_per_s = 2 * 16 * iters * blocks * 256 / time. */
int camp_probe_fma(double* d_sink, int blocks, int iters, void* stream, double* tflop_per_s);

/* --- Serving: requests are admitted by device-memory footprint and run concurrently on
 *     the device; each request's cells are solved exactly as by camp_solve_device. Several
 *     mechanisms may be resident at once, one compiled object each (paper Sect. 2.1: one
 *     core object per mechanism, several serving different mechanisms). --- */
typedef struct camp_server camp_server;

/* max_bytes: budget of device memory for in-flight requests (0 = 50% of free memory). A
 * request's footprint is its own arrays (state, environment, status) plus the scratch of
 * the launch chosen for it (the lane engines' per-call slabs or the wavefront engine's
 * stream workspace); autotuning a cold (mechanism, size) bucket reserves the trials'
 * scratch while they run. A request larger than the budget runs alone.
 * max_inflight: concurrent requests (streams), 1..64. One server thread admits requests
 * in FIFO order (tuning and launching outside the server's lock) and retires them. */
int camp_serve_create(long long max_bytes, int max_inflight, camp_server** out);

/* Submit a request on device-resident data (pointers stay owned by the caller and must
 * remain valid until the request completes; the data must be ready, i.e. the stream that
 * produced it synchronized, since requests run on the server's own streams). The request
 * is queued if it does not fit the memory budget or no stream slot is free. Returns a
 * ticket (> 0). Requests that overlap on the device never share arithmetic. */
int camp_serve_submit(camp_server* srv, camp_mech* mech, int n_cells, double* d_state,
                      const camp_env* d_env, double dt, double rtol, double atol,
                      const camp_opts* opts, int* d_cell_status, long long* ticket);

/* Poll: *done = 1 when finished; then *n_failed is its failed-cell count and
 * *latency_s the time from submission to completion. */
int camp_serve_poll(camp_server* srv, long long ticket, int* done, int* n_failed,
                    double* latency_s);

/* Block until the request completes. */
int camp_serve_wait(camp_server* srv, long long ticket);

/* Number of requests in flight (launched or being admitted) in *inflight and waiting in
 * the FIFO in *queued. Never blocks on the device. */
int camp_serve_progress(camp_server* srv, int* inflight, int* queued);

void camp_serve_destroy(camp_server* srv);

const char* camp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CAMP_H */
