/*
 * abm.h -- C ABI of the DeepABM-COVID daily transmission-and-progression step on
 * AMD MI355X (gfx950).
 *
 * The model (Chopra et al., "DeepABM: Scalable, Efficient and Differentiable
 * Agent-Based Simulations via Graph Neural Networks", arXiv 2110.04421):
 *   - agents with static age group / household / occupation and dynamic disease stage,
 *     quarantine and vaccination status (section 3, "Agent State Definition");
 *   - household, occupation and random contact networks, the last two redrawn every
 *     day (section 3, "Interaction Networks");
 *   - force of infection of eq. 1 summed over a susceptible's contacts and infection
 *     probability of eq. 2 (section 3, "Infection Transmission");
 *   - stage progression (section 3, "Disease Progression"), here SEIRM with fixed
 *     durations;
 *   - self-quarantine and testing (section 4), two-dose vaccination with the priority
 *     orders of Table 1 and sterilising immunity (section 5).
 *
 * Conventions
 *   - Every function returns int: ABM_OK (0) or a negative ABM_E_* code.  Nothing
 *     throws or aborts.  Errors are sticky per simulation: once a call fails, later
 *     calls on the same abm_sim return the same code; abm_last_error() has the text.
 *     Errors detected on the device (edge capacity overflow) surface at the next
 *     abm_sync / abm_run / abm_get.
 *   - "h_" pointers are host memory, "d_" pointers are device memory.  The caller owns
 *     all of them.  Host arrays passed to abm_create are copied; they may be freed on
 *     return.
 *   - The library allocates no device memory.  The caller passes one device workspace
 *     of at least abm_workspace_size() bytes and a HIP stream (hipStream_t as void*);
 *     both must outlive the abm_sim.  All device work is enqueued on that stream.
 *   - Agent ids are global over the concatenated replicates: replicate r owns agents
 *     [agent_offset[r], agent_offset[r+1]).  Households and workplaces never cross a
 *     replicate boundary.
 *   - Random numbers: Philox4x32-10 (Salmon et al., SC'11), key = (seed low word, seed
 *     high word), counter = (agent id within its replicate, day, stream word of the
 *     replicate, purpose << 24 | block).  Every draw is therefore a pure function of
 *     (seed, stream, day, agent), and a replicate's trajectory does not depend on
 *     which other replicates share the launch.
 */
#ifndef ABM_H
#define ABM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ABM_ABI_VERSION 4

enum {
  ABM_OK = 0,
  ABM_E_ARG = -1,        /* invalid argument or parameter value                   */
  ABM_E_ABI = -2,        /* struct_size / abi_version mismatch                    */
  ABM_E_WORKSPACE = -3,  /* workspace smaller than abm_workspace_size()           */
  ABM_E_CAPACITY = -4,   /* a day's contact graph exceeded the planned edge room  */
  ABM_E_HIP = -5,        /* HIP runtime error (text in abm_last_error)            */
  ABM_E_STATE = -6       /* call out of order (e.g. abm_grad before a soft run)   */
};

enum { ABM_HARD = 0, ABM_SOFT = 1 };
enum { ABM_STRATEGY_STANDARD = 0, ABM_STRATEGY_DELAYED = 1, ABM_STRATEGY_DELAYED_EXCEPT_65 = 2 };
enum { ABM_STAGE_S = 0, ABM_STAGE_E = 1, ABM_STAGE_I = 2, ABM_STAGE_R = 3, ABM_STAGE_M = 4,
       /* eleven-stage course (disease_model ABM_DISEASE_COURSE; section 3 "Agent State
          Definition"): S, R and M above are its susceptible, recovered and dead, and a
          susceptible agent with vaccine immunity is its "vaccinated" */
       ABM_STAGE_ASYM = 5, ABM_STAGE_PRE_MILD = 6, ABM_STAGE_PRE_SEVERE = 7, ABM_STAGE_MILD = 8,
       ABM_STAGE_SEVERE = 9, ABM_STAGE_HOSP = 10, ABM_STAGE_ICU = 11 };
#define ABM_DISEASE_SEIRM 0   /* fixed E and I durations, death drawn at removal      */
/* Vaccine immunity (section 5 considers both): a protected agent is not infected, or
 * (course model only) is infected as anyone else is and takes the asymptomatic course */
#define ABM_IMMUNITY_STERILISING 0
#define ABM_IMMUNITY_ASYMPTOMATIC 1
#define ABM_DISEASE_COURSE 1  /* eleven stages, age-dependent paths, random durations */
/* stage durations of the course (shift + Poisson(extra) days), in this order */
enum { ABM_DUR_PRE = 0, ABM_DUR_ASYM, ABM_DUR_MILD, ABM_DUR_SEV_HOSP, ABM_DUR_SEV_R,
       ABM_DUR_HOSP_ICU, ABM_DUR_HOSP_R, ABM_DUR_ICU_DIE, ABM_DUR_ICU_R, ABM_N_DUR };

/* Daily output slots, counts[day][replicate][ABM_NC] (int64). S..M are counts of the
 * state at the end of the day. */
enum {
  ABM_C_S = 0, ABM_C_E, ABM_C_I, ABM_C_R, ABM_C_M,
  ABM_C_NEW,        /* infections during the day (incidence)                       */
  ABM_C_TESTS,      /* tests administered                                          */
  ABM_C_POS,        /* positive results returned (quarantines started)             */
  ABM_C_DOSE1, ABM_C_DOSE2,
  ABM_C_EDGES,      /* directed edges of the day's contact graph (interactions)    */
  ABM_C_NEAR,       /* susceptible draws with |u - p| <= 1e-6 (rounding-sensitive)  */
  ABM_C_INF_EDGES,  /* edges of the day's graph whose source was infectious        */
  ABM_C_HOSP,       /* hospitalised agents (course only; 0 otherwise)                */
  ABM_C_ICU,        /* agents in intensive care (course only; 0 otherwise)           */
  ABM_C_NOTIFIED,   /* app users notified of an exposure (told to test tomorrow)      */
  ABM_NC
};

#define ABM_N_AGE 9
#define ABM_N_OCC 23
#define ABM_N_THETA 10      /* gradient slots: dR, dS[0..8] */
#define ABM_NEVER (-32768)  /* "never" for the int16 day fields of the agent state */

/* params.flags */
#define ABM_FLAG_PROFILE 1  /* time every kernel with HIP events (eager launches) */
#define ABM_FLAG_NO_GRAPH 2 /* launch day kernels eagerly instead of a HIP graph  */
#define ABM_FLAG_CLAIM_BUILDER 4 /* build the daily graph with per-edge atomic slot claims
                                    (the default partitions contacts by destination)     */
#define ABM_FLAG_AUTOTUNE 8 /* at create, time the force-of-infection kernel's tilings
                               (LDS chunk x grid x shape) on day 0's graph, keep the fastest;
                               results are bitwise the same for every tiling            */
#define ABM_FLAG_DENSE_MESSAGE 32 /* stream every edge through the force-of-infection
                                      kernel every day; without it, with 2^20 agents or
                                      more, a day with at most N/256 infectious agents
                                      sums only the rows that hold an infectious source
                                      (bitwise the same result)                          */
#define ABM_FLAG_FRONTIER_ANY_SIZE 64 /* test aid: allow that frontier path below 2^20
                                      agents too, where the day is bound by launches and
                                      the path's three extra kernels cost more than they
                                      save                                               */
#define ABM_FLAG_STRAIGHT_THROUGH 128 /* relaxed mode: the forward pass takes the hard
                                      infection draw (the relaxed sample's sign) and the
                                      adjoint the relaxed sample's derivative            */
#define ABM_FLAG_TWO_TILE_LEAVES 256 /* test aid: give the graph builder's partition
                                      leaves of two tiles (512 rows) at any population
                                      size, as it does by itself beyond 2^25 agents; the
                                      graph is bitwise the same                          */
#define ABM_FLAG_SEGMENT_VPLAN 512 /* test aid: plan the day's vaccination doses by
                                      segments of 256 tiles, each summed and ranked by
                                      its own workgroup, at any replicate size, as it is
                                      done by itself above 2048 tiles (2^19 agents) a
                                      replicate; the doses are the same                  */
#define ABM_FLAG_MIN_LDS_ROOM 16 /* test aid: give the graph builder's level-1 scatter
                                    and row pass their smallest LDS and register room,
                                    so that batches and tiles are written directly and
                                    received entries are read twice; the graph is
                                    bitwise the same                                    */

/* Model parameters; copied at create.  Section 3 eq. 1: lambda = R * S_a * A_s * B_n /
 * Ibar * integral of the Gamma infectiousness density over the day. */
typedef struct {
  uint32_t struct_size;            /* sizeof(abm_params)                                  */
  uint32_t abi_version;            /* ABM_ABI_VERSION                                     */
  int32_t n_steps;                 /* days reserved in the trajectory buffer             */
  int32_t mode;                    /* ABM_HARD or ABM_SOFT (relaxed, differentiable)      */
  uint64_t seed;                   /* Philox key                                          */
  float dt;                        /* days per step (1)                                   */
  float kappa;                     /* 1 / Ibar of eq. 1                                   */
  double gamma_shape, gamma_scale; /* infectiousness profile (2.5, 2)                     */
  double A_stage[5];               /* infector factor per stage S,E,I,R,M (A_s of eq. 1)  */
  float w_household, w_occupation, w_random;      /* network factor B_n of eq. 1        */
  double mu_random[ABM_N_AGE];     /* mean daily random in-degree per age group           */
  double mu_occupation[ABM_N_OCC]; /* mean daily workplace in-degree per occupation       */
  float p_death[ABM_N_AGE];        /* death probability at removal, per age group         */
  int32_t e_days, i_days;          /* exposed / infected durations (5, 10); sum <= 63     */
  int32_t quarantine_days;         /* 14; 0 disables quarantine                           */
  int32_t test_delay;              /* days from test to result (>= 1; see test_delay_max)  */
  float quarantine_dropout;        /* daily probability of leaving quarantine early       */
  float test_rate;                 /* daily probability an eligible agent is tested; 0 off*/
  float test_sensitivity;          /* P(positive | exposed or infected)                   */
  double vacc_rate;                /* daily doses as a fraction of the replicate; 0 off   */
  double vacc_trigger;             /* start when infected/N >= trigger (latched; E+I, plus the
                                      hospitalised and ICU agents of the course)         */
  float eff1, eff2;                /* immunity probability after dose 1 / dose 2          */
  int32_t dose_lag;                /* days from a dose to its effect (12)                 */
  int32_t strategy;                /* ABM_STRATEGY_* (priority order of Table 1)          */
  float gumbel_tau;                /* temperature of the relaxed infection (soft mode)    */
  int32_t checkpoint_every;        /* soft mode: days between adjoint checkpoints         */
  int64_t edge_capacity;           /* directed-edge room per day; 0 = mean + 8 sigma of
                                      the contact counts of independent replicates (give
                                      more room when replicates share a stream word)     */
  int32_t flags;                   /* ABM_FLAG_*                                          */
  int32_t disease_model;           /* ABM_DISEASE_SEIRM or ABM_DISEASE_COURSE (hard mode)  */
  /* the course, per age group: asymptomatic share of infections, severe share of the
   * symptomatic, hospitalised share of the severe, intensive-care share of the
   * hospitalised, and deaths among those in intensive care (each in [0, 1]) */
  float p_asym[ABM_N_AGE], p_severe[ABM_N_AGE], p_hosp[ABM_N_AGE], p_icu[ABM_N_AGE],
      p_die[ABM_N_AGE];
  double A_asym;                   /* infectiousness of asymptomatic agents; presymptomatic
                                      ones take A_stage[E], symptomatic ones A_stage[I], and
                                      hospitalised ones are isolated (0)                 */
  int32_t dur_shift[ABM_N_DUR];    /* stage durations: shift (1..60) ...                  */
  int32_t pad_;
  double dur_extra[ABM_N_DUR];     /* ... + Poisson(extra) days (0..20)                   */
  /* testing turnaround and digital exposure notification (section 4) */
  int32_t test_delay_max;          /* result after test_delay .. test_delay_max days,
                                      uniform (the RT-PCR test's 3..5); = test_delay: fixed */
  float app_adoption;              /* share of agents with the notification app; 0 = off;
                                      > 0 keeps den_window days of graphs (hard mode only) */
  float den_compliance;            /* notified app users who test the next day             */
  int32_t den_window;              /* days of contacts a positive result notifies (1..30) */
  int32_t vacc_immunity;           /* ABM_IMMUNITY_*                                      */
} abm_params;

/* Population, concatenated over replicates (host arrays, copied at create). */
typedef struct {
  int32_t n_replicates;
  int32_t n_households;            /* H */
  int32_t n_workplaces;            /* W (0 if none) */
  int32_t reserved;
  const int64_t* agent_offset;     /* [R+1], agent_offset[0] = 0, N = agent_offset[R];
                                      N < 2^30 (a graph column holds a 30-bit agent id)  */
  const uint8_t* age;              /* [N] age group 0..8                                  */
  const int32_t* hh_start;         /* [H+1] household h = agents [hh_start[h], hh_start[h+1]), sizes 1..255 */
  const uint8_t* occupation;       /* [N] occupation 0..22                                */
  const int32_t* wp_start;         /* [W+1] workplace w = wp_members[wp_start[w] .. wp_start[w+1]) */
  const int32_t* wp_members;       /* [wp_start[W]] agent ids, each agent at most once; sizes <= 65535 */
  const float* R;                  /* [R] R of eq. 1 per replicate                        */
  const float* susceptibility;     /* [R][9] S_a of eq. 1 per replicate                   */
  const int32_t* dose2_delay;      /* [R] days between doses                              */
  const int64_t* init_offset;      /* [R+1]                                               */
  const int32_t* initial_infected; /* [init_offset[R]] agents exposed on day -1           */
  const uint32_t* stream;          /* [R] Philox stream word per replicate; NULL = r      */
} abm_population;

typedef struct abm_sim abm_sim;

/* Device state of one agent, 16 bytes (abm_get(ABM_GET_STATE) returns N of these). */
typedef struct {
  uint8_t stage;      /* ABM_STAGE_* */
  uint8_t flags;      /* bit 0: test result pending, bit 1: that result is positive,
                         bit 2: notified of an exposure yesterday (tests today) */
  uint8_t vacc;       /* doses received (0, 1, 2) */
  uint8_t course;     /* course path: bits 0-1 0 asymptomatic / 1 mild / 2 severe, bit 2
                         hospitalised, bit 3 intensive care, bit 4 dies (course only) */
  int16_t t_exp;      /* day of exposure (ABM_NEVER if never) */
  int16_t q_until;    /* quarantined on days < q_until */
  int16_t test_day;   /* day of the pending test */
  int16_t d1, d2;     /* days of dose 1 / dose 2 */
  int16_t t_next;     /* day the current stage of the course ends (ABM_NEVER if none) */
} abm_agent_state;

/* Bytes of device workspace the simulation needs: the agent records of section 3
 * ("Agent State Definition"), one day's household + occupation + random contact graph
 * (section 3, "Interaction Networks") with an edge room of the mean plus 8 standard
 * deviations of the Poisson contact counts, and the graph builder's partitions.
 * Validates p and pop first (ABM_E_ARG / ABM_E_ABI / ABM_E_CAPACITY on a bad input;
 * *bytes untouched then). */
int abm_workspace_size(const abm_params* p, const abm_population* pop, size_t* bytes);

/* Validate, copy the population to the device, build the tables, set day 0, and
 * capture the day's kernel chain in a HIP graph.  The tables are those the paper's
 * model statement fixes: the Gamma integral over each day since exposure times the
 * stage factor A_s (section 3, eq. 1), the Poisson contact-count thresholds of the
 * daily networks (section 3, "Interaction Networks"), and the vaccination priority
 * classes of the three strategies (section 5, Table 1).  The initial infections are
 * exposed on day -1 (section 5's protocol of ten initial infections).  Synchronises
 * the stream before returning.  On failure *out is still set (free it with
 * abm_destroy; abm_last_error has the reason): ABM_E_ARG, ABM_E_ABI,
 * ABM_E_WORKSPACE (d_workspace NULL or smaller than abm_workspace_size), ABM_E_HIP. */
int abm_create(const abm_params* p, const abm_population* pop, void* d_workspace,
               size_t ws_bytes, void* hip_stream, abm_sim** out);

/* Enqueue n_days days (asynchronous, hard mode).  One day: results due today start
 * quarantines (section 4, "Self-quarantine", "Testing"); doses are allocated by the
 * Table 1 priority (section 5); the day's contact graph is drawn (section 3,
 * "Interaction Networks"); each agent's force of infection is eq. 1 summed over its
 * contacts, and it is infected with probability eq. 2, 1 - exp(-lambda dt); stages
 * advance (section 3, "Disease Progression"); tests are drawn.  ABM_E_STATE past
 * n_steps or in soft mode; device-side overflow surfaces at abm_sync/run/get. */
int abm_step(abm_sim* s, int32_t n_days);

/* Enqueue n_days days (the day of abm_step), wait, and copy their outputs:
 * h_counts [n_days][R][ABM_NC] (hard mode; may be NULL): the compartment counts,
 * infections, tests, doses and deaths the paper reports per run (section 4's sample
 * results, section 5's protocol); h_soft_incidence [R][n_days] (soft mode; may be
 * NULL): the relaxed daily incidence, where eq. 2's draw is replaced by a
 * Gumbel-softmax sample on the same uniform (the differentiable simulation the
 * abstract and section 1 motivate).  Returns ABM_E_CAPACITY if a day's graph
 * overflowed its room. */
int abm_run(abm_sim* s, int32_t n_days, int64_t* h_counts, float* h_soft_incidence);

/* Soft mode, after abm_run from day 0: gradient of L with respect to eq. 1's R and
 * S_0..S_8 of every replicate, given dL/d(soft incidence) h_dL [R][days run] (the
 * gradient-based calibration the abstract, section 1 and section 6 name as the use of
 * a differentiable simulator).  Reverse sweep over checkpoints kept every
 * checkpoint_every days; writes h_dtheta [R][ABM_N_THETA].  ABM_E_STATE in hard mode
 * or before a soft run. */
int abm_grad(abm_sim* s, const float* h_dL, float* h_dtheta);

/* Soft mode: replace every replicate's parameters theta = (R, S_0..S_8) with
 * h_theta [R][ABM_N_THETA] (host array, copied; each value finite and > 0, else
 * ABM_E_ARG) and rewind to day 0 with the initial state, so that the next abm_run
 * starts over at the new parameters (same population, seeds and Philox streams).
 * This is what an iterative fit of theta through abm_grad calls between steps
 * (section 6 of the paper names calibration by gradients as the direction beyond
 * grid search); it allocates nothing.  ABM_E_STATE in hard mode. */
int abm_set_theta(abm_sim* s, const float* h_theta);

enum {
  ABM_GET_STATE = 0,   /* abm_agent_state[N]                                          */
  ABM_GET_LAMBDA = 1,  /* float[N]: force of infection of the last day run           */
  ABM_GET_CODE = 2,    /* uint8[N]: infectiousness code (days since exposure, 0 = none) of the last day */
  ABM_GET_ROWPTR = 3,  /* int32[N+1]: CSR row pointers of the last day's graph        */
  ABM_GET_COL = 4,     /* int32[E]: source agent of each edge (E = rowptr[N])        */
  ABM_GET_W = 5,       /* float[E]: network factor of each edge                       */
  ABM_GET_ATAB = 6,    /* float[64]: A(stage) * Phi(tau) per days since exposure      */
  ABM_GET_POISSON = 7, /* uint32[32][64]: thresholds, occupations 0..22 then age groups */
  ABM_GET_DAY = 8,     /* int32: days run so far                                      */
  ABM_GET_LATCH = 9,   /* uint8[R]: vaccination started                              */
  ABM_GET_SOFT_S = 10, /* float[N]: soft susceptible mass                             */
  ABM_GET_COEF = 11,   /* float[R][9]: fl(fl(R*kappa)*S_a)                             */
  ABM_GET_TUNING = 12  /* int32[3]: message-kernel LDS chunk (edges), grid (workgroups),
                          shape: 0 one tile per workgroup with the masks in L2, 1 one
                          tile with the first mask level in LDS, 2 four tiles sharing
                          that LDS mask, 3 four tiles with each wave streaming the
                          edges of 64 rows through its own LDS chunk               */
};
/* Copy a device quantity to host (synchronous; h_bytes must be at least its size,
 * else ABM_E_ARG): the agent records of section 3 ("Agent State Definition"), eq. 1's
 * force of infection and infectiousness codes, the day's contact graph (section 3,
 * "Interaction Networks"), the tables. */
int abm_get(abm_sim* s, int32_t what, void* h_dst, size_t h_bytes);

/* Overwrite the hard-mode state: day, per-replicate vaccination latch (uint8[R]) and
 * agent states (abm_agent_state[N], section 3's agent state).  Used to resume and to
 * resynchronise with an external reference.  Every draw is keyed on (seed, stream,
 * day, agent), so a resumed run equals the uninterrupted one.  ABM_E_ARG on a wrong
 * agent count or day; ABM_E_STATE in soft mode. */
int abm_set_state(abm_sim* s, int32_t day, const uint8_t* h_latch,
                  const abm_agent_state* h_state, size_t n_agents);

/* Wait for the stream and surface device-side errors (ABM_E_CAPACITY).  A runtime
 * call with no counterpart in the paper. */
int abm_sync(abm_sim* s);

void abm_destroy(abm_sim* s);
const char* abm_error_string(int code);
const char* abm_last_error(const abm_sim* s);

/* Per-kernel timing (params.flags & ABM_FLAG_PROFILE): number of timed steps of the day
 * (one or a few kernels each), their names, accumulated milliseconds and launch counts
 * since create or reset. */
int abm_profile_kernels(const abm_sim* s);
const char* abm_profile_name(const abm_sim* s, int32_t k);
int abm_profile_get(abm_sim* s, double* h_ms, int64_t* h_launches);
int abm_profile_reset(abm_sim* s);

/* Philox4x32-10 of n counters (d_ctr [n][4]) under a 64-bit seed into d_out [n][4]
 * (device arrays; for checking the generator). */
int abm_philox(uint64_t seed, const uint32_t* d_ctr, int64_t n, uint32_t* d_out, void* hip_stream);

/* ---- Calibration network (maps a daily incidence curve to the parameters) ----------
 * Learned calibration of eq. 1's R and S_a from a run's incidence: section 1 names
 * the restrictive randomised search used to calibrate such simulators, and section 6
 * the move beyond grid search as future work; the network is trained on the
 * simulator's own runs and judged by re-simulating its prediction.
 * Fully connected 192 -> 256 -> 256 -> 16, ReLU after the two hidden layers.  BF16
 * weights and activations, FP32 accumulation on the matrix cores, FP32 master weights
 * with Adam.  Parameter blob layout (both the BF16 and the FP32 copies):
 *   W1 [256][192], b1 [256], W2 [256][256], b2 [256], W3 [16][256], b3 [16]
 * (row-major, out x in; biases in the same dtype as the weights).
 * The workspace holds the activations of the last forward pass for the backward. */
#define ABM_MLP_IN 192
#define ABM_MLP_H 256
#define ABM_MLP_OUT 16
#define ABM_MLP_NPARAM (256 * 192 + 256 + 256 * 256 + 256 + 16 * 256 + 16)

int abm_mlp_workspace_size(int32_t max_batch, size_t* bytes);
/* y [B][16] fp32 = MLP(x [B][192] fp32); params bf16 (ABM_MLP_NPARAM). */
int abm_mlp_forward(void* d_ws, size_t ws_bytes, const uint16_t* d_params_bf16, const float* d_x,
                    int32_t B, float* d_y, void* hip_stream);
/* The forward pass above with no workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses that forbid
 * allocation).  Same kernels and result as abm_mlp_forward; the activations go to a
 * scratch array of the library, one per GPU, sized for ABM_MLP_NOALLOC_MAX_BATCH rows
 * (about 1.5 MB, held until the process ends).  Allocates nothing.  B larger than
 * ABM_MLP_NOALLOC_MAX_BATCH: ABM_E_WORKSPACE; B < 1 or a null pointer: ABM_E_ARG.
 * Every call on one GPU shares that GPU's scratch: calls that overlap on one GPU (two
 * streams, two threads) race, so serialise them.  The backward pass cannot follow this
 * forward (it needs the activations in a workspace of the caller's). */
#define ABM_MLP_NOALLOC_MAX_BATCH 1024
int abm_mlp_forward_noalloc(const uint16_t* d_params_bf16, const float* d_x, int32_t B, float* d_y,
                            void* hip_stream);
/* MSE loss mean over B*n_out of (y - target) on the first n_out outputs; writes
 * d_grads_f32 (ABM_MLP_NPARAM) and the loss to d_loss (device float).  Uses the
 * activations of the last forward with the same params. */
int abm_mlp_backward(void* d_ws, size_t ws_bytes, const uint16_t* d_params_bf16,
                     const float* d_target, int32_t B, int32_t n_out, float* d_grads_f32,
                     float* d_loss, void* hip_stream);
/* One Adam step on the FP32 master copy, refreshing the BF16 copy. */
int abm_mlp_adam(float* d_master_f32, uint16_t* d_params_bf16, float* d_m, float* d_v,
                 const float* d_grads_f32, float lr, float b1, float b2, float eps,
                 int32_t step, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* ABM_H */
