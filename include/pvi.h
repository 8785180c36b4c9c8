/*
 * pvi.h - value iteration for perishable-inventory MDPs on one MI355X (gfx950).
 *
 * The library computes, for every state s of a perishable-inventory MDP, the
 * synchronous Bellman backup in its deterministic-transition form
 *
 *     V_{i+1}(s) = max_a  sum_w P(w|s,a) [ r_w + gamma V_i(s'_w) ],
 *     (s'_w, r_w) = T(s, a, w)
 *
 * (Methods, "Value iteration": the deterministic-transition update and policy
 * equations), stops when span(V_{i+1} - V_i) = max - min < eps (1-gamma)/gamma
 * (the span rule of Appendix B, with the discount folded into the threshold),
 * and extracts the greedy policy with one more backup of the returned V (the
 * extraction step of the vmap value-iteration algorithm).  Ties go to the
 * lowest action index.
 *
 * Three scenario families are supported:
 *   PVI_FAMILY_LEADTIME    Scenario A (Appendix A): one product, lead time L >= 1,
 *                          FIFO issuing.  State digits, most significant first:
 *                          [O_{L-1}, ..., O_1, X_m, ..., X_1], radix a_max+1.
 *                          Outcome: demand d in 0..d_max.
 *   PVI_FAMILY_SUBST2      Scenario B (Appendix B): two products, L = 0 (today's
 *                          order is on hand before demand), FIFO; unmet demand of
 *                          product 0 accepts product 1 with probability subst_rho
 *                          per customer (binomial), served from product 1 stock
 *                          left after its own demand.  State digits
 *                          [A_{m-1}..A_1, B_{m-1}..B_1]; action a = a0*(a_max[1]+1)+a1.
 *                          Reward -c_var.a + c_rev.issued.
 *   PVI_FAMILY_RUL_WEEKDAY Scenario C (Appendix C): weekday demand, L = 0, remaining
 *                          life on arrival ~ Multinomial(a; p_m(a)..p_1(a)), stock
 *                          of each life capped at a_max (excess refused at delivery).
 *                          State digits [tau, X_{m-1}, ..., X_1].
 *   PVI_FAMILY_SUBST2_L1   Scenario B as the paper runs it (Scenario B description,
 *                          Appendix B): two products a (0) and b (1), lead time 1
 *                          (yesterday's orders are in stock with m days of life), FIFO;
 *                          product b issues h_b = min(D_b, I_b) and its D_b - h_b unmet
 *                          customers each accept product a with probability subst_rho;
 *                          product a issues h_a = min(D_a + accepted, I_a).  State
 *                          digits [Xa_m..Xa_1, Xb_m..Xb_1]; action a = a0*(a_max[1]+1)+a1;
 *                          outcome (h_a, h_b); reward -c_var.a + c_rev.h.  gamma = 1 is
 *                          allowed (the span rule then stops at span < eps), and the
 *                          solve starts from the expected one-day sales revenue when
 *                          no v0 is given (Appendix B, initial value equation).
 *
 * Conventions
 *  - Every function returns pvi_status and never throws across the ABI.  On error
 *    a thread-local message is available from pvi_last_error(); outputs are left
 *    untouched unless stated.
 *  - Host pointers are caller-owned.  Descriptors, tables and v0 are copied.
 *  - A pvi_mdp owns its device buffers (tables, V, policy), which stay resident in
 *    HBM from the first solve until mdp_destroy.
 *  - Distinct pvi_mdp handles may be used from different threads.  One handle must
 *    not be used by two threads at once.  Server calls are thread-safe.
 *  - There is no CPU fallback: without a usable gfx950 device, solves return
 *    PVI_E_DEVICE.
 *  - Scenario C times its merge kernels at each candidate block width at the first
 *    solve of a shape (R, m, weekdays) in a process and keeps the fastest; results do
 *    not depend on the choice.  PVI_TUNE=0 in the environment skips the timing (the
 *    LDS rule then chooses); PVI_TUNE_VERBOSE=1 prints the choices to stderr;
 *    PVI_C_BLOCK=4|8|12|16|32 fixes the width wherever it fits (for tests).
 *  - Scenario A (FIFO) packs floor(64 / R) tiles into a wavefront, or 2 when that
 *    would leave fewer wavefronts than the device has SIMDs; results do not depend
 *    on the choice.  PVI_A_GROUP=<G>, 1 <= G <= floor(64 / R), read by mdp_create,
 *    fixes it (for tests).
 *  - Scenario B as the paper runs it (lead time 1) with 16 orders of each product
 *    sweeps with a final kernel over lanes of b's orders; PVI_B1_LANES=0 keeps the
 *    kernel over lanes of a's stock (for tests: both give the same values).
 *  - Scenario B (two products, L = 0) runs tiled stage kernels (sweeps and policy
 *    extraction) when a_max[0] <= 15 and d_max[0] <= 31; PVI_B_TILED=0, read by
 *    mdp_create, keeps the per-cell kernels (for tests: both give the same values).
 */
#ifndef PVI_H
#define PVI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PVI_OK = 0,
    PVI_E_INVALID = 1,       /* bad argument or descriptor */
    PVI_E_NOMEM = 2,         /* host or device allocation failed */
    PVI_E_DEVICE = 3,        /* HIP runtime error or no device */
    PVI_E_NOT_CONVERGED = 4, /* max_sweeps reached; V and policy still readable */
    PVI_E_NOT_READY = 5,     /* ticket still running, or no solve yet */
    PVI_E_CANCELLED = 6,     /* request cancelled or server shut down */
    PVI_E_BUSY = 7,          /* request does not fit the server's HBM budget */
    PVI_E_IO = 8             /* a checkpoint file could not be read or written */
} pvi_status;

typedef enum {
    PVI_FAMILY_LEADTIME = 0,
    PVI_FAMILY_SUBST2 = 1,
    PVI_FAMILY_RUL_WEEKDAY = 2,
    PVI_FAMILY_SUBST2_L1 = 3
} pvi_family;

typedef enum {
    PVI_DEMAND_NONE = 0,    /* demand is always 0 */
    PVI_DEMAND_POISSON = 1, /* mean */
    PVI_DEMAND_GAMMA = 2,   /* mean, shape = coefficient of variation sigma/mu;
                               P(d) = F(d+1/2) - F(d-1/2), F(x<=0) = 0 (Appendix A) */
    PVI_DEMAND_NEGBIN = 3,  /* mean, shape = n target successes, p = n/(n+mean)
                               (Appendix C, demand equation) */
    PVI_DEMAND_TABLE = 4    /* explicit PMF rows in demand_table */
} pvi_demand_kind;

typedef enum {
    PVI_FP64 = 0,      /* FP64 storage and FP64 accumulation in every sweep */
    PVI_FP32 = 1,      /* FP32 centred storage (V = c + v, c FP64 per instance),
                          compensated (Kahan) FP32 accumulation over outcomes;
                          FP64 span check, then FP64 polish sweeps to the threshold */
    PVI_FP32_WIDE = 2  /* FP32 centred storage, FP64 accumulation; FP64 check and
                          polish as PVI_FP32 */
} pvi_precision;

/* Scenario A issuing order (Appendix A): FIFO issues the oldest units first
 * (FIFO issuing/ageing equation), LIFO the youngest (LIFO issuing/ageing
 * equation).  The other families issue FIFO. */
typedef enum {
    PVI_FIFO = 0,
    PVI_LIFO = 1
} pvi_issuing;

/* Stopping rule of vi_solve.  SPAN (Appendix B convergence test): stop when
 * max(V_new - V) - min(V_new - V) < eps (1 - gamma) / gamma.  SUPNORM (Appendix A
 * convergence test): stop when max |V_new - V| < eps.  PERIODIC (Appendix C
 * convergence test, period P = n_periods): with the increments d_k = V_k - V_{k-1}
 * and D(s) = sum_{j=0}^{P-1} gamma^j d_{i-j}(s) (the paper's gamma^-(i-j-1)-weighted
 * sum times gamma^(i-1), the same test), stop at sweep i >= P once
 * max D - min D <= 2 eps min(|max D|, |min D|); eps is relative here.  The test
 * runs on FP64 sweeps, which keep the last P + 1 value tables; with the FP32
 * schedules the FP32 phase is a warm start of at most 2P sweeps. */
typedef enum {
    PVI_STOP_SPAN = 0,
    PVI_STOP_SUPNORM = 1,
    PVI_STOP_PERIODIC = 2
} pvi_stop_rule;

#define PVI_MAX_PERIODS 7
#define PVI_MAX_LIFE 8

/* Parametric MDP descriptor.  Parameters not used by a family are ignored.
 * Demand PMFs are truncated at d_max with the upper tail folded into d_max:
 * P(d_max) = P(D >= d_max) (Poisson, negative binomial) or 1 - F(d_max - 1/2)
 * (gamma). */
typedef struct pvi_mdp_desc {
    uint32_t struct_size;      /* sizeof(pvi_mdp_desc); a smaller size that ends before
                                  `issuing` is accepted, the missing fields read 0 */
    int32_t family;            /* pvi_family */
    int32_t m;                 /* maximum useful life, 1..PVI_MAX_LIFE */
    int32_t lead_time;         /* A: >= 1; B and C: 0; SUBST2_L1: 1 */
    int32_t n_periods;         /* C: 1..7 demand periods (weekdays); else 1 */
    int32_t a_max[2];          /* max order per product; B uses both */
    int32_t d_max[2];          /* demand truncation per product */
    int32_t demand_kind[2];    /* pvi_demand_kind per product */
    double demand_mean[2][PVI_MAX_PERIODS];
    double demand_shape[2][PVI_MAX_PERIODS];
    const double* demand_table[2]; /* TABLE: [n_periods][d_max+1], rows sum to 1 */
    double rul_c0[PVI_MAX_LIFE];   /* C: log(p_k(a)/p_1(a)) = c0[k-1] + c1[k-1] a, k>=2 */
    double rul_c1[PVI_MAX_LIFE];
    double subst_rho;          /* B: per-customer substitution probability */
    double c_var[2];           /* per-unit order cost */
    double c_fixed;            /* C: fixed cost when a > 0 */
    double c_hold, c_short, c_waste;
    double c_rev[2];           /* B: revenue per unit issued */
    double gamma;              /* discount factor, 0 < gamma < 1 (SUBST2_L1: <= 1) */
    int32_t issuing;           /* A: pvi_issuing (absent in older callers' struct_size: FIFO) */
} pvi_mdp_desc;

typedef struct pvi_solve_opts {
    uint32_t struct_size;      /* sizeof(pvi_solve_opts); a smaller size that ends before
                                  `stop_rule` is accepted, the missing field reads 0 */
    int32_t precision;         /* pvi_precision */
    double eps;                /* tolerance of the stopping rule (see pvi_stop_rule) */
    int32_t max_sweeps;        /* cap on sweeps (> 0) */
    int32_t fixed_sweeps;      /* > 0: run exactly this many sweeps, no early stop */
    const double* v0;          /* optional host [N_S] initial values; NULL = zeros */
    void* stream;              /* optional hipStream_t; NULL = the handle's own */
    int32_t check_every;       /* sweeps launched between host checks; 0 = default */
    int32_t time_kernels;      /* 1: time every backup launch with HIP events */
    int32_t stop_rule;         /* pvi_stop_rule (absent in older callers' struct_size: SPAN) */
    /* Checkpoint files (fields absent in older callers' struct_size read 0).  With
     * a path and checkpoint_every > 0, the FP64 sweeps write the file (to
     * `path`.tmp, then renamed over `path`) at the first host check after every
     * checkpoint_every sweeps, and once more when the solve ends.  With resume = 1
     * the solve starts from the file at `path` instead of v0: its value history
     * and sweep count (which max_sweeps and fixed_sweeps include), continuing with
     * FP64 sweeps whatever the precision, so a resumed solve with the same options
     * ends with the V, policy and FP64 sweep count of the uninterrupted solve whose
     * FP64 sweeps wrote the file.  The file must come from a handle with
     * the same descriptor (checked by a fingerprint of the state space, costs,
     * discount and demand and life distributions).  FP32 storage sweeps are not
     * checkpointed.  Not accepted by the request server. */
    const char* checkpoint_path;
    int32_t checkpoint_every;  /* >= 0; 0 = no checkpoints written */
    int32_t resume;            /* 1: start from the checkpoint at checkpoint_path */
} pvi_solve_opts;

typedef struct pvi_result {
    int32_t status;            /* pvi_status of the solve */
    int32_t sweeps_fp32;       /* sweeps run with FP32 storage */
    int32_t sweeps_fp64;       /* sweeps run in FP64 (including polish; a resumed
                                  solve counts its checkpoint's too) */
    int32_t backup_launches[2];/* backup launches timed (time_kernels = 1); [0] FP64
                                  storage sweeps, [1] FP32 storage sweeps */
    double final_span;         /* span of the last V_new - V */
    double threshold;          /* span rule: eps (1-gamma)/gamma; sup-norm and periodic: eps */
    double dmax, dmin;         /* max and min of the last V_new - V */
    double wall_ms;            /* host wall time of the solve */
    double backup_ms[2];       /* summed backup kernel time of those launches */
    int64_t logical_backups;   /* sum over the sweeps this call ran (and the policy
                                  extraction) of N_S * sum_a |Omega(s,a)| */
    int64_t executed_terms;    /* multiply-adds the kernels actually ran */
    double vhat_shift;         /* gamma/(1-gamma) (dmax + dmin)/2: V + vhat_shift is the
                                  midpoint of the MacQueen bounds on V* (0 when gamma = 1).
                                  The returned V already holds any FP32-storage offset,
                                  so no separate offset is reported */
    double device_ms;          /* stream time from the first to the last kernel of the
                                  solve (HIP events); 0 where not measured: requests
                                  served by the small-instance kernel and
                                  vi_solve_noalloc */
} pvi_result;

typedef struct pvi_mdp pvi_mdp;
typedef struct pvi_server pvi_server;

/* Validate a descriptor and build its tables on the host (demand PMFs, expected
 * one-day rewards, arrival and substitution probabilities).  No device memory is
 * taken until the first solve.  At most 2^31 states, except scenario C (at most
 * 2^40): beyond 2^31 its handle serves heuristic policy_rollouts and
 * heuristic_search only, and solves, single backups, table policies and server
 * requests on it return PVI_E_INVALID.  Errors: PVI_E_INVALID (bad descriptor:
 * sizes, probabilities, gamma, unsupported family/size combination), PVI_E_NOMEM. */
pvi_status mdp_create(const pvi_mdp_desc* desc, pvi_mdp** out);

/* Free host and device memory of a handle.  NULL is accepted. */
pvi_status mdp_destroy(pvi_mdp* mdp);

/* Number of states N_S and actions N_A; -1 for a NULL handle. */
int64_t mdp_num_states(const pvi_mdp* mdp);
int32_t mdp_num_actions(const pvi_mdp* mdp);
/* Number of state digits (A: m+L-1, B: 2(m-1), C: m). */
int32_t mdp_num_digits(const pvi_mdp* mdp);

/* Mixed-radix state encoding, digits most significant first (see families). */
pvi_status mdp_encode(const pvi_mdp* mdp, const int32_t* digits, int64_t* idx);
pvi_status mdp_decode(const pvi_mdp* mdp, int64_t idx, int32_t* digits);

/* The FP64 demand PMF the library built: out[d_max+1] for (product, period). */
pvi_status mdp_demand_pmf(const pvi_mdp* mdp, int32_t product, int32_t period,
                          double* out);

/* C: remaining-life probabilities p_k(a), out[(a_max+1) * m], entry a*m + (k-1). */
pvi_status mdp_life_probs(const pvi_mdp* mdp, double* out);

/* Blocking solve (see the header comment for the stopping rule and policy).
 * Precision PVI_FP32/PVI_FP32_WIDE run FP32 sweeps until the FP64 span reaches
 * the FP32 floor, then FP64 sweeps until the threshold; the last FP64 backup also
 * gives the policy and the best-minus-second Q gap.  With fixed_sweeps > 0
 * exactly that many sweeps run (all in the chosen storage precision) and the
 * policy comes from one FP64 backup of the result.  Returns PVI_E_NOT_CONVERGED
 * after max_sweeps (results still readable).  res may be NULL. */
pvi_status vi_solve(pvi_mdp* mdp, const pvi_solve_opts* opts, pvi_result* res);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the FP64 solve of
 * vi_solve for a scenario-A handle (FIFO or LIFO), with no device or pinned host
 * allocation.  The caller brings the outputs in device memory: d_v[N_S] (FP64,
 * also the first value table of the sweeps; V_0 is written into it: zeros, or
 * opts->v0 copied from the host), d_policy[N_S] (int32) and d_gap[N_S] (FP64).
 * Everything else (control block, tables, work list, span partials and the
 * second value table) lives in a fixed device array of the library, about
 * 33 MiB per device, held until the process ends.  Limits: N_S <= 4,194,304
 * states; the handle's tables and work list within 512 KiB, its span partials
 * within 512 KiB.  Options: precision PVI_FP64, stop_rule SPAN or SUPNORM, no
 * checkpoint files; opts->stream (NULL: the null stream) carries every launch and
 * copy, and the call returns after synchronising it.  The kernels and their
 * order are vi_solve's, so V, policy, gap and sweep counts equal vi_solve's
 * FP64 results bit for bit.  Calls on one device share the array: the library
 * serialises them within a process (each call takes a per-device lock); every
 * value a call reads is written by that call first.  Errors: PVI_E_INVALID (NULL
 * outputs, another family, precision or rule, sizes beyond the limits),
 * PVI_E_DEVICE, PVI_E_NOT_CONVERGED (results still written). */
pvi_status vi_solve_noalloc(const pvi_mdp* mdp, const pvi_solve_opts* opts, double* d_v,
                            int32_t* d_policy, double* d_gap, pvi_result* res);

/* One backup of a caller-given FP64 V (host [N_S]) in the given precision:
 * v_out[N_S] = T(V), policy[N_S] = argmax, q_gap[N_S] = best - second (FP64
 * precision only; NULL allowed).  For parity checks of single sweeps. */
pvi_status vi_backup(pvi_mdp* mdp, int32_t precision, const double* v_in, double* v_out,
                     int32_t* policy, double* q_gap);

/* Checkpoint file (little-endian): the 8 bytes "PVICKPT1", uint32 version (2),
 * uint32 family, uint64 fingerprint of the descriptor, int64 N_S, int32 N_A, int32
 * stop rule, int32 FP64 sweeps done, int32 stopped (1 when the stopping rule had
 * fired at that sweep), int32 H, int32 reserved (0), then four FP64: the threshold
 * the writing solve's rule tested (span rule: eps (1-gamma)/gamma; else eps), and
 * max, min and span of its last V_new - V; then H tables of N_S FP64
 * values: V after the last sweep, then the H - 1 before it (H = 1, or under the
 * periodic rule min(sweeps, P) + 1, the tables its test reads).  Files of version
 * 1 (no four FP64) are still read.  A resume from a file whose rule had fired
 * runs no sweep only when the rule is the same and the file's threshold is no
 * larger than the resuming solve's (its result then reports the file's
 * increments); with a tighter threshold, or a version-1 file, it goes on sweeping.
 * checkpoint_read checks the file against the handle and returns the sweep count,
 * stopped flag and the last table (v: host [N_S], NULL to skip).  Errors:
 * PVI_E_IO (missing, unreadable or short file), PVI_E_INVALID (wrong magic or
 * version, a file of another descriptor).  vi_solve returns the same codes for
 * its checkpoint files (PVI_E_IO also when one cannot be written). */
pvi_status checkpoint_read(const pvi_mdp* mdp, const char* path, double* v, int32_t* sweeps,
                           int32_t* stopped);

/* Results of the last solve: policy[N_S] (and q_gap[N_S], nullable) and the FP64
 * values V[N_S] (= c + v for FP32 storage).  PVI_E_NOT_READY before a solve. */
pvi_status policy_get(const pvi_mdp* mdp, int32_t* policy, double* q_gap);
pvi_status value_get(const pvi_mdp* mdp, double* v);
/* Copy the policy into caller device memory (int32[N_S]) on `stream`. */
pvi_status policy_get_device(const pvi_mdp* mdp, int32_t* d_policy, void* stream);

/* Request server: solves of many MDPs of different sizes, admitted by free HBM
 * within hbm_budget_bytes (0 = 80% of free device memory).  Small scenario-A
 * instances (FIFO, span rule, no v0, both value tables within 60 KB of LDS) go to a
 * persistent slot kernel with small_batch slots (at most as many work groups as stay
 * resident): one work group per slot solves one instance at a time, and a request
 * that arrives while the kernel runs takes the next free slot of that launch
 * (continuous refill).  A launch with no busy slot for 2 ms is stopped (set
 * PVI_SLOT_IDLE_MS in the environment at pvi_server_create to change it); the next
 * small request starts another.  Each ticket's
 * results stay in its pvi_mdp handle, which the caller keeps alive until the
 * ticket completes.  A handle that had no device state when its request started
 * gets its results in host memory and its device buffers freed once the solve
 * ends (policy_get, value_get and policy_get_device read them from there).
 * A request waiting for device memory re-reads the free memory at least every
 * 2 ms, so memory freed outside the server (a client's mdp_destroy) admits it
 * without any server call.  With PVI_SERVER_LOG=<path> in the environment at
 * pvi_server_create, the server appends one line per request event (submit,
 * start, done, busy, cancel: time in ms, ticket, class, worker, bytes, status). */
pvi_status pvi_server_create(int64_t hbm_budget_bytes, int32_t small_batch,
                             pvi_server** out);
pvi_status pvi_server_destroy(pvi_server* server);
pvi_status vi_batch_submit(pvi_server* server, pvi_mdp* const* mdps,
                           const pvi_solve_opts* opts, int32_t n, uint64_t* tickets_out);
pvi_status vi_poll(pvi_server* server, uint64_t ticket, pvi_result* res);
pvi_status vi_wait(pvi_server* server, uint64_t ticket, int64_t timeout_us,
                   pvi_result* res);
/* State of a ticket, for progress reports and diagnosis of slow requests.
 * Times are milliseconds since pvi_server_create (-1 before the event). */
typedef struct pvi_ticket_info {
    int32_t state;        /* 0 queued, 1 running, 2 done */
    int32_t small;        /* 1: batched small-instance path, 0: sweep loop */
    int32_t worker;       /* server worker that took it; -1 while queued */
    int32_t sweeps;       /* sweep-loop requests: sweeps completed at the last host check */
    int32_t status;       /* pvi_status once done, else PVI_E_NOT_READY */
    int32_t launch;       /* small requests: number of the slot-kernel launch that serves
                             it (1 = the server's first); 0 for sweep-loop requests */
    int64_t bytes;        /* device bytes a sweep-loop request holds while it runs */
    double t_submit_ms, t_start_ms, t_done_ms;
} pvi_ticket_info;
pvi_status vi_ticket_info(pvi_server* server, uint64_t ticket, pvi_ticket_info* out);
/* Latency statistics over completed tickets (milliseconds, submit to done). */
pvi_status pvi_server_stats(pvi_server* server, double* p50_ms, double* p99_ms,
                            int64_t* completed);

/* ------------------------------------------------------------------ rollouts
 * Policy evaluation by simulation (Simulation section): n_rollouts rollouts of
 * warmup_days + horizon_days days from start_state under each policy; the return
 * of a rollout is sum_{t < horizon} gamma^t R_{warmup + t}, and its KPIs, counted
 * over the horizon days, are the service level (100 x demand met / demand, 100
 * with no demand; scenario B counts demand of product 0 met by product 1 as met),
 * the wastage (100 x units expired / units received into stock, 0 with none
 * received) and the holding (units in stock at the end of the day, per day; the
 * units that expire that night count in scenario C and not in A or B).
 *
 * Randomness: Philox4x64-10 (Salmon, Moraes, Dror and Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC 2011), key (seed, 0), counter (rollout, day,
 * block, 0); word w maps to u = (x >> 11) 2^-53.  Block 0 word 0 draws the demand
 * of product 0 (the smallest d with u < CDF(d), else d_max), word 1 that of
 * product 1; unit i of the day uses word i%4 of block 1 + i/4: in scenario C the
 * remaining life of the i-th unit ordered (the smallest k with u < p_1(a) + ... +
 * p_k(a), else m), in scenario B whether the i-th unmet customer of product 0
 * accepts product 1 (u < subst_rho).  Every policy of a call sees the same
 * numbers.
 *
 * Policies (Simulation optimization of each scenario):
 *   TABLE           action per state: `table` (host, n_states entries in
 *                   [0, n_actions)), or NULL for the policy of the handle's last
 *                   solve; n_policies = 1.
 *   BASE_STOCK      scenario A: order [S - I]^+, I = stock on hand and in transit;
 *                   params[0] = S.
 *   MOD_BASE_STOCK  scenario B: per product k, floor([S_k - I_k + [X1_k - mu_k]^+]^+)
 *                   with I_k its stock, X1_k its oldest stock and mu_k its mean
 *                   demand; params[0..1] = S_0, S_1.
 *   S_S             scenario C: [S_tau - I]^+ when I <= s_tau and s_tau < S_tau,
 *                   else 0, for weekday tau; params[2 tau] = s_tau,
 *                   params[2 tau + 1] = S_tau.
 * Heuristic orders are placed as the formulas give them, without a cap at a_max
 * (a heuristic's largest order is its S; the scenario-B search of the
 * Simulation-optimization passage runs S_k up to 2 a_max[k]), except scenario C's,
 * capped at a_max, the range of its remaining-life distribution.  Parameters
 * must lie in [-2^20, 2^20], and horizon_days x the largest daily count (demand,
 * or 2 (m + L) x the largest order) must stay below 2^31. */
typedef enum {
    PVI_POLICY_TABLE = 0,
    PVI_POLICY_BASE_STOCK = 1,
    PVI_POLICY_MOD_BASE_STOCK = 2,
    PVI_POLICY_S_S = 3
} pvi_policy_kind;

#define PVI_POLICY_PARAMS 16

typedef struct pvi_rollout_opts {
    uint32_t struct_size;      /* sizeof(pvi_rollout_opts); at least the offset of
                                  product_kpis */
    int32_t kind;              /* pvi_policy_kind; must suit the handle's family */
    const int32_t* table;      /* TABLE: host [n_states], or NULL (last solved policy) */
    const int32_t* params;     /* heuristics: host [n_policies][PVI_POLICY_PARAMS] */
    int32_t n_policies;        /* >= 1 (TABLE: 1) */
    int32_t n_rollouts;        /* >= 1; n_policies x n_rollouts < 2^31 */
    int32_t warmup_days;       /* >= 0 */
    int32_t horizon_days;      /* >= 1 */
    uint64_t seed;
    int64_t start_state;       /* state index at day 0, 0 = empty */
    void* stream;              /* optional hipStream_t; NULL = a stream of the call */
    /* Per-product KPIs of the two-product families (Appendix B, KPI tables),
     * optional host outputs, NULL to skip (must be NULL for one product).  A
     * caller whose struct_size ends before these fields gets neither. */
    double* product_kpis;      /* [n_policies][n_rollouts][2][3]: service, wastage,
                                  holding of product k alone */
    double* product_stats;     /* [n_policies][2][6]: mean and sample standard
                                  deviation of the three KPIs of product k */
} pvi_rollout_opts;

/* Run the rollouts on the device and return, per policy, stats[8 p .. 8 p + 7] =
 * mean and sample standard deviation (n - 1) of the return, the service level,
 * the wastage and the holding.  returns ([n_policies][n_rollouts]) and kpis
 * ([n_policies][n_rollouts][3]: service, wastage, holding) are optional host
 * outputs (NULL to skip).  Per product, the service level of the product whose
 * unmet customers may substitute counts the units the other product gave them
 * (scenario B with lead time 0: product 0; with lead time 1: product 1), and
 * the wastage and holding count the product's own units.  Blocks until done.
 * Errors: PVI_E_INVALID (options, a kind that does not suit the family, table
 * entries out of range, per-product outputs for one product), PVI_E_NOT_READY
 * (TABLE with NULL table before any solve), PVI_E_NOMEM, PVI_E_DEVICE.  Device
 * buffers are taken and released within the call. */
pvi_status policy_rollouts(pvi_mdp* mdp, const pvi_rollout_opts* opts, double* stats,
                           double* returns, double* kpis);

/* Simulation optimization over a grid of heuristic parameter vectors (a
 * heuristic kind, n_policies candidates, common random numbers): the rollouts of
 * policy_rollouts, then *best = the candidate with the highest mean return, ties
 * to the lowest index.  stats as for policy_rollouts (may be NULL); the
 * per-product outputs of opts are filled as by policy_rollouts. */
pvi_status heuristic_search(pvi_mdp* mdp, const pvi_rollout_opts* opts, double* stats,
                            int32_t* best);

/* Thread-local message of the last failing call on this thread. */
const char* pvi_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PVI_H */
