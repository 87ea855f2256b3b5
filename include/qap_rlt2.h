/*
 * qap_rlt2.h -- C ABI of the MI355X RLT2 dual-ascent library.
 *
 * The library computes lower bounds for the Quadratic Assignment Problem
 *     min_perm  sum_i b_{i,perm(i)} + sum_{i,j} f_ij d_{perm(i),perm(j)}
 * (Lawler form, Eq. 1.1 of Date & Nagi, arXiv:1710.03732) by the Lagrangian
 * dual ascent on the level-2 RLT formulation (RLT2-DA, Section 2.3,
 * Algorithm 1, in its one-phase "fast" form F1 of Section 3.4), and solves
 * small QAPs exactly by branch-and-bound on those bounds (Section 4).
 *
 * Conventions for every entry point:
 *   - return 0 (QAP_OK) on success, a negative QAP_E* code on failure; no C++
 *     exception crosses the ABI; on failure the outputs are left untouched
 *     and qap_last_error(h) describes the problem;
 *   - "host" pointers are ordinary CPU memory, read or written during the
 *     call only (the caller keeps ownership); "device" pointers are HIP
 *     device memory on the handle's device;
 *   - all matrices are row-major; sizes are element counts;
 *   - a handle is used by one host thread at a time; the library keeps no
 *     global state;
 *   - results are deterministic: equal inputs and parameters give bitwise
 *     equal outputs (up to the sign of zero).
 *
 * Data layout in device memory (also the layout of exported state):
 *   n facilities/locations; m = n - 2.
 *   Pair index ("tile") t(i,p,j,q) for i != j, p != q:
 *       t = ((i*n + p)*(n-1) + j')*(n-1) + q',   j' = j - [j>i], q' = q - [q>p];
 *       T = n^2 (n-1)^2 tiles.
 *   y-level array (T doubles): entry (i,j,p,q) at t(i,p,j,q).  The Y-LAP of
 *       (i,p) is the contiguous (n-1)x(n-1) block t(i,p,.,.).
 *   z-level array (T*m*m doubles, tile-major): entry (i,j,k,p,q,r) at
 *       t(i,p,j,q)*m*m + k''*m + r'',  k'' = k - [k>i] - [k>j],
 *       r'' = r - [r>p] - [r>q].  Tile t is the Z-LAP of (i,j,p,q).
 *   x-level array (n*n doubles): entry (i,p) at i*n + p.
 */
#ifndef QAP_RLT2_H
#define QAP_RLT2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QAP_OK 0
#define QAP_EINVAL (-1)       /* bad argument: n out of range, NULL required pointer,
                                 non-finite data, kappa/phi outside [0,1] */
#define QAP_ENOMEM (-2)       /* device arena larger than free memory (checked first) */
#define QAP_EDEVICE (-3)      /* HIP runtime error (text in qap_last_error) */
#define QAP_ESTATE (-4)       /* call out of order, or bad checksum on import */
#define QAP_EUNSUPPORTED (-5) /* n outside 3..64, or a call a HALF, F2, S1 or annealing handle refuses */

typedef struct qap_ctx *qap_handle;

/* Device memory callbacks; NULL alloc selects hipMalloc/hipFree. */
typedef void *(*qap_alloc_fn)(size_t bytes, void *ctx);
typedef void (*qap_free_fn)(void *ptr, void *ctx);

/* Dual-ascent parameters.  kappa_* are the fractions of slack moved by the
 * Type 1 (z), Type 2 (y) and Type 3 (x) ascent rules (Eqs. da:rule1-3); phi_z
 * is the share each of the five symmetric partners receives (the phi^z_k of
 * the rules, all equal); phi_y the share of the y-pair rule (Eq. da:yrule1).
 * qap_default_params() gives the FULL preset: kappa_z = 5/6,
 * kappa_y = kappa_x = 1, phi_z = 1/5, phi_y = 1/2.
 *
 * scheme = QAP_SCHEME_HALF selects the HALF scheme of Section 5: only the
 * z variables whose first two facilities ascend (i < j) are kept; the Z-LAPs
 * of the other n^2 (n-1)^2 / 2 tiles are not solved and their entries stay 0.
 * In the sweep an upper member keeps (1 - kappa_z) of its slack and receives
 * phi_z of each upper partner's share plus 1/3 of each lower partner's (the
 * lower members, with no multiplier of their own, give their whole y and x
 * shares).  HALF needs phi_z = 1/2 (two upper partners), the scalar Z-LAP
 * mapping (zlap_lanes 0 or -1) and starts from the zero z costs of
 * qap_rlt2_init; multiplier tracking, qap_set_multipliers, warm starts and
 * branch-and-bound refuse a HALF handle (QAP_EUNSUPPORTED).  The HALF preset
 * is kappa_z = 2/3, kappa_y = kappa_x = 1, phi_z = phi_y = 1/2. */
#define QAP_SCHEME_FULL 0
#define QAP_SCHEME_HALF 1

typedef struct qap_params {
    double kappa_z, kappa_y, kappa_x;
    double phi_z;
    double phi_y;
    double min_gap;        /* stop when (UB - LB)/|UB| < min_gap; 0 disables */
    int device;            /* HIP device ordinal */
    int zlap_lanes;        /* Z-LAP mapping: lanes per LAP group (8/16/32/64), -1 one
                              LAP per wavefront, -2 two per wavefront (m <= 32);
                              0 = chosen by the autotuner (see qap_zlap_mapping) */
    int zlap_cols;         /* columns per lane for lane groups (1/2/4); 0 = autotuned */
    int timing;            /* 1: launch each kernel between HIP events on the
                              handle's stream and report per-phase device time
                              in qap_da_stats (no graph replay) */
    int scheme;            /* QAP_SCHEME_FULL (0) or QAP_SCHEME_HALF (1) */
    int two_phase;         /* 0: F1; 1: F2, the two-phase variant of Section 3.4:
                              from t = 1 on, after the Z-LAPs every orbit's
                              slacks are pooled (the members with slack > 0 drop
                              to 0, their total is shared equally by those with
                              slack <= 0; unchanged if either set is empty) and
                              the Z-LAPs are solved again, their values adding to
                              the y costs as well.  FULL scheme only; tracking
                              (outside S2), child folds, batched and B&B ascent
                              refuse an F2 handle (QAP_EUNSUPPORTED) */
    int slow;              /* 0: fast (F-form); 1: S1, the slow variant of Section 3.4:
                              the z multipliers v move by F1's sweep rule (Eq.
                              ch4:proof:2) and each iteration solves the LAPs on
                              the full costs b + f_ii d_pp, f_ij d_pq and -v, so
                              every X-LAP value is a whole bound (the left-hand
                              side of Eq. ch4:proof:4).  The y multipliers stay 0
                              (Theorem 1's setting; the y-pair rule is not
                              applied).  v lives in the tracking array
                              (qap_get_multipliers).  With two_phase = 1 this is
                              S2: the pooling also moves each pooled member's v by
                              its old slack minus its new one.  FULL, not with
                              annealing; import, multiplier setting, warm starts,
                              folds, batched and B&B ascent refuse S1/S2 handles */
    qap_alloc_fn alloc;    /* optional device allocator of the handle's arena
                              and bound trace (the branch-and-bound search
                              gives its node handles one that reuses the
                              arenas of finished nodes) */
    qap_free_fn free_fn;
    void *alloc_ctx;
} qap_params;

typedef struct qap_da_stats {
    int iterations_done;   /* iterations run by this call */
    int t;                 /* iterations run since init */
    double lb;             /* the state's bound: the last X-LAP bound, less what a
                              Type 4 step after it gave away (without annealing
                              the bounds never fall, so this is also the best) */
    double ub;             /* best X-LAP permutation cost (+inf if none) */
    double gap;            /* (ub - max(lb, best_lb))/|ub| */
    int proven;            /* 1 when lb certifies ub optimal (feasibility check) */
    int sa_steps;          /* Type 4 steps taken since init (qap_set_annealing) */
    long long laps;        /* LAPs solved by this call: iters*(T + n^2 + 1), T/2 for
                              HALF, 2T at t >= 1 for F2 */
    long long dijkstra_steps; /* Dijkstra steps of all LAPs of this call */
    double seconds;        /* wall time of the call (device-synchronised) */
    double ms_sweep;       /* with params.timing: summed device milliseconds of */
    double ms_zlap;        /* the ascent sweep (+x/y scaling), the Z-LAP kernel, */
    double ms_ylap;        /* the Y-LAP kernel and the X-LAP kernel over the call */
    double ms_xlap;        /* (with annealing, the X phase includes the Type 4 step) */
    double best_lb;        /* best bound of any iteration since init (-inf before any) */
} qap_da_stats;

typedef struct qap_bnb_params {
    int batch;             /* open nodes per batched launch (default 256) */
    int node_iters;        /* dual-ascent iteration cap per node (default 100) */
    int window;            /* early stop window (default 25) */
    int root_iters;        /* iterations at the root (default node_iters) */
    double min_improve;    /* stop a node when its bound rose by less than
                              min_improve*max(1,|UB|) over `window` (2e-4) */
    double ub0;            /* initial incumbent value (+inf allowed) */
    int enum_below;        /* enumerate nodes with at most this many free
                              facilities (default 3) */
    int rule;              /* branching rule (3 = lowest interaction first) */
    int depth_cap;         /* warm-start children from their parent's reduced
                              costs down to this depth; deeper nodes start
                              cold from their restricted QAP, so no parent
                              state is kept for them (Section 4's depth limit
                              d; 0 = no cap, the default) */
    int symmetry;          /* 1: symmetry elimination (Section 4, used there on
                              grid instances): with the location automorphisms
                              of D and B (qap_location_automorphisms), a child
                              is not built when an automorphism that keeps every
                              placed facility's location maps its location to a
                              lower one; 0 (default): off */
} qap_bnb_params;

typedef struct qap_bnb_stats {
    long long nodes;       /* nodes bounded (including enumerated leaves' parents) */
    long long da_iters;    /* node dual-ascent iterations */
    long long batches;     /* batched launches */
    long long enumerated;  /* leaves evaluated by enumeration */
    double seconds;
    long long symmetric_skipped; /* children not built by the symmetry elimination */
    long long automorphisms;     /* location automorphisms used, identity included */
    double node_bytes;           /* algorithmic HBM bytes of all node iterations: per
                                    iteration of a node of size n', m' = n' - 2,
                                    T' = n'^2 (n'-1)^2, V' = T' m'^2:
                                    8 (4 V' + 8 T' + 10 n'^2) (the sweep and the
                                    Z-LAPs read and write the z array once each,
                                    plus the y and x arrays) */
} qap_bnb_stats;

/* Location automorphisms of a QAP (host only, no device work): the
 * permutations sigma of the locations with D[sigma p][sigma q] = D[p][q] for
 * all p, q and B[i][sigma p] = B[i][p] for all i, p (B may be NULL: zero),
 * under which every assignment keeps its cost.  D, B: host, n*n row-major.
 * out: host, cap*n int32, permutation a at out[a*n .. a*n+n-1] (location p
 * goes to out[a*n+p]); *count gets how many were written, the identity
 * first.  A search budget and cap bound the work; every permutation written
 * is exact even when the list is not the whole group.  Errors: QAP_EINVAL. */
int qap_location_automorphisms(int n, const double *D, const double *B, int cap, int32_t *out, int *count);

/* Node rules of qap_batch_dual_ascent (branch-and-bound control, Section 4
 * and the early termination of Section 5.4).  Each handle runs at most
 * `iters` more iterations and stops on its own when (a) its bound certifies
 * its incumbent or its min_gap is reached, (b) it is fathomed against ub_cut
 * (ceil(LB - tol) >= min(ub_cut, own UB) for integer data, tol =
 * 1e-9*max(1,|UB|)), or (c) window > 0, min_improve > 0 and its bound rose
 * by less than min_improve*max(1,|UB|) over the last `window` iterations. */
typedef struct qap_batch_params {
    int iters;
    int window;
    double min_improve;
    double ub_cut;         /* +inf for none */
    int zlap_lanes;        /* Z-LAP mapping: 0 = chosen by timing per tile
                              size; 8, 16, 32, 64 = lane groups of that many
                              lanes (>= the largest m); -1 = one tile per
                              wavefront, -2 = two (m <= 32).  Every mapping
                              gives the same results.  QAP_EINVAL otherwise. */
    int reserved;          /* 0 */
} qap_batch_params;

typedef struct qap_batch_stats {
    long long iterations;  /* iterations of all handles so far (sum of t) */
    int stopped;           /* handles stopped */
    int fathomed;          /* ... by rule (a) or (b) */
    int window_stops;      /* ... by rule (c) */
    int compactions;       /* times the stopped nodes were dropped from the
                              batch's launches (no effect on results) */
    double seconds;
} qap_batch_stats;

/* State header of qap_export_state / qap_import_state. */
typedef struct qap_state_header {
    int n;
    int t;
    double lb, ub;
    uint64_t checksum;     /* FNV-1a over n, t, lb, ub and the three arrays */
} qap_state_header;

const char *qap_version(void);

/* FULL preset (see qap_params). */
int qap_default_params(qap_params *p);

/* Device bytes qap_rlt2_init will allocate for size n (0 if n unsupported). */
size_t qap_workspace_bytes(int n, const qap_params *p);

/* Initialise the dual ascent for a QAP of size n (Algorithm 1 step 1;
 * RLT1/RLT2 costs of Section 2.1): x costs b_ip + f_ii d_pp, y costs
 * C_ijpq = f_ij d_pq, z costs 0 (the QAP has no cubic terms), LB = 0.
 * F, D: host n*n flows and distances; B: host n*n fixed costs or NULL (zero).
 * Copies the data to the device; returns the handle in *out.
 * Errors: QAP_EINVAL (NULL F/D/out, non-finite entry, bad params),
 * QAP_EUNSUPPORTED (n < 3 or n > 64), QAP_ENOMEM, QAP_EDEVICE. */
int qap_rlt2_init(const double *F, const double *D, const double *B, int n,
                  const qap_params *p, qap_handle *out);

int qap_destroy(qap_handle h);

/* The Z-LAP mapping a handle uses (Section 2.3 "LAP Solution": every mapping
 * solves the same LAPs with bitwise-identical results; the mapping decides
 * only the speed).  With zlap_lanes = 0 the first qap_dual_ascent call
 * measures every mapping that holds m = n-2 on a fixed synthetic batch of
 * tiles and keeps the fastest, once per process, device and m (and, when the
 * environment variable QAP_TUNE_CACHE names a file, in that JSON file, keyed
 * by GPU architecture, kernel, m and kernel revision, for later processes).
 * Before that call the rule-based choice is reported.  lanes: lanes per LAP
 * group, or -1 / -2 for one / two LAPs per wavefront; cols: columns per lane;
 * tuned_us: the chosen mapping's time over the synthetic batch in
 * microseconds, or -1 if it was not measured.  Any output pointer may be
 * NULL.  Errors: QAP_EINVAL (h NULL). */
int qap_zlap_mapping(qap_handle h, int *lanes, int *cols, double *tuned_us);

/* Type 4 ascent with simulated annealing (Section 2.3's last ascent rule,
 * Section 5's schedule).  After the X-LAP of every iteration t >= 1 whose
 * bound nu is positive and does not stop the run, a random fraction
 * kappa^lb = kappa_max * u of nu is split over one fraction per facility and
 * one per location (in proportion to random weights); facility i's share is
 * added to every x slack of row i, location p's to every slack of column p,
 * so every permutation's cost = LB + slacks still holds.  The offer A is
 * taken when u' <= exp(-A / T), T = t0 * cool^floor(t / period), and LB then
 * drops by A; the trace keeps each iteration's X-LAP bound and best_lb the
 * best of them.  Random numbers: SplitMix64 (Steele, Lea and Flood 2014)
 * seeded with `seed`, its outputs t*(2n+2) + 1 ... + 2n+2 for iteration t,
 * so a run is reproducible.  Section 5 uses t0 = 4 % of the best known UB,
 * kappa_max = 0.25, cool = 0.99, period = 100. */
typedef struct qap_sa_params {
    double t0;             /* initial temperature (cost units); <= 0: annealing off */
    double kappa_max;      /* largest fraction of the bound offered per step, [0, 1] */
    double cool;           /* temperature factor per period, (0, 1] */
    int period;            /* iterations per cooling step, >= 1 */
    int pad;
    uint64_t seed;
} qap_sa_params;

/* Turn annealing on (p->t0 > 0) or off (p NULL or t0 <= 0) for the next
 * iterations of h.  Errors: QAP_EINVAL (parameters), QAP_EUNSUPPORTED (h
 * tracks multipliers).  A handle with annealing on refuses tracking, child
 * folds, batched and B&B ascent (QAP_EUNSUPPORTED). */
int qap_set_annealing(qap_handle h, const qap_sa_params *p);

/* Run `iters` more iterations (Algorithm 1 steps 2-5): ascent sweep of the
 * Type 1-3 rules (t >= 1), Z-LAPs (twice with pooling under F2), y-pair rule
 * (t >= 1), Y-LAPs, X-LAP, bound and incumbent update, and a Type 4 step if
 * annealing is on.  Stops early once the bound proves the incumbent optimal
 * or the gap falls below min_gap.  Writes the state's bound (qap_da_stats.lb)
 * to *lb_out and the X-LAP duals alpha (rows, n) and beta (columns, n) of
 * the last iteration to alpha_out/beta_out (host, nullable); st nullable.
 * Errors: QAP_EINVAL (iters < 0), QAP_EDEVICE. */
int qap_dual_ascent(qap_handle h, int iters, double *lb_out, double *alpha_out,
                    double *beta_out, qap_da_stats *st);

/* Host copy of the bound after each iteration so far; *len gets the count. */
int qap_get_trace(qap_handle h, double *lb, int cap, int *len);

/* Last X-LAP assignment and best permutation (host, n each, nullable);
 * perm[i] is the location of facility i. */
int qap_get_assignment(qap_handle h, int32_t *xperm, int32_t *best_perm);

/* Copy the current reduced costs (x: n*n, y: T, z: T*m*m, host, nullable) in
 * the layout above.  After k >= 1 iterations these are the LAP dual slacks
 * pi_x, pi_y, pi_z of the last iteration; before the first, the initial
 * costs.  For every permutation the identity
 *   cost = lb + sum x[i,s_i] + sum y[i,j,s_i,s_j] + sum z[i,j,k,s_i,s_j,s_k]
 * holds up to rounding. */
int qap_export_state(qap_handle h, qap_state_header *hdr, double *x, double *y, double *z);

/* Reduced costs of selected Z-LAP tiles only (the z part of
 * qap_export_state for `count` tile indices t, see the layout above).
 * tiles: host, count tile indices; out: host, count*m*m doubles.
 * Errors: QAP_EINVAL (index out of range, NULL pointer). */
int qap_export_z_tiles(qap_handle h, const int64_t *tiles, int count, double *out);

/* Replace the state with exported arrays (resume).  hdr->checksum must match;
 * the next iteration runs with t = hdr->t.  Errors: QAP_ESTATE on mismatch;
 * QAP_EINVAL on a HALF handle when a z entry of a tile with i > j is not 0. */
int qap_import_state(qap_handle h, const qap_state_header *hdr, const double *x,
                     const double *y, const double *z);

/* Use the given HIP stream (hipStream_t passed as void*) for all work.  On
 * the null stream (0) iterations are launched kernel by kernel instead of as
 * a replayed HIP graph, since HIP cannot capture that stream. */
int qap_set_stream(qap_handle h, void *hip_stream);

/* Solve the QAP held by h to optimality by branch-and-bound (Section 4):
 * polytomic branching in Rule-3 facility order, children warm started from
 * the parent's reduced costs (qap_fold_child), up to p->batch open nodes of
 * uneven size per batched dual ascent (qap_batch_dual_ascent), taken
 * depth-first from a stack; nodes with at most enum_below free facilities
 * are enumerated.  The batched Z-LAP mapping of a tile size is measured on
 * this search's own tiles by its first batch of that size with at least
 * 1e8 tile iterations of Z-LAP work (smaller batches take the process-wide
 * choice; the environment variable QAP_SEARCH_TUNE_WORK replaces 1e8);
 * results do not depend on it.  h's own state is not changed (the
 * root restarts from the initial costs).  perm_out (host, n): optimal
 * permutation; *obj_out its
 * exact cost.  p NULL selects the defaults.  Errors: QAP_EUNSUPPORTED
 * (n > 24), QAP_ESTATE (no permutation below ub0), QAP_EINVAL. */
int qap_bnb_solve(qap_handle h, const qap_bnb_params *p, int32_t *perm_out, double *obj_out,
                  qap_bnb_stats *st);

/* Warm-start a child node from h's current reduced costs (the children of a
 * branch-and-bound node start from their parent's multipliers, Section 4):
 * fix facility l to location s (indices of h's own problem, 0-based).  The
 * child is a handle of size n-1 whose QAP is h's restricted to the other
 * facilities and locations, with the fixed pair's cross terms folded into its
 * fixed costs and its constant cost added to an internal offset, so its
 * incumbents are full-problem costs.  Its bound starts at h's bound plus
 * pi_x[l][s]; every reduced-cost entry that holds (l,s) moves one level down
 * and the rest is restricted; it runs from t = 0.  h must have run at least
 * one iteration.  The child shares h's stream.  Errors: QAP_ESTATE (no
 * iteration yet), QAP_EUNSUPPORTED (n < 4), QAP_EINVAL, QAP_ENOMEM. */
int qap_fold_child(qap_handle h, int l, int s, qap_handle *child);

/* Advance `count` independent handles (sizes may differ, one device) by one
 * set of batched kernels per phase and iteration, replayed from one HIP
 * graph, with the node rules above.  Each handle's trajectory is exactly the
 * one qap_dual_ascent would produce until it stops.  Every 4 iterations the
 * host reads how many handles have stopped: it returns once all have, and
 * once the stopped ones hold an eighth of the launched work it drops them
 * from the launches (a handle already stopped at the call is never launched).
 * hs: host array of handles; st nullable. */
int qap_batch_dual_ascent(qap_handle *hs, int count, const qap_batch_params *bp, qap_batch_stats *st);

/* qap_batch_dual_ascent for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments and the same results, bitwise; it allocates
 * nothing.  Its node table, prefix tables, stop counter, stop flags and a
 * copy of the handles' scalar blocks live in a file-scope device array of
 * QAP_BATCH_STATIC_BYTES per GPU (held by each GPU
 * the library runs on until the process ends), set up on the first call on
 * a device; the iterations are launched one by one (no graph is captured or
 * instantiated), and the batched Z-LAP mapping is the one the autotuner
 * already chose in this process or the QAP_TUNE_CACHE file holds, else the
 * smallest lane group that holds the tiles (every mapping computes the same
 * LAPs).  Every call on a GPU shares that GPU's array and starts by
 * rewriting what it uses (the stop counter is cleared by a kernel): calls
 * that overlap on one GPU race and must be serialised by the caller.
 * Errors: QAP_EINVAL (count outside 0..QAP_BATCH_STATIC_MAX_NODES, tables
 * larger than the array), QAP_ESTATE (a handle's bound trace, 1024 entries
 * from init and grown only by the allocating calls, has no room for the
 * iterations), and those of qap_batch_dual_ascent. */
#define QAP_BATCH_STATIC_BYTES 131072
#define QAP_BATCH_STATIC_MAX_NODES 256
int qap_batch_dual_ascent_static(qap_handle *hs, int count, const qap_batch_params *bp, qap_batch_stats *st);

/* Scalars of a handle: iterations run, bound, incumbent, stop flag and the
 * batch rule that stopped it (0 none, 1 certificate/fathomed, 2 window,
 * 3 min_gap).  Pointers nullable. */
int qap_node_status(qap_handle h, int *t, double *lb, double *ub, int *stopped, int *reason);

/* Batched LAP solver (the Hungarian method used for every Z-, Y- and X-LAP,
 * Section 2.3 "LAP Solution"), exposed for validation.  cost: device,
 * count*m*m doubles (count matrices, row-major); outputs (device): u
 * (count*m, row duals), v (count*m, column duals), theta (count, optimal
 * values), row_of_col (count*m, the row assigned to each column).  All
 * pointers device memory; stream is a hipStream_t or NULL.  lanes/cols select
 * the mapping of LAPs with m <= 64 (0 = default): one LAP per wavefront or
 * per lane group, the matrix in LDS.  LAPs with 64 < m <= 1024 run one per
 * block of 256 threads (block-per-LAP; lanes/cols ignored), the matrix read
 * from global memory; the results are the same algorithm's, bitwise.
 * Errors: QAP_EINVAL (m < 1 or m > 1024, count < 0, NULL pointer),
 * QAP_EDEVICE. */
int qap_lap_batch(const double *cost, int count, int m, double *u, double *v, double *theta,
                  int32_t *row_of_col, int lanes, int cols, void *stream);

/* Text of the last error on h (or of the last failed init when h is NULL). */
const char *qap_last_error(qap_handle h);

/* ---------------------------------------------------------------------------
 * Lagrange multipliers and the learned warm start.
 *
 * The F1 transfers are multiplier updates of the Lagrangian dual LRLT2(u, v)
 * (Section 3.1): per ascent sweep, z entry e's multiplier v_e moves by
 * g_e - phi_z * sum_{f != e} g_f over its orbit (its own kappa-shares minus
 * what its partners pass to it, Eq. ch4:proof:2); per y-pair rule, u moves by
 * phi_y * (own - partner) (Eq. da:yrule1).  Both sum to zero over every orbit
 * (the six z variables of one set {(i,p),(j,q),(k,r)}, tied by Eq.
 * rlt2:con3) and every pair (ijpq, jiqp).  Any zero-sum (u, v) gives a valid
 * bound (weak duality, Eq. lgduality), so a run may restart from the costs
 * (b + f_ii d_pp, C - u, -v): the "S-form" start.
 *
 * Orbit ids: o = tri * n(n-1)(n-2) + (p*(n-1) + q')*(n-2) + r'', with tri
 * the index of the facility triple i<j<k in lexicographic order,
 * q' = q - [q>p], r'' = r - [r>p] - [r>q]; 0 <= o < qap_orbit_count(n).
 * Members in the order (A,B,C),(A,C,B),(B,A,C),(B,C,A),(C,A,B),(C,B,A) of
 * A=(i,p), B=(j,q), C=(k,r); member (P1,P2,P3) is the z entry
 * (P1.fac, P2.fac, P3.fac, P1.loc, P2.loc, P3.loc).
 * ------------------------------------------------------------------------- */

/* Start (on != 0: allocate, zero) or stop (0: free) tracking the multipliers
 * of the single-handle dual ascent.  Tracking costs T*m*m + T doubles of
 * device memory and one more read and write of that array per sweep.
 * Tracked handles are rejected by qap_batch_dual_ascent (QAP_ESTATE).  An
 * S1/S2 handle tracks from its first iteration on (its multipliers are its
 * state): on is then a no-op and off is refused.  HALF, F2 and annealing
 * handles refuse tracking.  Errors: QAP_ENOMEM, QAP_EDEVICE,
 * QAP_EUNSUPPORTED. */
int qap_track(qap_handle h, int on);

/* Device allocator for this handle's later allocations: tracking arrays
 * and the temporary buffers of the learned calls (the arena and the bound
 * trace keep the allocator of qap_params the handle was created with).  alloc NULL selects
 * hipMalloc/hipFree; a non-NULL alloc needs free_fn.
 * Errors: QAP_EINVAL, QAP_ESTATE (tracking arrays live). */
int qap_set_allocator(qap_handle h, qap_alloc_fn alloc, qap_free_fn free_fn, void *ctx);

/* Host copies of the tracked multipliers since tracking (re)started:
 * v (T*m*m doubles, z layout), u (T doubles, y layout); each nullable.
 * Errors: QAP_ESTATE (tracking off). */
int qap_get_multipliers(qap_handle h, double *v, double *u);

/* Restart at t = 0 from the S-form costs (b + f_ii d_pp, C - u, -v) with
 * LB = 0 (Algorithm 1 step 1 with given multipliers).  v: host, T*m*m
 * doubles (z layout) or NULL (zero); u: host, T doubles (y layout) or NULL.
 * Each orbit of v and each pair of u must sum to zero within 1e-9 of the
 * largest magnitude.  Tracking, if on, restarts from zero.
 * Errors: QAP_EINVAL (non-finite value, not zero-sum), QAP_EDEVICE. */
int qap_set_multipliers(qap_handle h, const double *v, const double *u);

/* Number of orbits of size n: C(n,3) * n(n-1)(n-2). */
int qap_orbit_count(int n, int64_t *count);

/* Scale of the warm start's outputs: max(1, max|F|) * max(1, max|D|) / (n-2). */
int qap_multiplier_scale(qap_handle h, double *scale);

/* Features of `count` orbits (ids: device int64; x: device, count*32
 * float32, row per orbit).  With Fn = F/sF, Dn = D/sD (sF, sD the largest
 * magnitudes, at least 1), sym(M)_ab = (M_ab + M_ba)/2, fa_a = sum_l
 * (Fn_al + Fn_la)/2n, dl likewise for Dn, Xn = (b + f_ii d_pp)/(sF sD), fbar
 * and dbar the off-diagonal means of Fn and Dn:
 *   0-5 Fn_ij Dn_pq, Fn_ji Dn_qp, Fn_ik Dn_pr, Fn_ki Dn_rp, Fn_jk Dn_qr, Fn_kj Dn_rq;
 *   6-8 sym(Fn) of ij, ik, jk;  9-11 sym(Dn) of pq, pr, qr;
 *   12-14 fa_i, fa_j, fa_k;  15-17 dl_p, dl_q, dl_r;  18-20 Xn_ip, Xn_jq, Xn_kr;
 *   21 1/(n-2);  22-24 sym(Fn) of ij, ik, jk times dbar;
 *   25-27 sym(Dn) of pq, pr, qr times fbar;  28-31 zero.
 * Ids outside [0, qap_orbit_count(n)) give rows of NaN.
 * Runs on the handle's stream and waits for it.
 * Errors: QAP_EINVAL, QAP_ENOMEM, QAP_EDEVICE. */
int qap_orbit_features(qap_handle h, const int64_t *ids, int64_t count, float *x);

/* Training targets: tracked v of each listed orbit's six members divided by
 * `scale` (FP64) and rounded to float32 (t: device, count*6; NaN rows for
 * ids out of range).  Runs on the handle's stream and waits for it.  Errors: QAP_ESTATE (tracking off),
 * QAP_EINVAL.
 * Device inputs of these calls must be complete when the call is made: the
 * handle's stream does not wait for the caller's streams. */
int qap_orbit_targets(qap_handle h, const int64_t *ids, int64_t count, double scale, float *t);

/* S-form restart from per-orbit outputs y (device, qap_orbit_count(n)*6
 * float32, orbit-id order): v_e = (y_e - mean) * scale in FP64, the mean a
 * left-to-right sum of the six outputs divided by 6; z costs 0 - v_e, x and
 * y costs of step 1, LB = 0, t = 0.  Errors: QAP_EINVAL, QAP_EDEVICE. */
int qap_warm_start_outputs(qap_handle h, const float *y, double scale);

/* The perceptron: 32 inputs, two hidden layers of 256 (ReLU), 6 outputs.
 * Parameters (float32, 75782): W1 [256][32], b1 [256], W2 [256][256],
 * b2 [256], W3 [6][256], b3 [6], back to back.  Forward:
 *   h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), y = W3 h2 + b3,
 * every matrix-product operand (inputs, weights, h1, h2) rounded to bf16,
 * float32 accumulation.  Loss: mean over samples and outputs of
 * (y - mean6(y) - t)^2.  Backward rounds its product operands to bf16 too
 * (output error, and the hidden errors after the ReLU masks); bias gradients
 * sum the unrounded errors.  Adam (Kingma and Ba) on float32 masters. */
typedef struct qap_mlp *qap_mlp_handle;

typedef struct qap_adam_params {
    double lr, beta1, beta2, eps;
} qap_adam_params;

typedef struct qap_warm_stats {
    long long orbits;
    double scale;      /* scale passed to the writer: qap_multiplier_scale * gain */
    double gain;
    double ms_mlp;     /* features + perceptron over all orbits (device time) */
    double ms_write;   /* z writer and restart (device time) */
    double seconds;    /* wall time of qap_warm_start */
    double mlp_flops;  /* 2 * orbits * (32*256 + 256*256 + 256*6) */
} qap_warm_stats;

/* params: host, 75782 floats; max_batch: largest training/forward batch;
 * stream: HIP stream for all of its work (NULL: the null stream).
 * Errors: QAP_EINVAL, QAP_ENOMEM, QAP_EDEVICE. */
int qap_mlp_create(const float *params, int max_batch, void *stream, qap_mlp_handle *out);
int qap_mlp_destroy(qap_mlp_handle p);
int qap_mlp_set_stream(qap_mlp_handle p, void *stream);
/* Host copy of the float32 master parameters. */
int qap_mlp_get_params(qap_mlp_handle p, float *params);
/* Forward of `count` <= max_batch samples: x device [count][32], y device
 * [count][6]; enqueued on the perceptron's stream. */
int qap_mlp_forward(qap_mlp_handle p, const float *x, int count, float *y);
/* Loss and gradients (host, 75782 floats, parameter order; nullable) of
 * `count` samples with targets t (device [count][6]); waits for the stream. */
int qap_mlp_gradients(qap_mlp_handle p, const float *x, const float *t, int count, float *grad,
                      double *loss);
/* One Adam step on `count` samples; *loss (nullable) gets the loss before the
 * step.  Errors: QAP_EINVAL (count, hyper-parameters), QAP_EDEVICE. */
int qap_mlp_train_step(qap_mlp_handle p, const float *x, const float *t, int count,
                       const qap_adam_params *opt, double *loss);

/* Features and perceptron over every orbit of the handle's instance (y:
 * device, qap_orbit_count(n)*6 float32, orbit-id order).  Runs on the
 * handle's stream after waiting for the perceptron's; waits for completion. */
int qap_orbit_outputs(qap_handle h, qap_mlp_handle p, float *y);

/* Learned warm start: qap_orbit_outputs into a temporary device buffer, then
 * qap_warm_start_outputs with scale = qap_multiplier_scale * gain.  The gain
 * (> 0) multiplies the predicted multipliers; any value keeps the bound
 * valid, and the trained weights come with one calibrated on the training
 * instances.  st nullable.
 * Errors: QAP_EINVAL (gain), QAP_ENOMEM (buffer of 24 bytes per orbit),
 * QAP_EDEVICE. */
int qap_warm_start(qap_handle h, qap_mlp_handle p, double gain, qap_warm_stats *st);

#ifdef __cplusplus
}
#endif
#endif /* QAP_RLT2_H */
