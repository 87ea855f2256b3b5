/*
 * rlt2_oracle.c -- plain, slow CPU oracle for the RLT2 Lagrangian dual ascent
 * (RLT2-DA) of Date & Nagi, "RLT2-based Parallel Algorithms for Solving Large
 * Quadratic Assignment Problems on GPU Clusters" (arXiv:1710.03732).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may load this code:
 * only the test suite, the package smoke check and the benchmark's CPU
 * baseline leg call it.  It shares no source with the GPU library.
 *
 * Everything is IEEE double, compiled with -ffp-contract=off and without
 * fast-math, so every expression below is evaluated exactly as written
 * (left to right, one rounding per operation).  Arrays are stored densely
 * (n^2, n^4, n^6) with the natural index order; invalid entries (repeated
 * facility or location indices) are never read or written.
 *
 * Parity: the LAP objective, bound and B&B optimum are pinned by brute force,
 * closed forms (Gilmore-Lawler bound, rearrangement) and invariants in the
 * test suite.  The trajectory LB_t for t >= 1 is a specified iteration whose
 * individual values the paper does not print: it is pinned only by the
 * invariants (reformulation identity, non-negative reduced costs, monotone
 * bound, bound <= optimum) -- "parity unpinned" for the exact values.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXM 128
#define ORC_MAXLAP 1024 /* largest LAP orc_lap takes (the LAP batch entry point goes to 1024) */
#define ORC_ROOT (-1)

#define IX2(n, i, p) ((size_t)(i) * (size_t)(n) + (size_t)(p))
#define IX4(n, i, j, p, q) \
    ((((size_t)(i) * (size_t)(n) + (size_t)(j)) * (size_t)(n) + (size_t)(p)) * (size_t)(n) + (size_t)(q))
#define IX6(n, i, j, k, p, q, r)                                                              \
    ((((((size_t)(i) * (size_t)(n) + (size_t)(j)) * (size_t)(n) + (size_t)(k)) * (size_t)(n) + \
       (size_t)(p)) * (size_t)(n) + (size_t)(q)) * (size_t)(n) + (size_t)(r))

void orc_set_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------
 * O1. Linear assignment problem by the Hungarian method (shortest augmenting
 * paths with row/column potentials).  The paper solves every Z-, Y- and X-LAP
 * with a primal-dual Hungarian algorithm (Section 2.3, "LAP Solution";
 * Section 3.2) and needs the optimal duals (xi/psi, gamma/delta, alpha/beta)
 * and the dual slacks pi = (M - u) - v of every LAP variable (complementary
 * slackness, Eq. compslack).  Which optimal duals are returned is not fixed
 * by the paper; this routine fixes it:
 *   - start (textbook column reduction): v[j] = min_i M[i][j], u = 0; every
 *     column proposes the lowest row attaining its minimum and each row
 *     proposed to is matched to the lowest proposing column; the running LAP
 *     value starts at the left fold of v[0..m-1];
 *   - the unmatched rows are then inserted in ascending order;
 *   - a Dijkstra step scans the newest tree row r: for every column j not yet
 *     in the tree, s = (M[r][j] - u[r]) - v[j], and minv[j] takes s when s is
 *     strictly smaller (remembering the column through which it was reached);
 *   - the next column j* is the non-tree column of least minv; ties prefer a
 *     column that is still unmatched, then the lowest index;
 *   - delta = minv[j*]; every tree row gets u += delta, every tree column
 *     v -= delta, every non-tree column minv -= delta; the LAP value gets
 *     += delta (the change of the dual objective sum(u) + sum(v));
 *   - on reaching an unmatched column the path is flipped back to the root.
 * Outputs: u[m], v[m], row_of_col[m], *theta; *steps counts Dijkstra steps.
 * ---------------------------------------------------------------------- */
int orc_lap(int m, const double *M, double *u, double *v, int *row_of_col,
            double *theta, long long *steps)
{
    double minv[ORC_MAXLAP];
    int used[ORC_MAXLAP], way[ORC_MAXLAP], prop[ORC_MAXLAP], owner[ORC_MAXLAP];
    if (m < 1 || m > ORC_MAXLAP) return -1;
    for (int i = 0; i < m; ++i) { u[i] = 0.0; owner[i] = -1; }
    for (int j = 0; j < m; ++j) {
        int arg = 0;
        double best = M[j];
        for (int i = 1; i < m; ++i)
            if (M[(size_t)i * m + j] < best) { best = M[(size_t)i * m + j]; arg = i; }
        v[j] = best;
        prop[j] = arg;
        row_of_col[j] = -1;
    }
    for (int j = 0; j < m; ++j)
        if (owner[prop[j]] < 0) { owner[prop[j]] = j; row_of_col[j] = prop[j]; }
    double th = v[0];
    for (int j = 1; j < m; ++j) th = th + v[j];
    long long st = 0;
    for (int i0 = 0; i0 < m; ++i0) {
        if (owner[i0] >= 0) continue;  /* matched by the column reduction */
        for (int j = 0; j < m; ++j) { minv[j] = HUGE_VAL; used[j] = 0; way[j] = ORC_ROOT; }
        int r = i0, last = ORC_ROOT;
        for (;;) {
            ++st;
            for (int j = 0; j < m; ++j) {
                if (used[j]) continue;
                double s = (M[(size_t)r * m + j] - u[r]) - v[j];
                if (s < minv[j]) { minv[j] = s; way[j] = last; }
            }
            int js = -1;
            for (int j = 0; j < m; ++j) {
                if (used[j]) continue;
                if (js < 0 || minv[j] < minv[js] ||
                    (minv[j] == minv[js] && row_of_col[j] < 0 && row_of_col[js] >= 0))
                    js = j;
            }
            double delta = minv[js];
            u[i0] = u[i0] + delta;
            for (int j = 0; j < m; ++j) {
                if (used[j]) {
                    u[row_of_col[j]] = u[row_of_col[j]] + delta;
                    v[j] = v[j] - delta;
                } else {
                    minv[j] = minv[j] - delta;
                }
            }
            th = th + delta;
            if (row_of_col[js] < 0) {
                /* flip the alternating path js <- way[js] <- ... <- root */
                int j = js;
                while (j != ORC_ROOT) {
                    int jp = way[j];
                    row_of_col[j] = (jp == ORC_ROOT) ? i0 : row_of_col[jp];
                    j = jp;
                }
                break;
            }
            used[js] = 1;
            r = row_of_col[js];
            last = js;
        }
    }
    *theta = th;
    if (steps) *steps += st;
    return 0;
}

/* ------------------------------------------------------------------------
 * QAP objective, Eq. (1.1): sum_ip b_ip x_ip + sum_ijpq f_ij d_pq x_ip x_jq,
 * for the permutation perm (perm[i] = location of facility i).  When every
 * input is integer-valued the sum is formed in int64 (exact).
 * ---------------------------------------------------------------------- */
static int all_integer(int n, const double *A)
{
    for (int t = 0; t < n * n; ++t) {
        double a = A[t];
        if (!(fabs(a) < 9.0e15) || a != floor(a)) return 0;
    }
    return 1;
}

int orc_is_integer_instance(int n, const double *F, const double *D, const double *B)
{
    return all_integer(n, F) && all_integer(n, D) && all_integer(n, B);
}

double orc_qap_cost(int n, const double *F, const double *D, const double *B, const int *perm)
{
    if (orc_is_integer_instance(n, F, D, B)) {
        int64_t c = 0;
        for (int i = 0; i < n; ++i) {
            c += (int64_t)B[IX2(n, i, perm[i])];
            for (int j = 0; j < n; ++j)
                c += (int64_t)F[IX2(n, i, j)] * (int64_t)D[IX2(n, perm[i], perm[j])];
        }
        return (double)c;
    }
    long double c = 0.0L;
    for (int i = 0; i < n; ++i) {
        c += (long double)B[IX2(n, i, perm[i])];
        for (int j = 0; j < n; ++j)
            c += (long double)F[IX2(n, i, j)] * (long double)D[IX2(n, perm[i], perm[j])];
    }
    return (double)c;
}

/* Brute force over all n! permutations (lexicographic order; the first
 * minimiser is reported).  n <= 11. */
static int next_perm(int n, int *a)
{
    int i = n - 2;
    while (i >= 0 && a[i] >= a[i + 1]) --i;
    if (i < 0) return 0;
    int j = n - 1;
    while (a[j] <= a[i]) --j;
    int t = a[i]; a[i] = a[j]; a[j] = t;
    for (int l = i + 1, r = n - 1; l < r; ++l, --r) { t = a[l]; a[l] = a[r]; a[r] = t; }
    return 1;
}

int orc_bruteforce(int n, const double *F, const double *D, const double *B,
                   int *best_perm, double *best_cost)
{
    if (n < 1 || n > 11) return -1;
    int a[16];
    for (int i = 0; i < n; ++i) a[i] = i;
    double best = HUGE_VAL;
    do {
        double c = orc_qap_cost(n, F, D, B, a);
        if (c < best) { best = c; memcpy(best_perm, a, sizeof(int) * n); }
    } while (next_perm(n, a));
    *best_cost = best;
    return 0;
}

/* ------------------------------------------------------------------------
 * Gilmore-Lawler bound.  With v = 0 the first RLT2-DA iteration yields the
 * Gilmore-Lawler bound (Section 5.1).  Its textbook definition: for every
 * (i, p), the least value of sum_{j != i} f_ij d_{p, s(j)} over bijections
 * s from {j != i} to {q != p} is the minimum scalar product of the two
 * vectors (rearrangement inequality: one sorted ascending, the other
 * descending); then one LAP over l_ip = b_ip + f_ii d_pp + that minimum.
 * ---------------------------------------------------------------------- */
static int cmp_dbl(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x < y) ? -1 : (x > y) ? 1 : 0;
}

int orc_glb(int n, const double *F, const double *D, const double *B, double *glb)
{
    if (n < 2 || n > ORC_MAXM) return -1;
    double *L = malloc(sizeof(double) * n * n);
    double fv[ORC_MAXM], dv[ORC_MAXM], u[ORC_MAXM], v[ORC_MAXM];
    int rc[ORC_MAXM];
    for (int i = 0; i < n; ++i)
        for (int p = 0; p < n; ++p) {
            int c = 0;
            for (int j = 0; j < n; ++j) if (j != i) fv[c++] = F[IX2(n, i, j)];
            c = 0;
            for (int q = 0; q < n; ++q) if (q != p) dv[c++] = D[IX2(n, p, q)];
            qsort(fv, n - 1, sizeof(double), cmp_dbl);
            qsort(dv, n - 1, sizeof(double), cmp_dbl);
            long double s = 0.0L;
            for (int t = 0; t < n - 1; ++t) s += (long double)fv[t] * (long double)dv[n - 2 - t];
            L[IX2(n, i, p)] = (double)((long double)B[IX2(n, i, p)] +
                                       (long double)F[IX2(n, i, i)] * (long double)D[IX2(n, p, p)] + s);
        }
    double th;
    orc_lap(n, L, u, v, rc, &th, NULL);
    long double s = 0.0L;
    for (int j = 0; j < n; ++j) s += (long double)L[IX2(n, rc[j], j)];
    *glb = (double)s;
    free(L);
    return 0;
}

/* ------------------------------------------------------------------------
 * O2. The F1 RLT2 dual ascent (Algorithm 1 in its "fast" form of Section 3.4,
 * one phase, no simulated annealing).
 *
 * State: LB and the three reduced-cost arrays R_x (n^2), R_y (n^4) and R_z
 * (n^6).  For every permutation sigma the reformulation identity
 *   cost(sigma) = LB + sum_i R_x[i,s_i] + sum_{i!=j} R_y[i,j,s_i,s_j]
 *                   + sum_{i,j,k distinct} R_z[i,j,k,s_i,s_j,s_k]
 * holds after every phase, and all R stay >= 0 (up to rounding).
 *
 * Initialisation (RLT1/RLT2 costs, Section 2.1): R_x[i,p] = b_ip + f_ii d_pp
 * (the diagonal products of Eq. 1.1 are linear in x), R_y[i,j,p,q] =
 * f_ij d_pq (C_ijpq), R_z = 0 (D_ijkpqr: the QAP has no cubic terms), LB = 0.
 *
 * Iteration t (Algorithm 1 steps 3-5):
 *   t >= 1: ascent sweep (Type 1, 2 and 3 rules, Eqs. da:rule1-3, combined as
 *           in the proof of Theorem 1, Eqs. ch4:proof:2-4, F-form of
 *           Section 3.4): for every z entry e with x parent P1(e) and y
 *           parent P1P2(e),
 *             g_e   = (kz*pi_z(e) + ky2*pi_y(P1P2(e))) + kx3*pi_x(P1(e)),
 *             new_e = okz*pi_z(e) + phi * (sum of g_f over the 5 partners f),
 *           with ky2 = ky/(n-2), kx3 = kx/((n-1)(n-2)), okz = 1-kz; then
 *           R_y <- oky*R_y and R_x <- okx*R_x (oky = 1-ky, okx = 1-kx).
 *   Z-LAPs: for every tile (i,j,p,q), i!=j, p!=q, the LAP on rows k (not i,j)
 *           and columns r (not p,q), both ascending; R_z <- pi_z and
 *           R_y[i,j,p,q] += theta (Algorithm 1 step 3e).
 *   t >= 1: y-pair rule (Eq. da:yrule1 applied by both members of each
 *           pair): a' = ophy*a + phy*b, b' = ophy*b + phy*a.
 *   Y-LAPs: for every (i,p) the LAP on rows j != i, columns q != p;
 *           R_y <- pi_y and R_x[i,p] += theta_y (step 4).
 *   X-LAP:  R_x <- pi_x, LB += theta_x (step 5); the X-LAP assignment is a
 *           QAP solution whose exact cost updates the upper bound UB.
 * ---------------------------------------------------------------------- */
typedef struct orc_da {
    int n;
    double kz, ky, kx, phi, phiy;
    double okz, oky, okx, ky2, kx3, ophiy;
    double *F, *D, *B;      /* original data, n^2 each (for exact UB) */
    double offset;          /* constant added to every permutation cost (fixed pairs of a B&B node) */
    int integer_data;
    double *X, *Y, *Z;
    double LB, UB;
    int t;
    int *xperm;             /* last X-LAP assignment */
    int *best_perm;         /* permutation achieving UB */
    long long lap_steps;
    double *trace;          /* LB after each iteration */
    int trace_len, trace_cap;
    double *Vt, *Ut;        /* tracked S-form multipliers v (n^6), u (n^4), or NULL */
    int half;               /* HALF scheme (orc_da_set_half) */
    int two_phase;          /* F2: pool and re-solve the Z-LAPs (orc_da_set_two_phase) */
    double min_gap;         /* gap stop of the running orc_da_run (no kick on a stopping iteration) */
    int sa_on;              /* Type 4 ascent with annealing (orc_da_set_annealing) */
    int sa_period;
    double sa_t0, sa_kmax, sa_cool;
    unsigned long long sa_seed;
    long long sa_accepted;  /* Type 4 steps taken */
    int slow;               /* S1: LAPs on the full costs each iteration (orc_da_set_slow) */
} orc_da;

static void orc_da_derive(orc_da *s)
{
    int n = s->n;
    double c2 = 1.0 / (double)(n - 2);
    double c3 = 1.0 / ((double)(n - 1) * (double)(n - 2));
    s->okz = 1.0 - s->kz;
    s->oky = 1.0 - s->ky;
    s->okx = 1.0 - s->kx;
    s->ky2 = s->ky * c2;
    s->kx3 = s->kx * c3;
    s->ophiy = 1.0 - s->phiy;
}

void orc_da_free(orc_da *s)
{
    if (!s) return;
    free(s->F); free(s->D); free(s->B);
    free(s->X); free(s->Y); free(s->Z);
    free(s->xperm); free(s->best_perm); free(s->trace);
    free(s->Vt); free(s->Ut);
    free(s);
}

/* Create the state from F, D, B (n x n row-major; B may be NULL = 0).
 * params = {kz, ky, kx, phi, phiy}; NULL selects the FULL preset
 * {5/6, 1, 1, 1/5, 1/2}. */
orc_da *orc_da_create(int n, const double *F, const double *D, const double *B,
                      const double *params)
{
    if (n < 3 || n > 64) return NULL;
    orc_da *s = calloc(1, sizeof(orc_da));
    if (!s) return NULL;
    s->n = n;
    if (params) {
        s->kz = params[0]; s->ky = params[1]; s->kx = params[2];
        s->phi = params[3]; s->phiy = params[4];
    } else {
        s->kz = 5.0 / 6.0; s->ky = 1.0; s->kx = 1.0; s->phi = 1.0 / 5.0; s->phiy = 0.5;
    }
    orc_da_derive(s);
    size_t n2 = (size_t)n * n, n4 = n2 * n2, n6 = n4 * n2;
    s->F = malloc(sizeof(double) * n2);
    s->D = malloc(sizeof(double) * n2);
    s->B = calloc(n2, sizeof(double));
    s->X = calloc(n2, sizeof(double));
    s->Y = calloc(n4, sizeof(double));
    s->Z = calloc(n6, sizeof(double));
    s->xperm = calloc(n, sizeof(int));
    s->best_perm = calloc(n, sizeof(int));
    s->trace_cap = 1024;
    s->trace = malloc(sizeof(double) * s->trace_cap);
    if (!s->F || !s->D || !s->B || !s->X || !s->Y || !s->Z || !s->xperm ||
        !s->best_perm || !s->trace) {
        orc_da_free(s);
        return NULL;
    }
    memcpy(s->F, F, sizeof(double) * n2);
    memcpy(s->D, D, sizeof(double) * n2);
    if (B) memcpy(s->B, B, sizeof(double) * n2);
    s->integer_data = orc_is_integer_instance(n, s->F, s->D, s->B);
    for (int i = 0; i < n; ++i)
        for (int p = 0; p < n; ++p)
            s->X[IX2(n, i, p)] = s->B[IX2(n, i, p)] + s->F[IX2(n, i, i)] * s->D[IX2(n, p, p)];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            for (int p = 0; p < n; ++p)
                for (int q = 0; q < n; ++q) {
                    if (q == p) continue;
                    s->Y[IX4(n, i, j, p, q)] = s->F[IX2(n, i, j)] * s->D[IX2(n, p, q)];
                }
        }
    s->LB = 0.0;
    s->UB = HUGE_VAL;
    s->t = 0;
    s->offset = 0.0;
    return s;
}

/* Build a state directly from given reduced-cost arrays (dense X n^2, Y n^4,
 * Z n^6) and LB; used by the branch-and-bound fold and by tests. */
orc_da *orc_da_from_arrays(int n, const double *F, const double *D, const double *B,
                           const double *params, double LB, const double *X,
                           const double *Y, const double *Z)
{
    orc_da *s = orc_da_create(n, F, D, B, params);
    if (!s) return NULL;
    size_t n2 = (size_t)n * n, n4 = n2 * n2, n6 = n4 * n2;
    memcpy(s->X, X, sizeof(double) * n2);
    memcpy(s->Y, Y, sizeof(double) * n4);
    memcpy(s->Z, Z, sizeof(double) * n6);
    s->LB = LB;
    return s;
}

/* Switch a fresh state to the HALF scheme (Section 5, after Goncalves
 * 2017).  In every orbit the three members whose first two facilities
 * ascend (the upper members) keep (1 - kz) of their z slack and take shares;
 * the three lower members give everything (kz = 1) and take nothing, so
 * their costs stay 0, their Z-LAPs (tiles with i > j) are all-zero LAPs of
 * value 0 and are not solved.  Shares: an upper giver's g goes half to each
 * other upper member (phi, 1/2); a lower giver's g a third to each of its
 * three upper partners.  Uses kz and phi from the params (2/3 and 1/2 in
 * the HALF preset).  Needs every lower z cost (first facility above the
 * second) to be 0, as on a fresh state, and no tracking; returns 0, or -1
 * when that does not hold.  A state without the z array (orc_da_create_xy)
 * may switch too: orc_iter1_tile then forms HALF tiles. */
int orc_da_set_half(orc_da *s)
{
    if (!s || s->Vt) return -1;
    int n = s->n;
    if (s->Z)
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < i; ++j)
            for (int k = 0; k < n; ++k)
                for (int p = 0; p < n; ++p)
                    for (int q = 0; q < n; ++q)
                        for (int r = 0; r < n; ++r)
                            if (s->Z[IX6(n, i, j, k, p, q, r)] != 0.0) return -1;
    s->half = 1;
    return 0;
}

/* The six members of the orbit {A=(i,p), B=(j,q), C=(k,r)} (i<j<k) in the
 * canonical order (A,B,C), (A,C,B), (B,A,C), (B,C,A), (C,A,B), (C,B,A); the
 * member (P1,P2,P3) is z_{P1.f P2.f P3.f P1.l P2.l P3.l}, the symmetric
 * variables of Eq. (rlt2:con3). */
static void orbit_members(int i, int j, int k, int p, int q, int r, int fac[6][3], int loc[6][3])
{
    int F3[3] = {i, j, k}, L3[3] = {p, q, r};
    static const int ord[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    for (int e = 0; e < 6; ++e)
        for (int c = 0; c < 3; ++c) {
            fac[e][c] = F3[ord[e][c]];
            loc[e][c] = L3[ord[e][c]];
        }
}

/* HALF scheme, lower giver: its g is split equally among its three upper
 * partners (the reading of Section 5's fractions that gives away exactly
 * the giver's g; 1/2 each would give away 3/2 of it). */
#define ORC_HALF_PHI_LOW (1.0 / 3.0)

void orc_da_sweep(orc_da *s)
{
    int n = s->n;
    double *X = s->X, *Y = s->Y, *Z = s->Z;
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j)
            for (int k = j + 1; k < n; ++k)
                for (int p = 0; p < n; ++p)
                    for (int q = 0; q < n; ++q) {
                        if (q == p) continue;
                        for (int r = 0; r < n; ++r) {
                            if (r == p || r == q) continue;
                            int fac[6][3], loc[6][3];
                            size_t zi[6];
                            double g[6], pz[6];
                            orbit_members(i, j, k, p, q, r, fac, loc);
                            if (s->half) {
                                /* upper members: the first two facilities ascend,
                                 * (A,B,C), (A,C,B), (B,C,A) = 0, 1, 3; lower: 2, 4, 5 */
                                static const int up[3] = {0, 1, 3};
                                for (int e = 0; e < 6; ++e) {
                                    const int upper = fac[e][0] < fac[e][1];
                                    zi[e] = IX6(n, fac[e][0], fac[e][1], fac[e][2], loc[e][0], loc[e][1], loc[e][2]);
                                    pz[e] = Z[zi[e]];
                                    double py = Y[IX4(n, fac[e][0], fac[e][1], loc[e][0], loc[e][1])];
                                    double px = X[IX2(n, fac[e][0], loc[e][0])];
                                    g[e] = ((upper ? s->kz : 1.0) * pz[e] + s->ky2 * py) + s->kx3 * px;
                                }
                                double acc_low = (g[2] + g[4]) + g[5];
                                for (int a = 0; a < 3; ++a) {
                                    int e = up[a];
                                    int f1 = up[a == 0 ? 1 : 0], f2 = up[a == 2 ? 1 : 2];
                                    double acc_up = g[f1] + g[f2];
                                    Z[zi[e]] = s->okz * pz[e] + (s->phi * acc_up + ORC_HALF_PHI_LOW * acc_low);
                                }
                                Z[zi[2]] = 0.0;
                                Z[zi[4]] = 0.0;
                                Z[zi[5]] = 0.0;
                                continue;
                            }
                            for (int e = 0; e < 6; ++e) {
                                zi[e] = IX6(n, fac[e][0], fac[e][1], fac[e][2], loc[e][0], loc[e][1], loc[e][2]);
                                pz[e] = Z[zi[e]];
                                double py = Y[IX4(n, fac[e][0], fac[e][1], loc[e][0], loc[e][1])];
                                double px = X[IX2(n, fac[e][0], loc[e][0])];
                                g[e] = (s->kz * pz[e] + s->ky2 * py) + s->kx3 * px;
                            }
                            for (int e = 0; e < 6; ++e) {
                                double acc = 0.0;
                                int first = 1;
                                for (int f = 0; f < 6; ++f) {
                                    if (f == e) continue;
                                    if (first) { acc = g[f]; first = 0; }
                                    else acc = acc + g[f];
                                }
                                Z[zi[e]] = s->okz * pz[e] + s->phi * acc;
                                if (s->Vt) s->Vt[zi[e]] = s->Vt[zi[e]] + (g[e] - s->phi * acc);
                            }
                        }
                    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            for (int p = 0; p < n; ++p)
                for (int q = 0; q < n; ++q) {
                    if (q == p) continue;
                    size_t y = IX4(n, i, j, p, q);
                    Y[y] = s->oky * Y[y];
                }
        }
    for (size_t a = 0; a < (size_t)n * n; ++a) X[a] = s->okx * X[a];
}

void orc_da_zphase(orc_da *s)
{
    int n = s->n, m = n - 2;
    double *Y = s->Y, *Z = s->Z;
    long long steps = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : steps)
    for (int i = 0; i < n; ++i) {
        double M[ORC_MAXM * 8], u[ORC_MAXM], v[ORC_MAXM], th;
        double *Mb = (m * m <= ORC_MAXM * 8) ? M : malloc(sizeof(double) * m * m);
        int rc[ORC_MAXM], ks[ORC_MAXM], rs[ORC_MAXM];
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            if (s->half && j < i) continue;  /* HALF: lower tiles stay all-zero (theta 0) */
            int c = 0;
            for (int k = 0; k < n; ++k) if (k != i && k != j) ks[c++] = k;
            for (int p = 0; p < n; ++p)
                for (int q = 0; q < n; ++q) {
                    if (q == p) continue;
                    c = 0;
                    for (int r = 0; r < n; ++r) if (r != p && r != q) rs[c++] = r;
                    for (int a = 0; a < m; ++a)
                        for (int b = 0; b < m; ++b)
                            Mb[a * m + b] = Z[IX6(n, i, j, ks[a], p, q, rs[b])];
                    orc_lap(m, Mb, u, v, rc, &th, &steps);
                    for (int a = 0; a < m; ++a)
                        for (int b = 0; b < m; ++b)
                            Z[IX6(n, i, j, ks[a], p, q, rs[b])] = (Mb[a * m + b] - u[a]) - v[b];
                    size_t y = IX4(n, i, j, p, q);
                    Y[y] = Y[y] + th;
                }
        }
        if (Mb != M) free(Mb);
    }
    s->lap_steps += steps;
}

void orc_da_yequal(orc_da *s)
{
    int n = s->n;
    double *Y = s->Y;
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j)
            for (int p = 0; p < n; ++p)
                for (int q = 0; q < n; ++q) {
                    if (q == p) continue;
                    size_t a = IX4(n, i, j, p, q), b = IX4(n, j, i, q, p);
                    double ya = Y[a], yb = Y[b];
                    Y[a] = s->ophiy * ya + s->phiy * yb;
                    Y[b] = s->ophiy * yb + s->phiy * ya;
                    if (s->Ut) {
                        s->Ut[a] = s->Ut[a] + s->phiy * (ya - yb);
                        s->Ut[b] = s->Ut[b] + s->phiy * (yb - ya);
                    }
                }
}

void orc_da_yphase(orc_da *s)
{
    int n = s->n, m = n - 1;
    double *X = s->X, *Y = s->Y;
    long long steps = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : steps)
    for (int i = 0; i < n; ++i) {
        double *M = malloc(sizeof(double) * m * m);
        double u[ORC_MAXM], v[ORC_MAXM], th;
        int rc[ORC_MAXM], js[ORC_MAXM], qs[ORC_MAXM];
        int c = 0;
        for (int j = 0; j < n; ++j) if (j != i) js[c++] = j;
        for (int p = 0; p < n; ++p) {
            c = 0;
            for (int q = 0; q < n; ++q) if (q != p) qs[c++] = q;
            for (int a = 0; a < m; ++a)
                for (int b = 0; b < m; ++b)
                    M[a * m + b] = Y[IX4(n, i, js[a], p, qs[b])];
            orc_lap(m, M, u, v, rc, &th, &steps);
            for (int a = 0; a < m; ++a)
                for (int b = 0; b < m; ++b)
                    Y[IX4(n, i, js[a], p, qs[b])] = (M[a * m + b] - u[a]) - v[b];
            X[IX2(n, i, p)] = X[IX2(n, i, p)] + th;
        }
        free(M);
    }
    s->lap_steps += steps;
}

static void orc_record_ub(orc_da *s, const int *perm_full, double cost)
{
    if (cost < s->UB) {
        s->UB = cost;
        memcpy(s->best_perm, perm_full, sizeof(int) * s->n);
    }
}

void orc_da_xphase(orc_da *s)
{
    int n = s->n;
    double *M = malloc(sizeof(double) * n * n);
    double u[ORC_MAXM], v[ORC_MAXM], th;
    int rc[ORC_MAXM];
    memcpy(M, s->X, sizeof(double) * n * n);
    orc_lap(n, M, u, v, rc, &th, &s->lap_steps);
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b)
            s->X[IX2(n, a, b)] = (M[IX2(n, a, b)] - u[a]) - v[b];
    s->LB = s->LB + th;
    for (int j = 0; j < n; ++j) s->xperm[rc[j]] = j;
    orc_record_ub(s, s->xperm, orc_qap_cost(n, s->F, s->D, s->B, s->xperm) + s->offset);
    free(M);
}

/* ------------------------------------------------------------------------
 * Type 4 ascent with simulated annealing (Section 2.3, last ascent rule;
 * schedule of Section 5).
 *
 * Random numbers: SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) used as a
 * counter-based generator: the c-th output (c >= 1) of the stream seeded
 * with `seed` mixes seed + c * 0x9e3779b97f4a7c15 with the published
 * finaliser; a uniform double in [0, 1) is its top 53 bits times 2^-53.
 * ---------------------------------------------------------------------- */
unsigned long long orc_splitmix64(unsigned long long seed, unsigned long long c)
{
    unsigned long long z = seed + c * 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

double orc_sa_uniform(unsigned long long seed, unsigned long long c)
{
    return (double)(orc_splitmix64(seed, c) >> 11) * (1.0 / 9007199254740992.0);
}

/* exp(x) for x <= 0, written out so that every platform computes the same
 * bits: x = k ln2 + r with k = floor(x log2(e) + 1/2) and |r| <= ln2 / 2
 * (ln2 split in a high part with trailing zero bits, so k * high is exact),
 * then the Taylor polynomial of degree 13 in Horner form (truncation below
 * 1e-17 relative) scaled by 2^k.  Returns 0 below -745. */
double orc_sa_exp(double x)
{
    const double ln2_hi = 6.93147180369123816490e-01;  /* ln 2 to 32 bits */
    const double ln2_lo = 1.90821492927058770002e-10;  /* ln 2 - ln2_hi */
    const double log2e = 1.44269504088896338700e+00;
    if (x < -745.0) return 0.0;
    double k = floor(x * log2e + 0.5);
    double r = (x - k * ln2_hi) - k * ln2_lo;
    double p = 1.0 / 6227020800.0;                    /* 1/13! */
    p = p * r + 1.0 / 479001600.0;
    p = p * r + 1.0 / 39916800.0;
    p = p * r + 1.0 / 3628800.0;
    p = p * r + 1.0 / 362880.0;
    p = p * r + 1.0 / 40320.0;
    p = p * r + 1.0 / 5040.0;
    p = p * r + 1.0 / 720.0;
    p = p * r + 1.0 / 120.0;
    p = p * r + 1.0 / 24.0;
    p = p * r + 1.0 / 6.0;
    p = p * r + 0.5;
    p = p * r + 1.0;
    p = p * r + 1.0;
    return ldexp(p, (int)k);
}

/* Enable annealing: temperature t0 (cost units; Section 5 starts at 4 % of
 * the best known UB) multiplied by `cool` every `period` iterations, at most
 * kappa_max of the bound offered per step, SplitMix64 seed.  t0 <= 0 turns
 * it off.  Not with tracking (the step moves bound into the x costs, which
 * the tracked multipliers do not follow).  0 or -1. */
int orc_da_set_annealing(orc_da *s, double t0, double kappa_max, double cool, int period,
                         unsigned long long seed)
{
    if (!s || s->Vt || s->slow) return -1;
    if (!(t0 > 0.0)) { s->sa_on = 0; return 0; }
    if (!(kappa_max >= 0.0 && kappa_max <= 1.0) || !(cool > 0.0 && cool <= 1.0) || period < 1) return -1;
    s->sa_on = 1;
    s->sa_t0 = t0;
    s->sa_kmax = kappa_max;
    s->sa_cool = cool;
    s->sa_period = period;
    s->sa_seed = seed;
    return 0;
}

/* One Type 4 step after the X-LAP of iteration it (bound nu = LB).  Draws
 * for this iteration, counters it*(2n+2) + 1 ... + 2n+2: u_s (size), u_a
 * (acceptance), w_1..w_2n (one per facility, then one per location).
 * kappa^lb = kappa_max * u_s is split over the 2n fractions in proportion to
 * the w (kappa_k = (kappa^lb * w_k) / W, W the left fold of the w); facility
 * i offers a_i = kappa_i * nu, location p offers a_p = kappa_p * nu, and the
 * offer A is the left fold of all 2n.  With temperature
 * T = t0 * cool^floor(it / period) (repeated products) the step is taken
 * when u_a <= exp(-A / T): every x slack of row i and column p grows,
 * pi_x[i][p] = (pi_x[i][p] + a_i) + a_p, and LB drops by A.  A permutation
 * meets each row and each column once, so cost = LB + reduced costs still
 * holds and all slacks stay >= 0: the bound stays valid.  No step when
 * nu <= 0.  Returns 1 when the step was taken. */
int orc_da_type4(orc_da *s, int it)
{
    int n = s->n;
    double nu = s->LB;
    if (!(nu > 0.0)) return 0;
    unsigned long long base = (unsigned long long)it * (unsigned long long)(2 * n + 2);
    double us = orc_sa_uniform(s->sa_seed, base + 1);
    double ua = orc_sa_uniform(s->sa_seed, base + 2);
    double w[2 * ORC_MAXM + 4], a[2 * ORC_MAXM + 4];
    double W = 0.0;
    for (int k = 0; k < 2 * n; ++k) {
        w[k] = orc_sa_uniform(s->sa_seed, base + 3 + (unsigned long long)k);
        W = (k == 0) ? w[k] : W + w[k];
    }
    if (!(W > 0.0)) return 0;
    double klb = s->sa_kmax * us;
    double A = 0.0;
    for (int k = 0; k < 2 * n; ++k) {
        a[k] = ((klb * w[k]) / W) * nu;
        A = (k == 0) ? a[k] : A + a[k];
    }
    double T = s->sa_t0;
    for (int c = 0; c < it / s->sa_period; ++c) T = T * s->sa_cool;
    if (!(ua <= orc_sa_exp(-(A / T)))) return 0;
    for (int i = 0; i < n; ++i)
        for (int p = 0; p < n; ++p) s->X[IX2(n, i, p)] = (s->X[IX2(n, i, p)] + a[i]) + a[n + p];
    s->LB = nu - A;
    s->sa_accepted += 1;
    return 1;
}

static void orc_trace_push(orc_da *s, double lb)
{
    if (s->trace_len == s->trace_cap) {
        s->trace_cap *= 2;
        s->trace = realloc(s->trace, sizeof(double) * s->trace_cap);
    }
    s->trace[s->trace_len++] = lb;
}

int orc_da_proven(const orc_da *s);

/* Two-phase variant F2 (Section 3.4): after the Z-LAPs, in every orbit
 * {(i,p),(j,q),(k,r)} with i < j < k and distinct p, q, r the six members
 * are split by their dual slack into S_B (slack 0) and S_N (slack > 0).
 * The S_N members' costs drop by their slack (to 0) and the slack total
 * (left fold in the canonical member order) is shared equally among the S_B
 * members; orbits with S_B or S_N empty are unchanged.  In the F-form the
 * arrays hold the slacks themselves, so "slack 0" reads as <= 0 (a slack
 * that rounding left negative belongs to S_B).  The transfer is zero-sum
 * per orbit (a multiplier move on the symmetry constraints), so the bound
 * stays valid. */
void orc_da_pool(orc_da *s)
{
    int n = s->n;
    double *Z = s->Z;
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j)
            for (int k = j + 1; k < n; ++k)
                for (int p = 0; p < n; ++p)
                    for (int q = 0; q < n; ++q) {
                        if (q == p) continue;
                        for (int r = 0; r < n; ++r) {
                            if (r == p || r == q) continue;
                            int fac[6][3], loc[6][3];
                            size_t zi[6];
                            double pi[6];
                            orbit_members(i, j, k, p, q, r, fac, loc);
                            double slack = 0.0;
                            int first = 1, nbasic = 0;
                            for (int e = 0; e < 6; ++e) {
                                zi[e] = IX6(n, fac[e][0], fac[e][1], fac[e][2], loc[e][0], loc[e][1], loc[e][2]);
                                pi[e] = Z[zi[e]];
                                if (pi[e] > 0.0) {
                                    if (first) { slack = pi[e]; first = 0; }
                                    else slack = slack + pi[e];
                                } else {
                                    ++nbasic;
                                }
                            }
                            if (nbasic == 0 || nbasic == 6) continue;
                            double share = slack / (double)nbasic;
                            for (int e = 0; e < 6; ++e) {
                                double nv = pi[e] > 0.0 ? 0.0 : pi[e] + share;
                                Z[zi[e]] = nv;
                                /* S2: the cost change is a multiplier move, v += old - new */
                                if (s->slow) s->Vt[zi[e]] = s->Vt[zi[e]] + (pi[e] - nv);
                            }
                        }
                    }
}

/* Switch a state to the two-phase variant (F2, or S2 with the slow
 * variant, whose tracked multipliers the pooling then moves too).  Not with
 * HALF, nor with tracking outside S1; 0 or -1. */
int orc_da_set_two_phase(orc_da *s)
{
    if (!s || s->half || (s->Vt && !s->slow)) return -1;
    s->two_phase = 1;
    return 0;
}

/* Slow variant S1 (Section 3.4): the LAPs of every iteration are solved on
 * the full costs b', C', D' - v (the left-hand side of Eq. ch4:proof:4)
 * rather than on the slacks.  The z multipliers follow F1's rule (tracked:
 * v moves by the sweep's g_e - phi * sum, Eq. ch4:proof:2, from the slacks
 * of the last full solve), and after the sweep the state is rebuilt from
 * them: x costs b + f_ii d_pp, y costs f_ij d_pq, z costs -v (D = 0),
 * LB = 0, so the X-LAP value is the whole bound nu(LRLT2(v)).  The y
 * multipliers stay 0 (the y-pair rule is not applied): that is the setting
 * of Theorem 1, under which these bounds never fall. */
static void orc_da_rebuild(orc_da *s)
{
    int n = s->n;
    size_t n2 = (size_t)n * n, n4 = n2 * n2;
    for (size_t e = 0; e < n4 * n2; ++e) s->Z[e] = -s->Vt[e];
    for (int i = 0; i < n; ++i)
        for (int p = 0; p < n; ++p)
            s->X[IX2(n, i, p)] = s->B[IX2(n, i, p)] + s->F[IX2(n, i, i)] * s->D[IX2(n, p, p)];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            for (int p = 0; p < n; ++p)
                for (int q = 0; q < n; ++q) {
                    if (q == p) continue;
                    s->Y[IX4(n, i, j, p, q)] = s->F[IX2(n, i, j)] * s->D[IX2(n, p, q)];
                }
        }
    s->LB = 0.0;
}

/* Switch a fresh state (t = 0) to S1 (S2 with the two-phase flag): turns
 * tracking on (the multipliers are its state).  Not with HALF or
 * annealing.  0 or -1. */
int orc_da_track(orc_da *s);
int orc_da_set_slow(orc_da *s)
{
    if (!s || s->t != 0 || s->half || s->sa_on) return -1;
    s->slow = 1;
    if (orc_da_track(s) != 0) { s->slow = 0; return -1; }
    return 0;
}

void orc_da_iterate(orc_da *s)
{
    if (s->t >= 1) orc_da_sweep(s);
    if (s->t >= 1 && s->slow) orc_da_rebuild(s);
    orc_da_zphase(s);
    if (s->two_phase && s->t >= 1) {
        /* F2: pool within the orbits, then re-solve the Z-LAPs on the pooled
         * slacks (their values add to Theta, as in the first solve) */
        orc_da_pool(s);
        orc_da_zphase(s);
    }
    if (s->t >= 1 && !s->slow) orc_da_yequal(s);  /* S1 keeps u = 0 */
    orc_da_yphase(s);
    orc_da_xphase(s);
    orc_trace_push(s, s->LB);
    s->t += 1;
    /* Type 4 after every iteration t >= 1 unless this one stops the run */
    if (s->sa_on && s->t >= 2 && !orc_da_proven(s) &&
        !(s->min_gap > 0.0 && s->UB < HUGE_VAL && s->UB != 0.0 && (s->UB - s->LB) / fabs(s->UB) < s->min_gap))
        orc_da_type4(s, s->t - 1);
}

/* Optimality certificate (feasibility check, Section 2.3): the X-LAP
 * permutation's exact cost meets the bound. */
int orc_da_proven(const orc_da *s)
{
    if (!(s->UB < HUGE_VAL)) return 0;
    double tol = 1e-9 * fmax(1.0, fabs(s->UB));
    if (s->integer_data) return ceil(s->LB - tol) >= s->UB;
    return s->UB - s->LB <= tol;
}

/* Run up to iters more iterations (Algorithm 1 step 2): stop early when the
 * bound is proven optimal or GAP = (UB - LB) / UB drops below min_gap.
 * Returns the number of iterations run. */
int orc_da_run(orc_da *s, int iters, double min_gap)
{
    int done = 0;
    s->min_gap = min_gap;
    for (int it = 0; it < iters; ++it) {
        if (s->t > 0) {
            if (orc_da_proven(s)) break;
            if (min_gap > 0.0 && s->UB < HUGE_VAL && s->UB != 0.0 &&
                (s->UB - s->LB) / fabs(s->UB) < min_gap) break;
        }
        orc_da_iterate(s);
        ++done;
    }
    return done;
}

/* Accessors used by the ctypes wrapper. */
int orc_da_n(const orc_da *s) { return s->n; }
int orc_da_t(const orc_da *s) { return s->t; }
double orc_da_lb(const orc_da *s) { return s->LB; }
long long orc_da_sa_accepted(const orc_da *s) { return s->sa_accepted; }
double orc_da_ub(const orc_da *s) { return s->UB; }
long long orc_da_steps(const orc_da *s) { return s->lap_steps; }
int orc_da_trace(const orc_da *s, double *out, int cap)
{
    int k = s->trace_len < cap ? s->trace_len : cap;
    memcpy(out, s->trace, sizeof(double) * k);
    return s->trace_len;
}
void orc_da_perms(const orc_da *s, int *xperm, int *best)
{
    if (xperm) memcpy(xperm, s->xperm, sizeof(int) * s->n);
    if (best) memcpy(best, s->best_perm, sizeof(int) * s->n);
}
void orc_da_export(const orc_da *s, double *X, double *Y, double *Z)
{
    size_t n2 = (size_t)s->n * s->n, n4 = n2 * n2;
    if (X) memcpy(X, s->X, sizeof(double) * n2);
    if (Y) memcpy(Y, s->Y, sizeof(double) * n4);
    if (Z) memcpy(Z, s->Z, sizeof(double) * n4 * n2);
}

/* The z reduced costs of selected tiles, without the dense n^6 copy: for
 * tile a, given as facilities (i, j) and locations (p, q) in ijpq[4a..4a+3],
 * out[a*m*m + k''*m + r''] = R_z[i,j,k,p,q,r] with k and r running over the
 * remaining facilities and locations in ascending order (m = n - 2).
 * Returns 0, or -1 for an index out of range or repeated within a pair. */
int orc_da_z_tiles(const orc_da *s, int count, const int *ijpq, double *out)
{
    int n = s->n, m = n - 2;
    for (int a = 0; a < count; ++a) {
        int i = ijpq[4 * a], j = ijpq[4 * a + 1], p = ijpq[4 * a + 2], q = ijpq[4 * a + 3];
        if (i < 0 || j < 0 || p < 0 || q < 0 || i >= n || j >= n || p >= n || q >= n || i == j || p == q)
            return -1;
        int ks[ORC_MAXM], rs[ORC_MAXM], c = 0;
        for (int k = 0; k < n; ++k) if (k != i && k != j) ks[c++] = k;
        c = 0;
        for (int r = 0; r < n; ++r) if (r != p && r != q) rs[c++] = r;
        for (int x = 0; x < m; ++x)
            for (int y = 0; y < m; ++y)
                out[(size_t)a * m * m + (size_t)x * m + y] = s->Z[IX6(n, i, j, ks[x], p, q, rs[y])];
    }
    return 0;
}

/* Multiplier tracking.  The F1 transfers are Lagrange multiplier updates in
 * the sense of the ascent rules: per sweep, entry e's multiplier moves by
 * g_e - phi * sum_{f != e} g_f (Eq. ch4:proof:2: its own kappa-shares minus
 * Omega_e), per y-pair rule u_ijpq moves by phy * (a - b) (Eq. da:yrule1).
 * Both are zero-sum over an orbit / a pair.  Tracking starts at zero. */
int orc_da_track(orc_da *s)
{
    if (s->half || (s->two_phase && !s->slow) || s->sa_on) return -1;  /* tracking follows the FULL transfers */
    size_t n2 = (size_t)s->n * s->n, n4 = n2 * n2;
    if (!s->Vt) s->Vt = calloc(n4 * n2, sizeof(double));
    if (!s->Ut) s->Ut = calloc(n4, sizeof(double));
    return (s->Vt && s->Ut) ? 0 : -1;
}

void orc_da_multipliers(const orc_da *s, double *V, double *U)
{
    size_t n2 = (size_t)s->n * s->n, n4 = n2 * n2;
    if (V && s->Vt) memcpy(V, s->Vt, sizeof(double) * n4 * n2);
    if (U && s->Ut) memcpy(U, s->Ut, sizeof(double) * n4);
}

/* Lagrangian relaxation LRLT2(u, v) in its initial form (Algorithm 1 step 1
 * with given multipliers): x costs b + f_ii d_pp, y costs C - u, z costs
 * D - v = -v, LB = 0; any zero-sum u, v keep every bound valid (Eq.
 * lgduality). */
orc_da *orc_da_from_multipliers(int n, const double *F, const double *D, const double *B,
                                const double *params, const double *V, const double *U)
{
    orc_da *s = orc_da_create(n, F, D, B, params);
    if (!s) return NULL;
    size_t n2 = (size_t)n * n, n4 = n2 * n2;
    if (U)
        for (size_t a = 0; a < n4; ++a) s->Y[a] = s->Y[a] - U[a];
    if (V)
        for (size_t a = 0; a < n4 * n2; ++a) s->Z[a] = 0.0 - V[a];
    return s;
}

/* O3. Reformulation identity: LB plus the reduced costs picked by perm. */
double orc_da_identity(const orc_da *s, const int *perm)
{
    int n = s->n;
    long double acc = (long double)s->LB;
    for (int i = 0; i < n; ++i) acc += (long double)s->X[IX2(n, i, perm[i])];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            acc += (long double)s->Y[IX4(n, i, j, perm[i], perm[j])];
        }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            for (int k = 0; k < n; ++k) {
                if (k == i || k == j) continue;
                acc += (long double)s->Z[IX6(n, i, j, k, perm[i], perm[j], perm[k])];
            }
        }
    return (double)acc;
}

/* Most negative valid entry of each level (non-negativity check). */
void orc_da_min_entries(const orc_da *s, double *out3)
{
    int n = s->n;
    double mx = HUGE_VAL, my = HUGE_VAL, mz = HUGE_VAL;
    for (size_t a = 0; a < (size_t)n * n; ++a) if (s->X[a] < mx) mx = s->X[a];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            for (int p = 0; p < n; ++p)
                for (int q = 0; q < n; ++q) {
                    if (q == p) continue;
                    double y = s->Y[IX4(n, i, j, p, q)];
                    if (y < my) my = y;
                    for (int k = 0; k < n; ++k) {
                        if (k == i || k == j) continue;
                        for (int r = 0; r < n; ++r) {
                            if (r == p || r == q) continue;
                            double z = s->Z[IX6(n, i, j, k, p, q, r)];
                            if (z < mz) mz = z;
                        }
                    }
                }
        }
    out3[0] = mx; out3[1] = my; out3[2] = mz;
}

/* ------------------------------------------------------------------------
 * Sampled evaluation for sizes whose n^6 array does not fit a test (n = 30,
 * 42).  At t = 0 the z level is identically zero, so every Z-LAP has value 0
 * and zero duals and iteration 0 is exactly the Y-LAPs on f_ij d_pq followed
 * by the X-LAP; orc_da_create_xy builds a state without the z array and
 * orc_da_iter0_xy runs that iteration.  orc_iter1_tile then forms one tile of
 * the iteration-1 Z-LAPs entry by entry from the sweep formula (pi_z = 0 at
 * t = 0, so g_f = (kz*0 + ky2*pi_y) + kx3*pi_x, new_e = okz*0 + phi*sum) and
 * solves it.  Under HALF only upper tiles (i < j) are formed, with the HALF
 * shares of orc_da_sweep (a lower member's g has factor 1 on its zero z).
 * Iteration 0 is the same under both schemes: every Z-LAP is all-zero.
 * ---------------------------------------------------------------------- */
orc_da *orc_da_create_xy(int n, const double *F, const double *D, const double *B,
                         const double *params)
{
    if (n < 3 || n > 64) return NULL;
    orc_da *s = calloc(1, sizeof(orc_da));
    if (!s) return NULL;
    s->n = n;
    if (params) {
        s->kz = params[0]; s->ky = params[1]; s->kx = params[2];
        s->phi = params[3]; s->phiy = params[4];
    } else {
        s->kz = 5.0 / 6.0; s->ky = 1.0; s->kx = 1.0; s->phi = 1.0 / 5.0; s->phiy = 0.5;
    }
    orc_da_derive(s);
    size_t n2 = (size_t)n * n, n4 = n2 * n2;
    s->F = malloc(sizeof(double) * n2);
    s->D = malloc(sizeof(double) * n2);
    s->B = calloc(n2, sizeof(double));
    s->X = calloc(n2, sizeof(double));
    s->Y = calloc(n4, sizeof(double));
    s->Z = NULL;
    s->xperm = calloc(n, sizeof(int));
    s->best_perm = calloc(n, sizeof(int));
    s->trace_cap = 16;
    s->trace = malloc(sizeof(double) * s->trace_cap);
    memcpy(s->F, F, sizeof(double) * n2);
    memcpy(s->D, D, sizeof(double) * n2);
    if (B) memcpy(s->B, B, sizeof(double) * n2);
    s->integer_data = orc_is_integer_instance(n, s->F, s->D, s->B);
    for (int i = 0; i < n; ++i)
        for (int p = 0; p < n; ++p)
            s->X[IX2(n, i, p)] = s->B[IX2(n, i, p)] + s->F[IX2(n, i, i)] * s->D[IX2(n, p, p)];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            for (int p = 0; p < n; ++p)
                for (int q = 0; q < n; ++q) {
                    if (q == p) continue;
                    s->Y[IX4(n, i, j, p, q)] = s->F[IX2(n, i, j)] * s->D[IX2(n, p, q)];
                }
        }
    s->LB = 0.0;
    s->UB = HUGE_VAL;
    return s;
}

int orc_da_iter0_xy(orc_da *s)
{
    if (s->t != 0 || s->Z != NULL) return -1;
    /* Z-phase on all-zero tiles: theta = 0, so R_y = R_y + 0.0 */
    int n = s->n;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            for (int p = 0; p < n; ++p)
                for (int q = 0; q < n; ++q) {
                    if (q == p) continue;
                    size_t y = IX4(n, i, j, p, q);
                    s->Y[y] = s->Y[y] + 0.0;
                }
        }
    orc_da_yphase(s);
    orc_da_xphase(s);
    orc_trace_push(s, s->LB);
    s->t = 1;
    return 0;
}

/* Tile (i,j,p,q) of the iteration-1 Z-LAPs, from a state after iteration 0
 * (X = pi_x, Y = pi_y).  Outputs the tile M (m*m, rows k, columns r
 * ascending), its LAP slacks pi (m*m) and value theta. */
int orc_iter1_tile(const orc_da *s, int i, int j, int p, int q, double *M_out, double *pi_out,
                   double *theta_out)
{
    int n = s->n, m = n - 2;
    if (s->t != 1 || i == j || p == q || m < 1 || m > ORC_MAXM) return -1;
    if (s->half && i > j) return -1;  /* lower tiles stay all-zero */
    double *M = malloc(sizeof(double) * m * m);
    int a = 0;
    for (int k = 0; k < n; ++k) {
        if (k == i || k == j) continue;
        int b = 0;
        for (int r = 0; r < n; ++r) {
            if (r == p || r == q) continue;
            /* the orbit of (i,p),(j,q),(k,r), sorted by facility */
            int f[3] = {i, j, k}, l[3] = {p, q, r};
            for (int x = 0; x < 3; ++x)
                for (int y = x + 1; y < 3; ++y)
                    if (f[y] < f[x]) {
                        int tf = f[x]; f[x] = f[y]; f[y] = tf;
                        int tl = l[x]; l[x] = l[y]; l[y] = tl;
                    }
            int fac[6][3], loc[6][3];
            orbit_members(f[0], f[1], f[2], l[0], l[1], l[2], fac, loc);
            double g[6];
            int me = -1;
            for (int e = 0; e < 6; ++e) {
                double pz = 0.0;
                double py = s->Y[IX4(n, fac[e][0], fac[e][1], loc[e][0], loc[e][1])];
                double px = s->X[IX2(n, fac[e][0], loc[e][0])];
                const double kze = (s->half && fac[e][0] > fac[e][1]) ? 1.0 : s->kz;
                g[e] = (kze * pz + s->ky2 * py) + s->kx3 * px;
                if (fac[e][0] == i && fac[e][1] == j && fac[e][2] == k &&
                    loc[e][0] == p && loc[e][1] == q && loc[e][2] == r) me = e;
            }
            if (s->half) {
                /* me is an upper member (i < j): 0, 1 or 3 */
                double acc_up = 0.0;
                int first = 1;
                for (int e = 0; e < 6; ++e) {
                    if (e == me || e == 2 || e == 4 || e == 5) continue;
                    if (first) { acc_up = g[e]; first = 0; }
                    else acc_up = acc_up + g[e];
                }
                double acc_low = (g[2] + g[4]) + g[5];
                M[a * m + b] = s->okz * 0.0 + (s->phi * acc_up + ORC_HALF_PHI_LOW * acc_low);
                ++b;
                continue;
            }
            double acc = 0.0;
            int first = 1;
            for (int e = 0; e < 6; ++e) {
                if (e == me) continue;
                if (first) { acc = g[e]; first = 0; }
                else acc = acc + g[e];
            }
            M[a * m + b] = s->okz * 0.0 + s->phi * acc;
            ++b;
        }
        ++a;
    }
    double u[ORC_MAXM], v[ORC_MAXM], th;
    int rc[ORC_MAXM];
    orc_lap(m, M, u, v, rc, &th, NULL);
    for (int x = 0; x < m; ++x)
        for (int y = 0; y < m; ++y) pi_out[x * m + y] = (M[x * m + y] - u[x]) - v[y];
    if (M_out) memcpy(M_out, M, sizeof(double) * m * m);
    *theta_out = th;
    free(M);
    return 0;
}

/* ------------------------------------------------------------------------
 * O4. Depth-first branch-and-bound with RLT2-DA bounds (Section 4).
 *
 * Polytomic branching: a node at depth d has d facilities fixed; the next
 * facility in the static Rule-3 order is placed at every free location in
 * ascending order.  Rule 3 (lowest total interaction first): the first
 * facility minimises sum_j (f_ij + f_ji); each next one minimises the summed
 * interaction with the facilities already placed (ties: lowest index).
 *
 * A child inherits its parent's reduced costs (the warm start of Section 4):
 * fixing facility l to location s in the identity above turns every term
 * holding (l,s) into a term of one level lower:
 *   LB'   = LB + R_x[l,s]
 *   X'[i,p] = (R_x[i,p] + R_y[l,i,s,p]) + R_y[i,l,p,s]
 *   Y'[i,j,p,q] = ((R_y[i,j,p,q] + R_z[l,i,j,s,p,q]) + R_z[i,l,j,p,s,q])
 *                 + R_z[i,j,l,p,q,s]
 *   Z' = R_z restricted to the free facilities and locations,
 * all relabelled ascending.  A child then runs the dual ascent from t = 0.
 *
 * Node dual ascent stops after node_iters iterations, when the node is
 * fathomed (ceil(LB - tol) >= UB for integer data, LB >= UB - tol otherwise),
 * or when over the last `window` iterations the bound rose by less than
 * min_improve * max(1, |UB|) (the GAP criterion of Section 5.4).  Nodes with
 * at most 3 free facilities are enumerated exactly.  Every X-LAP assignment,
 * completed with the fixed pairs, is a candidate incumbent.
 * ---------------------------------------------------------------------- */
typedef struct {
    int n;
    const double *F, *D, *B;
    const double *params;
    int node_iters, window;
    double min_improve;
    int enum_below;
    int order[64];
    double UB;
    int best[64];
    long long nodes, da_iters, enumerated;
} orc_bnb_ctx;

void orc_rule3_order(int n, const double *F, int *order)
{
    int placed[64] = {0};
    for (int t = 0; t < n; ++t) {
        int best = -1;
        double bv = HUGE_VAL;
        for (int i = 0; i < n; ++i) {
            if (placed[i]) continue;
            double s = 0.0;
            for (int j = 0; j < n; ++j) {
                if (t == 0) { if (j != i) s += F[IX2(n, i, j)] + F[IX2(n, j, i)]; }
                else if (placed[j]) s += F[IX2(n, i, j)] + F[IX2(n, j, i)];
            }
            if (s < bv) { bv = s; best = i; }
        }
        order[t] = best;
        placed[best] = 1;
    }
}

/* Child state for fixing facility l to location sidx (local indices of the
 * parent), per the fold described above.  The child is itself a QAP on the
 * free facilities and locations: F and D restricted, the fixed pair's cross
 * terms folded into the fixed costs, b'_ip = (b_ip + f_il d_ps) + f_li d_sp,
 * and its own constant b_ls + f_ll d_ss added to the parent's offset, so
 * that every child permutation's cost (plus offset) is the full QAP cost. */
orc_da *orc_da_fold(const orc_da *s, int l, int sidx)
{
    int n = s->n, n1 = n - 1;
    if (n1 < 3 || l < 0 || l >= n || sidx < 0 || sidx >= n) return NULL;
    int fi[64], li[64], a = 0;
    for (int t = 0; t < n; ++t) if (t != l) fi[a++] = t;
    a = 0;
    for (int t = 0; t < n; ++t) if (t != sidx) li[a++] = t;
    size_t m2 = (size_t)n1 * n1, m4 = m2 * m2, m6 = m4 * m2;
    double *Fc = malloc(sizeof(double) * m2), *Dc = malloc(sizeof(double) * m2);
    double *Bc = malloc(sizeof(double) * m2);
    double *Xc = malloc(sizeof(double) * m2);
    double *Yc = calloc(m4, sizeof(double));
    double *Zc = calloc(m6, sizeof(double));
    for (int a1 = 0; a1 < n1; ++a1)
        for (int a2 = 0; a2 < n1; ++a2) {
            Fc[IX2(n1, a1, a2)] = s->F[IX2(n, fi[a1], fi[a2])];
            Dc[IX2(n1, a1, a2)] = s->D[IX2(n, li[a1], li[a2])];
            int i = fi[a1], p = li[a2];
            Bc[IX2(n1, a1, a2)] = (s->B[IX2(n, i, p)] + s->F[IX2(n, i, l)] * s->D[IX2(n, p, sidx)]) +
                                  s->F[IX2(n, l, i)] * s->D[IX2(n, sidx, p)];
        }
    for (int a1 = 0; a1 < n1; ++a1)
        for (int b1 = 0; b1 < n1; ++b1) {
            int i = fi[a1], p = li[b1];
            Xc[IX2(n1, a1, b1)] = (s->X[IX2(n, i, p)] + s->Y[IX4(n, l, i, sidx, p)]) +
                                  s->Y[IX4(n, i, l, p, sidx)];
        }
    for (int a1 = 0; a1 < n1; ++a1)
        for (int a2 = 0; a2 < n1; ++a2) {
            if (a2 == a1) continue;
            for (int b1 = 0; b1 < n1; ++b1)
                for (int b2 = 0; b2 < n1; ++b2) {
                    if (b2 == b1) continue;
                    int i = fi[a1], j = fi[a2], p = li[b1], q = li[b2];
                    Yc[IX4(n1, a1, a2, b1, b2)] =
                        ((s->Y[IX4(n, i, j, p, q)] + s->Z[IX6(n, l, i, j, sidx, p, q)]) +
                         s->Z[IX6(n, i, l, j, p, sidx, q)]) + s->Z[IX6(n, i, j, l, p, q, sidx)];
                    for (int a3 = 0; a3 < n1; ++a3) {
                        if (a3 == a1 || a3 == a2) continue;
                        for (int b3 = 0; b3 < n1; ++b3) {
                            if (b3 == b1 || b3 == b2) continue;
                            Zc[IX6(n1, a1, a2, a3, b1, b2, b3)] = s->Z[IX6(n, i, j, fi[a3], p, q, li[b3])];
                        }
                    }
                }
        }
    double params[5] = {s->kz, s->ky, s->kx, s->phi, s->phiy};
    double lbc = s->LB + s->X[IX2(n, l, sidx)];
    orc_da *cs = orc_da_from_arrays(n1, Fc, Dc, Bc, params, lbc, Xc, Yc, Zc);
    if (cs) cs->offset = s->offset + (s->B[IX2(n, l, sidx)] + s->F[IX2(n, l, l)] * s->D[IX2(n, sidx, sidx)]);
    free(Fc); free(Dc); free(Bc); free(Xc); free(Yc); free(Zc);
    return cs;
}

double orc_da_offset(const orc_da *s) { return s->offset; }

static int fathomed(double LB, double UB, int integer_data)
{
    if (!(UB < HUGE_VAL)) return 0;
    double tol = 1e-9 * fmax(1.0, fabs(UB));
    if (integer_data) return ceil(LB - tol) >= UB;
    return LB >= UB - tol;
}

/* Exact completion of a partial assignment: fac[0..k) free facilities (orig
 * ids), loc[0..k) free locations; perm has the fixed pairs. */
static void enumerate_completions(orc_bnb_ctx *c, int *perm, const int *fac, const int *loc, int k)
{
    int a[16];
    for (int t = 0; t < k; ++t) a[t] = t;
    do {
        for (int t = 0; t < k; ++t) perm[fac[t]] = loc[a[t]];
        double cost = orc_qap_cost(c->n, c->F, c->D, c->B, perm);
        c->enumerated++;
        if (cost < c->UB) { c->UB = cost; memcpy(c->best, perm, sizeof(int) * c->n); }
    } while (next_perm(k, a));
}

static void bnb_node(orc_bnb_ctx *c, int depth, int *perm, const int *fac, const int *loc,
                     int nl, orc_da *s)
{
    int integer_data = orc_is_integer_instance(c->n, c->F, c->D, c->B);
    c->nodes++;
    if (nl <= c->enum_below) {
        enumerate_completions(c, perm, fac, loc, nl);
        return;
    }
    /* node dual ascent */
    double hist[4096];
    int h = 0;
    for (int it = 0; it < c->node_iters; ++it) {
        orc_da_iterate(s);
        c->da_iters++;
        /* candidate incumbent from the X-LAP assignment */
        for (int t = 0; t < nl; ++t) perm[fac[t]] = loc[s->xperm[t]];
        double cost = orc_qap_cost(c->n, c->F, c->D, c->B, perm);
        if (cost < c->UB) { c->UB = cost; memcpy(c->best, perm, sizeof(int) * c->n); }
        if (fathomed(s->LB, c->UB, integer_data)) return;
        if (h < 4096) hist[h++] = s->LB;
        if (h > c->window) {
            double ref = (c->UB < HUGE_VAL) ? fabs(c->UB) : fabs(s->LB);
            if (hist[h - 1] - hist[h - 1 - c->window] < c->min_improve * fmax(1.0, ref)) break;
        }
    }
    /* branch on the next facility of the static order */
    int fl = c->order[depth];
    int l = -1;
    for (int t = 0; t < nl; ++t) if (fac[t] == fl) l = t;
    int n = nl, n1 = nl - 1;
    int cfac[64], cloc[64];
    for (int sidx = 0; sidx < n; ++sidx) {
        double lbc = s->LB + s->X[IX2(n, l, sidx)];
        if (fathomed(lbc, c->UB, integer_data)) continue;
        int a = 0;
        for (int t = 0; t < n; ++t) if (t != l) cfac[a++] = fac[t];
        a = 0;
        for (int t = 0; t < n; ++t) if (t != sidx) cloc[a++] = loc[t];
        perm[fl] = loc[sidx];
        if (n1 <= c->enum_below) {
            c->nodes++;
            enumerate_completions(c, perm, cfac, cloc, n1);
            continue;
        }
        orc_da *cs = orc_da_fold(s, l, sidx);
        bnb_node(c, depth + 1, perm, cfac, cloc, n1, cs);
        orc_da_free(cs);
    }
    perm[fl] = -1;
}

/* Solve to optimality.  params as in orc_da_create; node_iters (e.g. 100),
 * window (25) and min_improve (2e-4) control the node dual ascent; UB0 is the
 * initial incumbent value (HUGE_VAL for none).  stats[0..2] = nodes,
 * dual-ascent iterations, enumerated leaves. */
int orc_bnb(int n, const double *F, const double *D, const double *B, const double *params,
            int node_iters, int window, double min_improve, double UB0,
            int *perm_out, double *obj_out, long long *stats)
{
    if (n < 2 || n > 16) return -1;
    orc_bnb_ctx c;
    memset(&c, 0, sizeof(c));
    double *Bz = NULL;
    if (!B) { Bz = calloc((size_t)n * n, sizeof(double)); B = Bz; }
    c.n = n; c.F = F; c.D = D; c.B = B; c.params = params;
    c.node_iters = node_iters; c.window = window; c.min_improve = min_improve;
    c.enum_below = 3;
    c.UB = UB0;
    orc_rule3_order(n, F, c.order);
    int perm[64], fac[64], loc[64];
    for (int t = 0; t < n; ++t) { perm[t] = -1; fac[t] = t; loc[t] = t; }
    if (n <= c.enum_below) {
        enumerate_completions(&c, perm, fac, loc, n);
    } else {
        orc_da *s = orc_da_create(n, F, D, B, params);
        bnb_node(&c, 0, perm, fac, loc, n, s);
        orc_da_free(s);
    }
    memcpy(perm_out, c.best, sizeof(int) * n);
    *obj_out = c.UB;
    if (stats) { stats[0] = c.nodes; stats[1] = c.da_iters; stats[2] = c.enumerated; }
    free(Bz);
    return 0;
}

/* ------------------------------------------------------------------------
 * O5. An independent exact solver: depth-first B&B with Gilmore-Lawler
 * bounds (no RLT2), same Rule-3 order.  For the partial assignment,
 *   l_ip = b_ip + f_ii d_pp + sum_{fixed j} (f_ij d_{p,s_j} + f_ji d_{s_j,p})
 *          + minprod(f_i. over free j != i, d_p. over free q != p)
 * and the bound is fixed cost + LAP(l).
 * ---------------------------------------------------------------------- */
typedef struct {
    int n;
    const double *F, *D, *B;
    int order[64];
    double UB;
    int best[64];
    long long nodes;
} glb_ctx;

static void glb_node(glb_ctx *c, int depth, int *perm, int *locused)
{
    int n = c->n;
    c->nodes++;
    int fac[64], loc[64], k = 0, kl = 0;
    int isfixed[64] = {0};
    for (int t = 0; t < depth; ++t) isfixed[c->order[t]] = 1;
    for (int i = 0; i < n; ++i) if (!isfixed[i]) fac[k++] = i;
    for (int p = 0; p < n; ++p) if (!locused[p]) loc[kl++] = p;
    if (k == 0) {
        double cost = orc_qap_cost(n, c->F, c->D, c->B, perm);
        if (cost < c->UB) { c->UB = cost; memcpy(c->best, perm, sizeof(int) * n); }
        return;
    }
    /* fixed-fixed cost */
    long double fixed = 0.0L;
    for (int t = 0; t < depth; ++t) {
        int i = c->order[t];
        fixed += c->B[IX2(n, i, perm[i])];
        for (int t2 = 0; t2 < depth; ++t2) {
            int j = c->order[t2];
            fixed += (long double)c->F[IX2(n, i, j)] * c->D[IX2(n, perm[i], perm[j])];
        }
    }
    double *L = malloc(sizeof(double) * k * k);
    double fv[64], dv[64];
    for (int a = 0; a < k; ++a)
        for (int b = 0; b < k; ++b) {
            int i = fac[a], p = loc[b];
            long double s = (long double)c->B[IX2(n, i, p)] + (long double)c->F[IX2(n, i, i)] * c->D[IX2(n, p, p)];
            for (int t = 0; t < depth; ++t) {
                int j = c->order[t];
                s += (long double)c->F[IX2(n, i, j)] * c->D[IX2(n, p, perm[j])];
                s += (long double)c->F[IX2(n, j, i)] * c->D[IX2(n, perm[j], p)];
            }
            int cf = 0, cd = 0;
            for (int a2 = 0; a2 < k; ++a2) if (a2 != a) fv[cf++] = c->F[IX2(n, i, fac[a2])];
            for (int b2 = 0; b2 < k; ++b2) if (b2 != b) dv[cd++] = c->D[IX2(n, p, loc[b2])];
            qsort(fv, cf, sizeof(double), cmp_dbl);
            qsort(dv, cd, sizeof(double), cmp_dbl);
            for (int t = 0; t < cf; ++t) s += (long double)fv[t] * dv[cd - 1 - t];
            L[a * k + b] = (double)s;
        }
    double u[64], v[64], th;
    int rc[64];
    orc_lap(k, L, u, v, rc, &th, NULL);
    long double lb = fixed;
    for (int b = 0; b < k; ++b) lb += L[rc[b] * k + b];
    /* candidate from the LAP assignment */
    int trial[64];
    memcpy(trial, perm, sizeof(int) * n);
    for (int b = 0; b < k; ++b) trial[fac[rc[b]]] = loc[b];
    double tc = orc_qap_cost(n, c->F, c->D, c->B, trial);
    if (tc < c->UB) { c->UB = tc; memcpy(c->best, trial, sizeof(int) * n); }
    free(L);
    double tol = 1e-9 * fmax(1.0, fabs(c->UB));
    if (c->UB < HUGE_VAL && (double)lb >= c->UB - tol) return;
    int f = c->order[depth];
    for (int b = 0; b < kl; ++b) {
        int p = loc[b];
        perm[f] = p;
        locused[p] = 1;
        glb_node(c, depth + 1, perm, locused);
        locused[p] = 0;
        perm[f] = -1;
    }
}

int orc_glb_bnb(int n, const double *F, const double *D, const double *B, double UB0,
                int *perm_out, double *obj_out, long long *nodes)
{
    if (n < 1 || n > 20) return -1;
    glb_ctx c;
    memset(&c, 0, sizeof(c));
    double *Bz = NULL;
    if (!B) { Bz = calloc((size_t)n * n, sizeof(double)); B = Bz; }
    c.n = n; c.F = F; c.D = D; c.B = B; c.UB = UB0;
    orc_rule3_order(n, F, c.order);
    int perm[64], locused[64] = {0};
    for (int t = 0; t < n; ++t) perm[t] = -1;
    glb_node(&c, 0, perm, locused);
    memcpy(perm_out, c.best, sizeof(int) * n);
    *obj_out = c.UB;
    if (nodes) *nodes = c.nodes;
    free(Bz);
    return 0;
}
