/*
 * dock_oracle.c -- plain single-threaded FP64 reference of the geometric docking
 * hot path (Alg. 1 of Vitali et al., "GPU-optimized Approaches to Molecular
 * Docking-based Virtual Screening in Drug Discovery: A Comparative Analysis",
 * arXiv:2209.05069; Section "Application Description").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle the GPU library is checked
 * against.  Only the tests, the smoke check and the benchmark's CPU-baseline leg
 * may load it; the product path never calls it and shares no code with it.
 *
 * What is computed, per ligand (Alg. 1, and the data-dependency discussion that
 * follows it):
 *   for every restart r (Generate_Starting_Pose):  the ligand, centred on its
 *     centroid, is turned by start orientation q_r and put at the grid centre;
 *   Alignment (Rigid Rotation, Alg. 1 x/y loops): every orientation
 *     R_y(2*pi*j/A) * R_x(2*pi*i/A), i,j in [0,A), about the pose centroid is
 *     scored; the best (first maximum in (i,j) order) is applied;
 *   Optimize Pose (Alg. 1 fragment loop): for P passes, for each rotatable bond
 *     in order, for each step k in [0,T) the moving fragment is turned by
 *     2*pi*k/T about the bond axis; a candidate with an intramolecular bump is
 *     rejected, the others are scored; the best (first maximum in k) is applied;
 *   Select Poses: restarts in order of score (ties by restart index); a pose is
 *     kept unless it is closer than dedup_rmsd (plain RMSD) to one already kept;
 *     at most top_k;
 *   final step (stand-in for the chemical Rescore Pose, whose function the paper
 *     does not give): the alignment again on each kept pose, then its score;
 *     outputs ordered by final score (ties by restart index).
 * Score = sum over atoms of the trilinearly interpolated grid of the atom's
 * type; higher is better.  Bump = some atom pair, one moving and one not, at
 * least bump_min_bonds bonds apart and closer than bump_dist.
 *
 * Parity is pinned by the tests (hand-computed grids, library rotations,
 * exhaustive torsion search on 1-2 bond ligands, geometric invariants,
 * hand-made selection cases); see tests/test_oracle_pins.py.
 *
 * Pairwise rescoring stand-in (oracle_contacts): the paper's Rescore Pose
 * compares every ligand atom with every pocket atom and accumulates the pair
 * terms per pose; its chemical terms are not given, so the stand-in pair term is
 * an integer weight per (ligand type, pocket atom type) for pairs closer than a
 * contact distance.
 *
 * Follow mode: given another implementation's decisions (alignment index and
 * torsion step per decision, kept restarts and final alignment index), the
 * oracle recomputes every candidate in FP64, checks that the given choice is
 * its own argmax or a near-tie (score within tie_rel*max(1,|best|), or a bump
 * decided by a pair distance within bump_tol of bump_dist), counts the cases,
 * and continues with the given choice so later decisions stay comparable.
 * Each followed decision gets a class (exact, score tie, bump tie, mismatch),
 * written per decision when the caller asks for it.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "dock_oracle.h"

#define NONE_ACCEPTED 0xFFFFu

/* ------------------------------------------------------------------------- */
/* Trilinear interpolation of grid t at point p.  The grid point (i,j,k) sits at
 * origin + spacing*(i,j,k).  Coordinates are clamped to the grid box (edge
 * values extend outwards).  Written as the textbook weighted sum over the 8
 * corners of the cell. */
double oracle_interp(const or_grid *g, int t, const double p[3]) {
    const int n[3] = {g->nx, g->ny, g->nz};
    int i0[3];
    double f[3];
    for (int a = 0; a < 3; ++a) {
        double u = (p[a] - g->origin[a]) / g->spacing;
        if (u < 0.0) u = 0.0;
        if (u > (double)(n[a] - 1)) u = (double)(n[a] - 1);
        int c = (int)floor(u);
        if (c > n[a] - 2) c = n[a] - 2;
        i0[a] = c;
        f[a] = u - (double)c;
    }
    const float *v = g->values + (size_t)t * g->nx * g->ny * g->nz;
    double s = 0.0;
    for (int dz = 0; dz <= 1; ++dz)
        for (int dy = 0; dy <= 1; ++dy)
            for (int dx = 0; dx <= 1; ++dx) {
                double w = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1]) *
                           (dz ? f[2] : 1.0 - f[2]);
                size_t idx = ((size_t)(i0[2] + dz) * g->ny + (size_t)(i0[1] + dy)) * g->nx +
                             (size_t)(i0[0] + dx);
                s += w * (double)v[idx];
            }
    return s;
}

/* Score of a pose: sum over atoms (in index order) of the grid of its type. */
double oracle_score(const or_grid *g, int n, const uint8_t *type, const double *xyz) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += oracle_interp(g, type[i], xyz + 3 * i);
    return s;
}

/* ------------------------------------------------------------------------- */
/* Topological (bond-count) distances by breadth-first search from each atom.
 * Unreachable pairs get a large value. */
int oracle_topo(int n, int nbonds, const int32_t *bonds, int32_t *dist) {
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    if (!queue) return -2;
    for (int s = 0; s < n; ++s) {
        for (int j = 0; j < n; ++j) dist[s * n + j] = 1 << 20;
        dist[s * n + s] = 0;
        int head = 0, tail = 0;
        queue[tail++] = s;
        while (head < tail) {
            int x = queue[head++];
            for (int e = 0; e < nbonds; ++e) {
                int y = -1;
                if (bonds[2 * e] == x) y = bonds[2 * e + 1];
                else if (bonds[2 * e + 1] == x) y = bonds[2 * e];
                if (y >= 0 && dist[s * n + y] > dist[s * n + x] + 1) {
                    dist[s * n + y] = dist[s * n + x] + 1;
                    queue[tail++] = y;
                }
            }
        }
    }
    free(queue);
    return 0;
}

static int mask_bit(const uint64_t *m, int i) { return (int)((m[i >> 6] >> (i & 63)) & 1ULL); }

/* Input checks: every index in range; each rotatable bond (a,b) has b in its
 * moving set and a outside it, and the moving set is exactly the atoms that b
 * still reaches once the bond a-b is removed (so the bond splits the ligand in
 * two fragments, as the paper defines rotatable bonds). */
int oracle_check_ligand(const or_grid *g, const or_ligand *L) {
    if (L->n < 1 || L->mask_words < 1 || L->n > 64 * L->mask_words) return -1;
    for (int i = 0; i < L->n; ++i)
        if ((int)L->type[i] >= g->ntypes) return -1;
    for (int e = 0; e < L->nbonds; ++e) {
        int a = L->bonds[2 * e], b = L->bonds[2 * e + 1];
        if (a < 0 || b < 0 || a >= L->n || b >= L->n || a == b) return -1;
    }
    int *seen = (int *)malloc(sizeof(int) * L->n);
    int *stack = (int *)malloc(sizeof(int) * L->n);
    int rc = 0;
    for (int r = 0; r < L->nrot && rc == 0; ++r) {
        int a = L->rot_bond[2 * r], b = L->rot_bond[2 * r + 1];
        const uint64_t *m = L->rot_mask + (size_t)r * L->mask_words;
        if (a < 0 || b < 0 || a >= L->n || b >= L->n || a == b) { rc = -1; break; }
        for (int i = L->n; i < 64 * L->mask_words; ++i)
            if (mask_bit(m, i)) rc = -1;
        int bond_found = 0;
        for (int e = 0; e < L->nbonds; ++e)
            if ((L->bonds[2 * e] == a && L->bonds[2 * e + 1] == b) ||
                (L->bonds[2 * e] == b && L->bonds[2 * e + 1] == a)) bond_found = 1;
        if (!bond_found) rc = -1;
        /* component of b without the edge a-b */
        for (int i = 0; i < L->n; ++i) seen[i] = 0;
        int top = 0;
        stack[top++] = b;
        seen[b] = 1;
        while (top > 0) {
            int x = stack[--top];
            for (int e = 0; e < L->nbonds; ++e) {
                int u = L->bonds[2 * e], v = L->bonds[2 * e + 1];
                if ((u == a && v == b) || (u == b && v == a)) continue;
                int y = (u == x) ? v : (v == x) ? u : -1;
                if (y >= 0 && !seen[y]) { seen[y] = 1; stack[top++] = y; }
            }
        }
        if (seen[a]) rc = -1; /* bond inside a ring: not rotatable */
        for (int i = 0; i < L->n; ++i)
            if (seen[i] != mask_bit(m, i)) rc = -1;
    }
    free(seen);
    free(stack);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Rotation matrix of the unit quaternion (w,x,y,z) (normalised first). */
void oracle_quat_matrix(const float q[4], double M[9]) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    double s = sqrt(w * w + x * x + y * y + z * z);
    w /= s; x /= s; y /= s; z /= s;
    M[0] = 1 - 2 * (y * y + z * z); M[1] = 2 * (x * y - w * z);     M[2] = 2 * (x * z + w * y);
    M[3] = 2 * (x * y + w * z);     M[4] = 1 - 2 * (x * x + z * z); M[5] = 2 * (y * z - w * x);
    M[6] = 2 * (x * z - w * y);     M[7] = 2 * (y * z + w * x);     M[8] = 1 - 2 * (x * x + y * y);
}

static void matmul3(const double A[9], const double B[9], double C[9]) {
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            C[3 * r + c] = A[3 * r] * B[c] + A[3 * r + 1] * B[3 + c] + A[3 * r + 2] * B[6 + c];
}

/* Alignment orientation o = i*A + j: R_y(beta_j) * R_x(alpha_i). */
void oracle_align_matrix(int A, int o, double M[9]) {
    int i = o / A, j = o % A;
    double al = 2.0 * M_PI * i / A, be = 2.0 * M_PI * j / A;
    double Rx[9] = {1, 0, 0, 0, cos(al), -sin(al), 0, sin(al), cos(al)};
    double Ry[9] = {cos(be), 0, sin(be), 0, 1, 0, -sin(be), 0, cos(be)};
    matmul3(Ry, Rx, M);
}

static void centroid(int n, const double *X, double c[3]) {
    c[0] = c[1] = c[2] = 0.0;
    for (int i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) c[a] += X[3 * i + a];
    for (int a = 0; a < 3; ++a) c[a] /= n;
}

/* Z = M (Y - c) + c */
static void rotate_about(int n, const double *Y, const double M[9], const double c[3], double *Z) {
    for (int i = 0; i < n; ++i) {
        double d[3] = {Y[3 * i] - c[0], Y[3 * i + 1] - c[1], Y[3 * i + 2] - c[2]};
        for (int a = 0; a < 3; ++a)
            Z[3 * i + a] = M[3 * a] * d[0] + M[3 * a + 1] * d[1] + M[3 * a + 2] * d[2] + c[a];
    }
}

/* Rodrigues: turn v by theta about unit axis u. */
static void rodrigues(const double u[3], double ct, double st, const double v[3], double out[3]) {
    double cr[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
    double ud = u[0] * v[0] + u[1] * v[1] + u[2] * v[2];
    for (int a = 0; a < 3; ++a) out[a] = v[a] * ct + cr[a] * st + u[a] * ud * (1.0 - ct);
}

static double rmsd_plain(int n, const double *P, const double *Q) {
    double s = 0.0;
    for (int i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) {
            double d = P[3 * i + a] - Q[3 * i + a];
            s += d * d;
        }
    return sqrt(s / n);
}

/* ------------------------------------------------------------------------- */
/* Select Poses: order restarts by (score desc, index asc); keep a pose unless
 * its RMSD to a kept one is below delta; stop at K.  Returns the count. */
int oracle_select(int R, int n, const double *score, const double *pose, int K, double delta,
                  int32_t *sel) {
    int *ord = (int *)malloc(sizeof(int) * (R > 0 ? R : 1));
    for (int r = 0; r < R; ++r) ord[r] = r;
    /* insertion sort: stable, by descending score */
    for (int i = 1; i < R; ++i) {
        int v = ord[i], j = i - 1;
        while (j >= 0 && score[ord[j]] < score[v]) { ord[j + 1] = ord[j]; --j; }
        ord[j + 1] = v;
    }
    int ns = 0;
    for (int t = 0; t < R && ns < K; ++t) {
        int r = ord[t], keep = 1;
        for (int s = 0; s < ns; ++s)
            if (rmsd_plain(n, pose + (size_t)r * n * 3, pose + (size_t)sel[s] * n * 3) < delta) {
                keep = 0;
                break;
            }
        if (keep) sel[ns++] = r;
    }
    free(ord);
    return ns;
}

/* ------------------------------------------------------------------------- */
typedef struct {
    const or_grid *g;
    const or_ligand *L;
    const or_params *P;
    const or_follow *F;
    int32_t *topo;     /* [n][n] */
    double *stats;     /* follow statistics */
    uint8_t *cls_out;  /* where the class of the next followed decision goes, or NULL */
} ctx_t;

static double tie_tol(const ctx_t *C, double best) {
    double m = fabs(best) > 1.0 ? fabs(best) : 1.0;
    return C->F->tie_rel * m;
}

/* Count a followed decision of class cls; gap = best score minus the score of
 * the given choice (score ties only). */
static void record(const ctx_t *C, int cls, double gap) {
    C->stats[0] += 1;
    C->stats[1 + cls] += 1;
    if (cls == OR_SCORE_TIE) {
        if (gap > C->stats[6]) C->stats[6] = gap;
        if (gap > OR_ABS_TIE) C->stats[7] += 1;
    }
    if (C->cls_out) *C->cls_out = (uint8_t)cls;
}

/* Alignment of pose Y (in place).  Returns the chosen orientation index. */
static int align_pose(const ctx_t *C, double *Y, int follow_idx) {
    const int n = C->L->n, A = C->P->align_steps, NO = A * A;
    double c[3], M[9];
    double *Z = (double *)malloc(sizeof(double) * 3 * n);
    centroid(n, Y, c);
    double best = -INFINITY;
    int best_o = 0;
    double *S = (double *)malloc(sizeof(double) * NO);
    for (int o = 0; o < NO; ++o) {
        oracle_align_matrix(A, o, M);
        rotate_about(n, Y, M, c, Z);
        S[o] = oracle_score(C->g, n, C->L->type, Z);
        if (S[o] > best) { best = S[o]; best_o = o; }
    }
    int use = best_o;
    if (follow_idx >= 0) {
        if (follow_idx >= NO) record(C, OR_MISMATCH, 0.0);
        else if (follow_idx == best_o) record(C, OR_EXACT, 0.0);
        else if (best - S[follow_idx] <= tie_tol(C, best))
            record(C, OR_SCORE_TIE, best - S[follow_idx]);
        else record(C, OR_MISMATCH, 0.0);
        if (follow_idx < NO) use = follow_idx;
    }
    oracle_align_matrix(A, use, M);
    rotate_about(n, Y, M, c, Z);
    memcpy(Y, Z, sizeof(double) * 3 * n);
    free(Z);
    free(S);
    return use;
}

/* Candidate k of rotatable bond b applied to Y -> Z. */
static void torsion_candidate(const ctx_t *C, int b, int k, const double *Y, double *Z) {
    const int n = C->L->n, T = C->P->torsion_steps;
    const int a_at = C->L->rot_bond[2 * b], b_at = C->L->rot_bond[2 * b + 1];
    const uint64_t *m = C->L->rot_mask + (size_t)b * C->L->mask_words;
    double u[3] = {Y[3 * b_at] - Y[3 * a_at], Y[3 * b_at + 1] - Y[3 * a_at + 1],
                   Y[3 * b_at + 2] - Y[3 * a_at + 2]};
    double ul = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    for (int a = 0; a < 3; ++a) u[a] /= ul;
    double th = 2.0 * M_PI * k / T, ct = cos(th), st = sin(th);
    for (int i = 0; i < n; ++i) {
        if (!mask_bit(m, i)) {
            for (int a = 0; a < 3; ++a) Z[3 * i + a] = Y[3 * i + a];
            continue;
        }
        double v[3] = {Y[3 * i] - Y[3 * a_at], Y[3 * i + 1] - Y[3 * a_at + 1],
                       Y[3 * i + 2] - Y[3 * a_at + 2]};
        double w[3];
        rodrigues(u, ct, st, v, w);
        for (int a = 0; a < 3; ++a) Z[3 * i + a] = Y[3 * a_at + a] + w[a];
    }
}

/* Bump check of candidate Z for bond b.  With early exit (free mode) returns at
 * the first bump; otherwise computes the smallest eligible pair distance. */
static int bumped(const ctx_t *C, int b, const double *Z, int early_exit, double *dmin_out) {
    const int n = C->L->n;
    const uint64_t *m = C->L->rot_mask + (size_t)b * C->L->mask_words;
    const double d2lim = C->P->bump_dist * C->P->bump_dist;
    double dmin2 = INFINITY;
    int hit = 0;
    for (int i = 0; i < n; ++i) {
        if (!mask_bit(m, i)) continue;
        for (int j = 0; j < n; ++j) {
            if (mask_bit(m, j)) continue;
            if (C->topo[i * n + j] < C->P->bump_min_bonds) continue;
            double dx = Z[3 * i] - Z[3 * j], dy = Z[3 * i + 1] - Z[3 * j + 1],
                   dz = Z[3 * i + 2] - Z[3 * j + 2];
            double d2 = dx * dx + dy * dy + dz * dz;
            if (d2 < dmin2) dmin2 = d2;
            if (d2 < d2lim) {
                hit = 1;
                if (early_exit) {
                    if (dmin_out) *dmin_out = sqrt(dmin2);
                    return 1;
                }
            }
        }
    }
    if (dmin_out) *dmin_out = sqrt(dmin2);
    return hit;
}

/* One torsion decision for bond b on pose Y (in place).  Returns the applied
 * step, or NONE_ACCEPTED when every candidate bumps. */
static int torsion_decision(const ctx_t *C, int b, double *Y, int follow_k, double *score_after) {
    const int n = C->L->n, T = C->P->torsion_steps;
    double *Z = (double *)malloc(sizeof(double) * 3 * n);
    int chosen;
    if (follow_k < 0) {
        /* free mode: bump check first (early exit), score only bump-free poses */
        double best = -INFINITY;
        int best_k = -1;
        for (int k = 0; k < T; ++k) {
            torsion_candidate(C, b, k, Y, Z);
            if (bumped(C, b, Z, 1, NULL)) continue;
            double s = oracle_score(C->g, n, C->L->type, Z);
            if (s > best) { best = s; best_k = k; }
        }
        chosen = best_k < 0 ? (int)NONE_ACCEPTED : best_k;
    } else {
        /* follow mode: evaluate every candidate fully */
        double *S = (double *)malloc(sizeof(double) * T);
        double *D = (double *)malloc(sizeof(double) * T);
        const double bd = C->P->bump_dist, tol = C->F->bump_tol;
        double best = -INFINITY, best_sure = -INFINITY;
        int best_k = -1;
        for (int k = 0; k < T; ++k) {
            torsion_candidate(C, b, k, Y, Z);
            int hit = bumped(C, b, Z, 0, &D[k]);
            S[k] = oracle_score(C->g, n, C->L->type, Z);
            if (!hit && S[k] > best) { best = S[k]; best_k = k; }
            if (D[k] >= bd + tol && S[k] > best_sure) best_sure = S[k];
        }
        /* diagnostic: candidates scoring above the applied one (all bumped when the
         * applied one is the best bump-free candidate) */
        if (follow_k >= 0 && follow_k < T)
            for (int k = 0; k < T; ++k)
                if (S[k] > S[follow_k]) C->stats[5] += 1;
        if (follow_k == (int)NONE_ACCEPTED) {
            if (best_k < 0) record(C, OR_EXACT, 0.0);
            else if (best_sure == -INFINITY) record(C, OR_BUMP_TIE, 0.0); /* only near-boundary candidates */
            else record(C, OR_MISMATCH, 0.0);
        } else if (follow_k >= T) {
            record(C, OR_MISMATCH, 0.0);
        } else if (follow_k == best_k) {
            record(C, OR_EXACT, 0.0);
        } else {
            int given_ok = D[follow_k] >= bd - tol;                 /* not surely bumped */
            double ref = best_sure;                                 /* best surely-free score */
            if (given_ok && (ref == -INFINITY || S[follow_k] >= ref - tie_tol(C, ref))) {
                if (D[follow_k] < bd || (best_k >= 0 && best - S[follow_k] > tie_tol(C, best)))
                    record(C, OR_BUMP_TIE, 0.0);                    /* decided by a bump near-tie */
                else
                    record(C, OR_SCORE_TIE, fabs(best - S[follow_k]));
            } else {
                record(C, OR_MISMATCH, 0.0);
            }
        }
        chosen = follow_k;
        free(S);
        free(D);
    }
    if (chosen != (int)NONE_ACCEPTED && chosen < T) {
        torsion_candidate(C, b, chosen, Y, Z);
        memcpy(Y, Z, sizeof(double) * 3 * n);
    }
    if (score_after) *score_after = oracle_score(C->g, n, C->L->type, Y);
    free(Z);
    return chosen;
}

/* ------------------------------------------------------------------------- */
int oracle_dock_ligand(const or_grid *g, const or_ligand *L, const or_params *P,
                       const or_follow *F, or_result *out) {
    if (oracle_check_ligand(g, L)) return -1;
    if (P->restarts < 1 || P->torsion_steps < 1 || P->sweep_passes < 0 || P->align_steps < 1 ||
        P->top_k < 1 || g->nx < 2 || g->ny < 2 || g->nz < 2)
        return -1;
    const int n = L->n, R = P->restarts, D = 1 + P->sweep_passes * L->nrot;
    ctx_t C;
    C.g = g; C.L = L; C.P = P; C.F = F;
    C.stats = out->stats;
    C.cls_out = NULL;
    for (int s = 0; s < 8; ++s) out->stats[s] = 0.0;
    if (out->decision_class) memset(out->decision_class, OR_NOT_FOLLOWED, (size_t)R * D);
    if (out->final_class) memset(out->final_class, OR_NOT_FOLLOWED, (size_t)P->top_k);
    C.topo = (int32_t *)malloc(sizeof(int32_t) * n * n);
    oracle_topo(n, L->nbonds, L->bonds, C.topo);

    /* ligand centroid in its own frame */
    double *X = (double *)malloc(sizeof(double) * 3 * n);
    for (int i = 0; i < 3 * n; ++i) X[i] = (double)L->xyz[i];
    double c0[3];
    centroid(n, X, c0);
    const double gc[3] = {g->origin[0] + g->spacing * (g->nx - 1) / 2.0,
                          g->origin[1] + g->spacing * (g->ny - 1) / 2.0,
                          g->origin[2] + g->spacing * (g->nz - 1) / 2.0};

    double *poses = (double *)malloc(sizeof(double) * 3 * n * R);
    double *scores = (double *)malloc(sizeof(double) * R);
    double *Y = (double *)malloc(sizeof(double) * 3 * n);
    const int DS = 2 + P->sweep_passes * L->nrot;

    for (int r = 0; r < R; ++r) {
        /* Generate_Starting_Pose */
        double Q[9];
        oracle_quat_matrix(P->start_quat + 4 * r, Q);
        for (int i = 0; i < n; ++i) {
            double d[3] = {X[3 * i] - c0[0], X[3 * i + 1] - c0[1], X[3 * i + 2] - c0[2]};
            for (int a = 0; a < 3; ++a)
                Y[3 * i + a] = Q[3 * a] * d[0] + Q[3 * a + 1] * d[1] + Q[3 * a + 2] * d[2] + gc[a];
        }
        if (out->decision_score)
            out->decision_score[(size_t)r * DS] = oracle_score(g, n, L->type, Y);
        /* Alignment */
        const uint16_t *ftr = F ? F->trace + (size_t)r * D : NULL;
        C.cls_out = out->decision_class ? out->decision_class + (size_t)r * D : NULL;
        int o = align_pose(&C, Y, ftr ? (int)ftr[0] : -1);
        if (out->trace) out->trace[(size_t)r * D] = (uint16_t)o;
        if (out->decision_score)
            out->decision_score[(size_t)r * DS + 1] = oracle_score(g, n, L->type, Y);
        /* Optimize Pose: fragments in order, P passes */
        int d = 1;
        for (int p = 0; p < P->sweep_passes; ++p)
            for (int b = 0; b < L->nrot; ++b, ++d) {
                double sa;
                C.cls_out = out->decision_class ? out->decision_class + (size_t)r * D + d : NULL;
                int k = torsion_decision(&C, b, Y, ftr ? (int)ftr[d] : -1, &sa);
                if (out->trace) out->trace[(size_t)r * D + d] = (uint16_t)k;
                if (out->decision_score) out->decision_score[(size_t)r * DS + 1 + d] = sa;
            }
        memcpy(poses + (size_t)r * 3 * n, Y, sizeof(double) * 3 * n);
        scores[r] = oracle_score(g, n, L->type, Y);
    }
    if (out->restart_score) memcpy(out->restart_score, scores, sizeof(double) * R);
    if (out->restart_pose) memcpy(out->restart_pose, poses, sizeof(double) * 3 * n * R);

    /* Select Poses */
    const int K = P->top_k;
    int32_t *sel = (int32_t *)malloc(sizeof(int32_t) * (K > R ? K : R));
    int ns;
    if (F && F->sel_restart) {
        ns = F->nsel;
        for (int s = 0; s < ns; ++s) sel[s] = F->sel_restart[s];
    } else {
        ns = oracle_select(R, n, scores, poses, K, P->dedup_rmsd, sel);
    }

    /* final rigid step and final score */
    double *fpose = (double *)malloc(sizeof(double) * 3 * n * (ns > 0 ? ns : 1));
    double *fscore = (double *)malloc(sizeof(double) * (ns > 0 ? ns : 1));
    int *fidx = (int *)malloc(sizeof(int) * (ns > 0 ? ns : 1));
    for (int s = 0; s < ns; ++s) {
        int r = sel[s];
        if (r < 0 || r >= R) { r = 0; C.stats[4] += 1; }  /* not a decision: kept restart out of range */
        memcpy(Y, poses + (size_t)r * 3 * n, sizeof(double) * 3 * n);
        fidx[s] = 0;
        if (P->final_align) {
            int fo = (F && F->final_trace) ? (int)F->final_trace[s] : -1;
            C.cls_out = (out->final_class && s < P->top_k) ? out->final_class + s : NULL;
            fidx[s] = align_pose(&C, Y, fo);
        }
        memcpy(fpose + (size_t)s * 3 * n, Y, sizeof(double) * 3 * n);
        fscore[s] = oracle_score(g, n, L->type, Y);
    }
    /* order outputs by (final score desc, restart asc); follow mode keeps the given order */
    int *ord = (int *)malloc(sizeof(int) * (ns > 0 ? ns : 1));
    for (int s = 0; s < ns; ++s) ord[s] = s;
    if (!(F && F->sel_restart)) {
        for (int i = 1; i < ns; ++i) {
            int v = ord[i], j = i - 1;
            while (j >= 0 && (fscore[ord[j]] < fscore[v] ||
                              (fscore[ord[j]] == fscore[v] && sel[ord[j]] > sel[v]))) {
                ord[j + 1] = ord[j];
                --j;
            }
            ord[j + 1] = v;
        }
    }
    out->n_sel = ns;
    for (int s = 0; s < ns; ++s) {
        int q = ord[s];
        if (out->sel_restart) out->sel_restart[s] = sel[q];
        if (out->pose_score) out->pose_score[s] = fscore[q];
        if (out->pose_xyz) memcpy(out->pose_xyz + (size_t)s * 3 * n, fpose + (size_t)q * 3 * n,
                                  sizeof(double) * 3 * n);
        if (out->final_trace) out->final_trace[s] = (uint16_t)fidx[q];
    }
    free(ord); free(fidx); free(fscore); free(fpose); free(sel);
    free(Y); free(scores); free(poses); free(X); free(C.topo);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Contact score of a pose (stand-in for the chemical Rescore Pose): the sum,
 * over every ligand atom i and every pocket atom j, of weight[type_i][type_j]
 * for the pairs with |x_i - p_j| < contact_dist.  All l x p pairs are visited,
 * as the paper's rescoring does.  *boundary (when not NULL) receives the sum of
 * |weight| over the pairs whose distance lies within tol of contact_dist: the
 * pairs whose verdict a rounding of the positions by up to tol could change. */
long long oracle_contacts(const or_pocket_atoms *pa, int n, const uint8_t *type,
                          const double *xyz, double tol, long long *boundary) {
    const double dc = pa->contact_dist;
    long long sum = 0, edge = 0;
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < pa->n_atoms; ++j) {
            const double dx = xyz[3 * i + 0] - (double)pa->xyz[3 * j + 0];
            const double dy = xyz[3 * i + 1] - (double)pa->xyz[3 * j + 1];
            const double dz = xyz[3 * i + 2] - (double)pa->xyz[3 * j + 2];
            const double d = sqrt(dx * dx + dy * dy + dz * dz);
            const int32_t w = pa->weight[(size_t)type[i] * pa->ntypes + pa->type[j]];
            if (d < dc) sum += w;
            if (fabs(d - dc) <= tol) edge += w < 0 ? -(long long)w : (long long)w;
        }
    }
    if (boundary) *boundary = edge;
    return sum;
}
