/*
 * dock_oracle.h -- FP64 reference of the docking hot path (Alg. 1 of
 * arXiv:2209.05069).  TEST INFRASTRUCTURE ONLY: used by the tests, the smoke
 * check and the benchmark's CPU-baseline leg; never by the GPU library.
 */
#ifndef DOCK_ORACLE_H
#define DOCK_ORACLE_H
#include <stdint.h>

typedef struct {
    int ntypes, nx, ny, nz;
    double spacing;
    double origin[3];
    const float *values; /* [ntypes][nz][ny][nx] */
} or_grid;

typedef struct {
    int n;                    /* atoms */
    const float *xyz;         /* [n][3] ligand frame */
    const uint8_t *type;      /* [n] */
    int nbonds;
    const int32_t *bonds;     /* [nbonds][2] all covalent bonds */
    int nrot;
    const int32_t *rot_bond;  /* [nrot][2] (fixed atom a, moving atom b), sweep order */
    const uint64_t *rot_mask; /* [nrot][mask_words], bit i set = atom i moves */
    int mask_words;
} or_ligand;

typedef struct {
    int restarts;
    const float *start_quat;  /* [restarts][4] (w,x,y,z) */
    int torsion_steps, sweep_passes, align_steps, top_k, final_align, bump_min_bonds;
    double bump_dist, dedup_rmsd;
} or_params;

typedef struct {
    const uint16_t *trace;        /* [restarts][1 + passes*nrot] */
    int nsel;
    const int32_t *sel_restart;   /* [nsel] kept restarts, in output order (NULL: own selection) */
    const uint16_t *final_trace;  /* [nsel] final alignment index */
    double tie_rel, bump_tol;
} or_follow;

/* Class of a followed decision (decision_class / final_class entries). */
enum { OR_EXACT = 0, OR_SCORE_TIE = 1, OR_BUMP_TIE = 2, OR_MISMATCH = 3, OR_NOT_FOLLOWED = 255 };
/* Score ties whose gap exceeds this absolute amount are counted in stats[7]. */
#define OR_ABS_TIE 1e-5

typedef struct {
    double *restart_score;   /* [R] or NULL */
    double *restart_pose;    /* [R][n][3] or NULL */
    double *decision_score;  /* [R][2 + passes*nrot] or NULL */
    uint16_t *trace;         /* [R][1 + passes*nrot] or NULL */
    int32_t n_sel;
    int32_t *sel_restart;    /* [top_k] or NULL */
    double *pose_score;      /* [top_k] or NULL */
    double *pose_xyz;        /* [top_k][n][3] or NULL */
    uint16_t *final_trace;   /* [top_k] or NULL */
    uint8_t *decision_class; /* [R][1 + passes*nrot] class of each followed decision, or NULL */
    uint8_t *final_class;    /* [top_k] class of each followed final alignment, or NULL */
    /* follow statistics: decisions, exact, score ties, bump ties, mismatches,
     * candidates scoring above the applied torsion step (summed), max tie gap,
     * score ties whose gap exceeds OR_ABS_TIE */
    double stats[8];
} or_result;

/* Pocket atoms of the pairwise rescoring stand-in (Rescore Pose). */
typedef struct {
    int n_atoms;
    int ntypes;                /* pocket atom types */
    const float *xyz;          /* [n_atoms][3], pocket frame (the grid's), Angstrom */
    const uint8_t *type;       /* [n_atoms] */
    double contact_dist;       /* Angstrom */
    int lig_ntypes;            /* ligand atom types (the grid's types) */
    const int32_t *weight;     /* [lig_ntypes][ntypes] */
} or_pocket_atoms;

double oracle_interp(const or_grid *g, int t, const double p[3]);
double oracle_score(const or_grid *g, int n, const uint8_t *type, const double *xyz);
int oracle_topo(int n, int nbonds, const int32_t *bonds, int32_t *dist);
int oracle_check_ligand(const or_grid *g, const or_ligand *L);
void oracle_quat_matrix(const float q[4], double M[9]);
void oracle_align_matrix(int A, int o, double M[9]);
int oracle_select(int R, int n, const double *score, const double *pose, int K, double delta,
                  int32_t *sel);
long long oracle_contacts(const or_pocket_atoms *pa, int n, const uint8_t *type,
                          const double *xyz, double tol, long long *boundary);
int oracle_dock_ligand(const or_grid *g, const or_ligand *L, const or_params *P,
                       const or_follow *F, or_result *out);

#endif
