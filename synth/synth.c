/*
 * synth.c -- seeded synthetic inputs for the docking hot path.
 *
 * This module only MAKES INPUTS: pocket score grids, random-tree ligand
 * libraries (coordinates, atom types, covalent bonds, rotatable bonds and their
 * moving-fragment masks) and the table of start orientations.  It holds none
 * of the docking arithmetic; both the FP64 oracle and the GPU library consume
 * its outputs as plain arrays.
 *
 * Randomness: splitmix64 (Steele, Lea, Flood, "Fast splittable pseudorandom
 * number generators", OOPSLA 2014), one independent stream per (seed, tag,
 * index), so every ligand is reproducible on its own.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SYNTH_MAX_ATOMS 256
#define SYNTH_MAX_ROT 32

static inline uint64_t sm64(uint64_t *s) {
    uint64_t z = (*s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Independent stream for (seed, tag, index). */
static uint64_t stream_init(uint64_t seed, uint64_t tag, uint64_t index) {
    uint64_t s = seed ^ (tag * 0xD1B54A32D192ED03ULL);
    (void)sm64(&s);
    s ^= (index + 1) * 0x9E3779B97F4A7C15ULL;
    (void)sm64(&s);
    return s;
}

static inline double u01(uint64_t *s) { return (double)(sm64(s) >> 11) * 0x1.0p-53; }
static inline double uab(uint64_t *s, double a, double b) { return a + (b - a) * u01(s); }
/* uniform integer in [lo, hi] */
static inline int uint_range(uint64_t *s, int lo, int hi) {
    uint64_t span = (uint64_t)(hi - lo + 1);
    return lo + (int)(sm64(s) % span);
}

/* ------------------------------------------------------------------------- */
/* Pocket grids: per atom type, a sum of isotropic Gaussians sampled in FP64 at
 * the grid points and stored as FP32, layout [type][z][y][x] (x fastest).
 * Grid point (i,j,k) sits at origin + h*(i,j,k) with origin = -h*(n-1)/2, so
 * the grid centre is (0,0,0).  Gaussian centres are uniform in the cube
 * [-centre_half, centre_half]^3, sigma ~ U(sig_lo, sig_hi), amplitude ~
 * U(amp_lo, amp_hi).  gauss_out (optional) receives [type][g][cx,cy,cz,sigma,amp].
 */
int synth_pocket(uint64_t seed, int ntypes, int n, double h, int ngauss, double centre_half,
                 double sig_lo, double sig_hi, double amp_lo, double amp_hi, float *out,
                 double *gauss_out) {
    if (ntypes < 1 || n < 2 || h <= 0 || ngauss < 0) return -1;
    double *g = (double *)malloc(sizeof(double) * 5 * (size_t)(ngauss > 0 ? ngauss : 1));
    if (!g) return -2;
    const double origin = -h * (n - 1) / 2.0;
    for (int t = 0; t < ntypes; ++t) {
        uint64_t st = stream_init(seed, 0x706f636b6574ULL /* "pocket" */, (uint64_t)t);
        for (int q = 0; q < ngauss; ++q) {
            g[5 * q + 0] = uab(&st, -centre_half, centre_half);
            g[5 * q + 1] = uab(&st, -centre_half, centre_half);
            g[5 * q + 2] = uab(&st, -centre_half, centre_half);
            g[5 * q + 3] = uab(&st, sig_lo, sig_hi);
            g[5 * q + 4] = uab(&st, amp_lo, amp_hi);
        }
        if (gauss_out) memcpy(gauss_out + (size_t)t * 5 * ngauss, g, sizeof(double) * 5 * ngauss);
        float *vt = out + (size_t)t * n * n * n;
#pragma omp parallel for schedule(static)
        for (int k = 0; k < n; ++k) {
            const double z = origin + h * k;
            for (int j = 0; j < n; ++j) {
                const double y = origin + h * j;
                for (int i = 0; i < n; ++i) {
                    const double x = origin + h * i;
                    double v = 0.0;
                    for (int q = 0; q < ngauss; ++q) {
                        const double dx = x - g[5 * q], dy = y - g[5 * q + 1], dz = z - g[5 * q + 2];
                        const double s = g[5 * q + 3];
                        v += g[5 * q + 4] * exp(-(dx * dx + dy * dy + dz * dz) / (2.0 * s * s));
                    }
                    vt[((size_t)k * n + j) * n + i] = (float)v;
                }
            }
        }
    }
    free(g);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Ligand sizes.  kind 0: n ~ U{a0..a1}, B ~ U{b0..b1}.
 * kind 1: n ~ round(lognormal(median a0, sigma_log s)) clipped [a1lo, a1hi],
 *         B ~ Poisson(lam) clipped [0, bmax].
 * B is NOT clipped to what the tree allows here; synth_library does that. */
int synth_sizes_uniform(uint64_t seed, int L, int a0, int a1, int b0, int b1, int32_t *n_out,
                        int32_t *b_out) {
    if (a0 < 1 || a1 < a0 || a1 > SYNTH_MAX_ATOMS || b0 < 0 || b1 < b0 || b1 > SYNTH_MAX_ROT) return -1;
    for (int l = 0; l < L; ++l) {
        uint64_t st = stream_init(seed, 0x73697a6573ULL /* "sizes" */, (uint64_t)l);
        n_out[l] = uint_range(&st, a0, a1);
        b_out[l] = uint_range(&st, b0, b1);
    }
    return 0;
}

int synth_sizes_lognormal(uint64_t seed, int L, double median, double sigma_log, int nlo, int nhi,
                          double lam, int bmax, int32_t *n_out, int32_t *b_out) {
    if (nlo < 1 || nhi < nlo || nhi > SYNTH_MAX_ATOMS || bmax < 0 || bmax > SYNTH_MAX_ROT) return -1;
    for (int l = 0; l < L; ++l) {
        uint64_t st = stream_init(seed, 0x6c6f676e6fULL /* "logno" */, (uint64_t)l);
        /* Box-Muller normal */
        double u1 = u01(&st), u2 = u01(&st);
        if (u1 < 1e-300) u1 = 1e-300;
        double z = sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
        long n = lround(median * exp(sigma_log * z));
        if (n < nlo) n = nlo;
        if (n > nhi) n = nhi;
        /* Poisson by Knuth's multiplication method (lam is small) */
        double Lm = exp(-lam), p = 1.0;
        int k = 0;
        do { ++k; p *= u01(&st); } while (p > Lm);
        int b = k - 1;
        if (b > bmax) b = bmax;
        n_out[l] = (int32_t)n;
        b_out[l] = b;
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Random-tree ligand geometry.
 *
 * Atom 0 is the root at the origin.  Atom c>0 picks a parent uniformly among
 * earlier atoms with fewer than 4 bonds and is placed by NeRF (Parsons et al.,
 * J. Comput. Chem. 2005) from (great-grandparent, grandparent, parent) with bond
 * U(1.45,1.55) A, bond angle U(104.5,114.5) deg; the first child of a parent takes
 * a dihedral U[0,360) and later siblings are offset by 120 deg.  An atom is
 * redrawn (new parent and geometry) while it lies closer than clash_dist to any
 * atom 4 or more bonds away, so every input conformation is clash-free.
 *
 * Rotatable bonds: B distinct tree edges whose two atoms both have >= 2 bonds,
 * chosen uniformly; the moving fragment is the subtree below the edge (away
 * from atom 0).  They are listed by increasing moving-atom index. */

typedef struct { double x, y, z; } v3;
static inline v3 v3sub(v3 a, v3 b) { v3 r = {a.x - b.x, a.y - b.y, a.z - b.z}; return r; }
static inline v3 v3add(v3 a, v3 b) { v3 r = {a.x + b.x, a.y + b.y, a.z + b.z}; return r; }
static inline v3 v3scale(v3 a, double s) { v3 r = {a.x * s, a.y * s, a.z * s}; return r; }
static inline double v3dot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static inline v3 v3cross(v3 a, v3 b) {
    v3 r = {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
    return r;
}
static inline v3 v3unit(v3 a) { return v3scale(a, 1.0 / sqrt(v3dot(a, a))); }

/* Place d such that |cd| = bond, angle(b,c,d) = ang, dihedral(a,b,c,d) = phi. */
static v3 nerf(v3 a, v3 b, v3 c, double bond, double ang, double phi) {
    v3 bc = v3unit(v3sub(c, b));
    v3 nrm = v3cross(v3sub(b, a), bc);
    double nn = sqrt(v3dot(nrm, nrm));
    if (nn < 1e-8) { /* a,b,c collinear: any perpendicular */
        v3 t = fabs(bc.x) < 0.9 ? (v3){1, 0, 0} : (v3){0, 1, 0};
        nrm = v3cross(t, bc);
        nn = sqrt(v3dot(nrm, nrm));
    }
    nrm = v3scale(nrm, 1.0 / nn);
    v3 m = v3cross(nrm, bc);
    double dx = -bond * cos(ang), dy = bond * sin(ang) * cos(phi), dz = bond * sin(ang) * sin(phi);
    return v3add(c, v3add(v3scale(bc, dx), v3add(v3scale(m, dy), v3scale(nrm, dz))));
}

typedef struct {
    int n;
    int parent[SYNTH_MAX_ATOMS];
    int deg[SYNTH_MAX_ATOMS];
    int nchild[SYNTH_MAX_ATOMS];
    int first_child[SYNTH_MAX_ATOMS];
    double phi0[SYNTH_MAX_ATOMS];
    v3 pos[SYNTH_MAX_ATOMS];
    unsigned char topo[SYNTH_MAX_ATOMS][SYNTH_MAX_ATOMS];
} tree_t;

/* Try to add atom c with parent p; returns 1 on success (no clash). */
static int try_place(tree_t *T, int c, int p, uint64_t *st, double clash_dist) {
    const double deg2rad = M_PI / 180.0;
    double bond = uab(st, 1.45, 1.55);
    double ang = uab(st, 104.5, 114.5) * deg2rad;
    v3 pc;
    /* reference atoms g (grandparent side) and a (great-grandparent side) */
    int g = -1;
    if (T->parent[p] >= 0) g = T->parent[p];
    else if (T->nchild[p] > 0) g = T->first_child[p];
    if (g < 0) {
        /* p is the root with no neighbour yet: put c along +x */
        pc = v3add(T->pos[p], (v3){bond, 0, 0});
    } else {
        /* The dihedral reference must not change between siblings, so it is the
         * parent of g when p is not the root, else a fixed point built from g, p. */
        v3 a;
        int aa = (T->parent[p] >= 0) ? T->parent[g] : -1;
        if (aa >= 0) a = T->pos[aa];
        else {
            v3 gp = v3unit(v3sub(T->pos[p], T->pos[g]));
            v3 t = fabs(gp.x) < 0.9 ? (v3){1, 0, 0} : (v3){0, 1, 0};
            a = v3add(T->pos[g], v3cross(t, gp));
        }
        /* children of p other than its reference g */
        int sib = T->nchild[p] - ((T->parent[p] < 0 && g >= 0) ? 1 : 0);
        double phi;
        if (sib <= 0) phi = uab(st, 0.0, 2.0 * M_PI);
        else phi = T->phi0[p] + (2.0 * M_PI / 3.0) * sib;
        pc = nerf(a, T->pos[g], T->pos[p], bond, ang, phi);
        if (sib <= 0) T->phi0[p] = phi;  /* harmless if this try is rejected: redrawn next time */
    }
    /* clash check against atoms >= 4 bonds away: topo(c,x) = topo(p,x) + 1 */
    for (int x = 0; x < c; ++x) {
        int tcx = T->topo[p][x] + 1;
        if (tcx >= 4) {
            v3 d = v3sub(pc, T->pos[x]);
            if (v3dot(d, d) < clash_dist * clash_dist) return 0;
        }
    }
    T->pos[c] = pc;
    T->parent[c] = p;
    T->deg[c] = 1;
    T->deg[p] += 1;
    if (T->nchild[p] == 0) T->first_child[p] = c;
    T->nchild[p] += 1;
    T->nchild[c] = 0;
    T->first_child[c] = -1;
    for (int x = 0; x < c; ++x) {
        int tcx = T->topo[p][x] + 1;
        T->topo[c][x] = T->topo[x][c] = (unsigned char)(tcx > 255 ? 255 : tcx);
    }
    T->topo[c][c] = 0;
    return 1;
}

static int build_tree(tree_t *T, int n, uint64_t *st, double clash_dist) {
    T->n = n;
    T->parent[0] = -1;
    T->deg[0] = 0;
    T->nchild[0] = 0;
    T->first_child[0] = -1;
    T->pos[0] = (v3){0, 0, 0};
    T->topo[0][0] = 0;
    int cand[SYNTH_MAX_ATOMS];
    for (int c = 1; c < n; ++c) {
        int ok = 0;
        for (int tries = 0; tries < 2000 && !ok; ++tries) {
            int nc = 0;
            for (int x = 0; x < c; ++x)
                if (T->deg[x] < 4) cand[nc++] = x;
            if (nc == 0) return 0;
            int p = cand[uint_range(st, 0, nc - 1)];
            ok = try_place(T, c, p, st, clash_dist);
        }
        if (!ok) return 0;
    }
    return 1;
}

/* Count atoms in the subtree of c (c and its descendants). */
static void subtree_mask(const tree_t *T, int c, uint64_t *mask, int words) {
    memset(mask, 0, sizeof(uint64_t) * words);
    mask[c >> 6] |= 1ULL << (c & 63);
    /* parents always have smaller indices, so one ascending pass suffices */
    for (int x = c + 1; x < T->n; ++x) {
        int p = T->parent[x];
        if (p >= 0 && (mask[p >> 6] >> (p & 63) & 1ULL)) mask[x >> 6] |= 1ULL << (x & 63);
    }
}

/*
 * Build a CSR library of L ligands with the given sizes.
 * Outputs (caller-allocated; totals from synth_library_totals):
 *   atom_off[L+1], xyz[A*3] (float), type[A] (uint8), bond_off[L+1], bonds[(A-L)*2],
 *   rot_off[L+1], rot_bond[Btot*2] (fixed atom, moving atom), rot_mask[Btot*mask_words].
 * B is clipped to the number of non-terminal edges of the drawn tree;
 * b_actual[L] receives the value used.  Returns 0 or a negative error.
 */
static int ligand_one(uint64_t seed, int l, int n, int breq, int ntypes, double clash_dist,
                      tree_t *T, int *rot_a, int *rot_b, int *nrot, uint8_t *types) {
    for (int attempt = 0; attempt < 64; ++attempt) {
        uint64_t st = stream_init(seed, 0x6c6967616e64ULL /* "ligand" */, (uint64_t)l * 64 + attempt);
        if (!build_tree(T, n, &st, clash_dist)) continue;
        for (int i = 0; i < n; ++i) types[i] = (uint8_t)uint_range(&st, 0, ntypes - 1);
        /* candidate rotatable edges: (parent[c], c) with both degrees >= 2 */
        int ce[SYNTH_MAX_ATOMS], nce = 0;
        for (int c = 1; c < n; ++c)
            if (T->deg[c] >= 2 && T->deg[T->parent[c]] >= 2) ce[nce++] = c;
        int b = breq < nce ? breq : nce;
        /* partial Fisher-Yates */
        for (int i = 0; i < b; ++i) {
            int j = uint_range(&st, i, nce - 1);
            int t = ce[i]; ce[i] = ce[j]; ce[j] = t;
        }
        /* sort chosen by moving atom index */
        for (int i = 1; i < b; ++i) {
            int v = ce[i], j = i - 1;
            while (j >= 0 && ce[j] > v) { ce[j + 1] = ce[j]; --j; }
            ce[j + 1] = v;
        }
        for (int i = 0; i < b; ++i) { rot_a[i] = T->parent[ce[i]]; rot_b[i] = ce[i]; }
        *nrot = b;
        return 0;
    }
    return -3;
}

int synth_library(uint64_t seed, int L, const int32_t *n_atoms, const int32_t *n_rot, int ntypes,
                  double clash_dist, int mask_words, int32_t *atom_off, float *xyz, uint8_t *type,
                  int32_t *bond_off, int32_t *bonds, int32_t *rot_off, int32_t *rot_bond,
                  uint64_t *rot_mask, int32_t *b_actual) {
    if (ntypes < 1 || ntypes > 255 || mask_words < 1) return -1;
    tree_t *T = (tree_t *)malloc(sizeof(tree_t));
    if (!T) return -2;
    int32_t a = 0, bo = 0, ro = 0;
    atom_off[0] = 0; bond_off[0] = 0; rot_off[0] = 0;
    for (int l = 0; l < L; ++l) {
        int n = n_atoms[l];
        if (n < 1 || n > SYNTH_MAX_ATOMS || n > 64 * mask_words || n_rot[l] < 0 ||
            n_rot[l] > SYNTH_MAX_ROT) { free(T); return -1; }
        int ra[SYNTH_MAX_ROT], rb[SYNTH_MAX_ROT], nr = 0;
        int rc = ligand_one(seed, l, n, n_rot[l], ntypes, clash_dist, T, ra, rb, &nr, type + a);
        if (rc) { free(T); return rc; }
        for (int i = 0; i < n; ++i) {
            xyz[3 * (a + i) + 0] = (float)T->pos[i].x;
            xyz[3 * (a + i) + 1] = (float)T->pos[i].y;
            xyz[3 * (a + i) + 2] = (float)T->pos[i].z;
        }
        for (int c = 1; c < n; ++c) {
            bonds[2 * bo + 0] = T->parent[c];
            bonds[2 * bo + 1] = c;
            ++bo;
        }
        for (int r = 0; r < nr; ++r) {
            rot_bond[2 * ro + 0] = ra[r];
            rot_bond[2 * ro + 1] = rb[r];
            subtree_mask(T, rb[r], rot_mask + (size_t)ro * mask_words, mask_words);
            ++ro;
        }
        b_actual[l] = nr;
        a += n;
        atom_off[l + 1] = a;
        bond_off[l + 1] = bo;
        rot_off[l + 1] = ro;
    }
    free(T);
    return 0;
}

/* Totals for allocation: atoms and an upper bound for rotatable bonds. */
void synth_library_totals(int L, const int32_t *n_atoms, const int32_t *n_rot, int64_t *atoms,
                          int64_t *rot_upper) {
    int64_t a = 0, r = 0;
    for (int l = 0; l < L; ++l) { a += n_atoms[l]; r += n_rot[l]; }
    *atoms = a;
    *rot_upper = r;
}

/* ------------------------------------------------------------------------- */
/* Start orientations: R uniformly distributed unit quaternions (w,x,y,z),
 * Shoemake's method (Graphics Gems III, 1992) from three uniforms. */
int synth_start_quats(uint64_t seed, int R, float *out) {
    uint64_t st = stream_init(seed, 0x7374617274ULL /* "start" */, 0);
    for (int r = 0; r < R; ++r) {
        double u1 = u01(&st), u2 = u01(&st), u3 = u01(&st);
        double s1 = sqrt(1.0 - u1), s2 = sqrt(u1);
        double x = s1 * sin(2 * M_PI * u2), y = s1 * cos(2 * M_PI * u2);
        double z = s2 * sin(2 * M_PI * u3), w = s2 * cos(2 * M_PI * u3);
        out[4 * r + 0] = (float)w;
        out[4 * r + 1] = (float)x;
        out[4 * r + 2] = (float)y;
        out[4 * r + 3] = (float)z;
    }
    return 0;
}
