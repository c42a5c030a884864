/*
 * dock.h -- C ABI of the MI355X (gfx950) geometric-docking library.
 *
 * The library docks ligands into a rigid pocket with the greedy multi-restart
 * method of Alg. 1 in Vitali et al., "GPU-optimized Approaches to Molecular
 * Docking-based Virtual Screening in Drug Discovery: A Comparative Analysis"
 * (arXiv:2209.05069), Section "Application Description":
 *   for each ligand and each restart r:
 *     Generate_Starting_Pose: the ligand, centred on its centroid, is turned by
 *       the r-th start orientation and placed at the grid centre;
 *     Alignment (rigid rotation): of the A*A orientations R_y(2 pi j/A) R_x(2 pi i/A)
 *       about the pose centroid the best-scoring one is applied
 *       (orientation index o = i*A + j; the first maximum wins);
 *     Optimize Pose: for sweep_passes passes, for each rotatable bond in the
 *       given order, of the torsion_steps rotations by 2 pi k/T of the bond's
 *       moving fragment about the bond axis, those with an intramolecular bump
 *       are rejected and the best-scoring remaining one is applied (the first
 *       maximum wins; k = 0 keeps the conformation);
 *   Select Poses: restarts by score (ties: lower restart), a pose is kept unless
 *     its plain RMSD to an already kept pose is below dedup_rmsd, at most top_k;
 *   final step: the alignment again on each kept pose (if final_align), then its
 *     score; outputs ordered by final score (ties: lower restart).
 * Score of a pose = sum over atoms of the trilinearly interpolated score grid of
 * the atom's type (grid coordinates clamped to the box); higher is better.
 * Bump = a pair with one atom moving and one not, at least bump_min_bonds bonds
 * apart, closer than bump_dist.
 * The paper's chemical rescoring (Rescore Pose) is not part of this library: its
 * function is not given in the paper; the final step above stands in for it.
 *
 * All entry points return a dock_status value and never throw.  On failure,
 * dock_last_error() returns a message for the calling thread.
 * A context is bound to one device.  Its entry points may be called from
 * several host threads; calls that use the same stream are serialised by that
 * stream, and each stream gets its own workspace.
 */
#ifndef DOCK_H
#define DOCK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dock_ctx dock_ctx;

typedef enum {
    DOCK_OK = 0,
    DOCK_EINVAL = -1,   /* bad argument (message says which) */
    DOCK_ENOMEM = -2,   /* device or host allocation failed */
    DOCK_EAGAIN = -3,   /* dock_submit: not enough free device memory now; retry later */
    DOCK_ENOENT = -4,   /* unknown pocket id or ticket */
    DOCK_EDEVICE = -5,  /* HIP runtime error (message has the HIP error string) */
    DOCK_EBUSY = -6     /* pocket still used by submitted work */
} dock_status;

/* Per-ligand status written to dock_results.status.  A ligand that fails a
 * check is not docked; its outputs are n_poses = 0 and best_score = -inf. */
typedef enum {
    DOCK_LIG_OK = 0,
    DOCK_LIG_BAD_SIZE = 1,   /* atoms not in [1, DOCK_MAX_ATOMS], rotatable bonds > DOCK_MAX_ROT,
                                or bonds > 8 * atoms */
    DOCK_LIG_BAD_TYPE = 2,   /* atom type >= pocket ntypes */
    DOCK_LIG_BAD_BOND = 3,   /* bond or rotatable bond atom index out of range / self bond */
    DOCK_LIG_BAD_MASK = 4,   /* moving mask is not the fragment the bond cuts off, or the bond
                                is in a ring, or the ligand is not connected */
    DOCK_LIG_BAD_OFFSETS = 5 /* CSR offsets decreasing or past the declared totals */
} dock_ligand_status;

#define DOCK_MAX_ATOMS 256
#define DOCK_MAX_ROT 64
#define DOCK_MAX_TORSION_STEPS 1024
#define DOCK_MAX_ALIGN_STEPS 255
#define DOCK_MAX_TOP_K 64
#define DOCK_TRACE_NONE 0xFFFFu /* torsion decision where every candidate bumped */

/* Create a context on HIP device `device` (its index as hipSetDevice takes it).
 * hbm_budget_bytes bounds the device memory the context's dock_submit work may
 * hold at once (library copies, results and workspaces of requests not yet
 * retired by dock_poll/dock_wait, plus the per-stream workspaces kept between
 * requests); 0 = no fixed budget, admit against the device's free memory less
 * a 1 GiB reserve.  (The paper's batched form sizes its batches from the memory
 * and occupancy of the GPU; Batched Implementation subsection.) */
int dock_create(int device, uint64_t hbm_budget_bytes, dock_ctx **out);
/* Wait for all submitted work, free every device buffer of the context. */
int dock_destroy(dock_ctx *ctx);
/* Message of the calling thread's last failure ("" if none).  Valid until the
 * thread's next call into the library. */
const char *dock_last_error(void);

/* Pocket score grids (paper: the pocket is read-only and shared by all work on a
 * GPU; Latency Implementation subsection).  Grid point (i,j,k) of type t holds
 * values[((t*nz + k)*ny + j)*nx + i] at position origin + spacing*(i,j,k), Angstrom.
 * Requires ntypes in [1,255], nx,ny,nz >= 2, spacing > 0, nx*ny*nz < 2^24 and
 * all grids together under 4 GiB.
 * `values` is host memory; it is copied before the call returns. */
typedef struct {
    int32_t ntypes, nx, ny, nz;
    float spacing;
    float origin[3];
    const float *values;
} dock_grid_desc;

int dock_pocket_load(dock_ctx *ctx, const dock_grid_desc *grid, int32_t *pocket_id);
/* DOCK_EBUSY while dock_submit work that uses the pocket is not finished. */
int dock_pocket_unload(dock_ctx *ctx, int32_t pocket_id);

/* Pocket atoms for the pairwise rescoring stand-in.  The paper's Rescore Pose
 * evaluates every ligand atom against every pocket atom and accumulates the pair
 * terms per pose (Rescore Pose subsections of the latency and batched
 * implementations); its chemical terms are not given, so here the contact score
 * of a pose is the sum over ligand atoms i and pocket atoms j with
 * |x_i - p_j| < contact_dist of weight[type_i * ntypes + type_j] (type_i: the
 * ligand atom's grid type; an integer).  Host memory, copied before the call
 * returns; replaces the pocket's previous atom list.  Requires ntypes in
 * [1,255], types < ntypes, finite coordinates, 0 < contact_dist <= 1000 and
 * (grid ntypes) * ntypes <= 1024.  DOCK_EBUSY while dock_submit work that uses
 * the pocket is not finished; waits for the device's other work. */
typedef struct {
    int32_t n_atoms;
    int32_t ntypes;            /* pocket atom types */
    float contact_dist;        /* Angstrom */
    const float *xyz;          /* [n_atoms][3], the grid's frame, Angstrom */
    const uint8_t *type;       /* [n_atoms] */
    const int32_t *weight;     /* [grid ntypes][ntypes] */
} dock_pocket_atoms;

int dock_pocket_set_atoms(dock_ctx *ctx, int32_t pocket_id, const dock_pocket_atoms *atoms);

/* Ligand library in CSR form (paper: coordinates, atom types and the fragments
 * of the rotatable bonds; Batched Implementation subsection).  Ligand l owns
 * atoms [atom_off[l], atom_off[l+1]), bonds [bond_off[l], bond_off[l+1]) and
 * rotatable bonds [rot_off[l], rot_off[l+1]); atom indices inside bonds are
 * local to the ligand.  rot_bond[r] = (a, b): a stays, b moves; the sweep visits
 * the rotatable bonds in this order.  rot_mask[r*mask_words + w] bit i (i = 64w +
 * bit) is set when atom i moves with bond r (the fragment on b's side).
 * For dock_ligands_batch every pointer is DEVICE memory; for dock_submit every
 * pointer is HOST memory.  The totals are host values and must equal
 * atom_off[L], bond_off[L] and rot_off[L]. */
typedef struct {
    int32_t n_ligands;
    int32_t mask_words;        /* >= ceil(max atoms / 64), <= 4 */
    int64_t n_atoms_total;
    int64_t n_bonds_total;
    int64_t n_rot_total;
    const int32_t *atom_off;   /* [n_ligands+1] */
    const float *xyz;          /* [n_atoms_total][3], Angstrom, any frame */
    const uint8_t *type;       /* [n_atoms_total] */
    const int32_t *bond_off;   /* [n_ligands+1] */
    const int32_t *bond;       /* [n_bonds_total][2] */
    const int32_t *rot_off;    /* [n_ligands+1] */
    const int32_t *rot_bond;   /* [n_rot_total][2] */
    const uint64_t *rot_mask;  /* [n_rot_total][mask_words] */
} dock_library;

enum { DOCK_MODE_BATCHED = 0, DOCK_MODE_PLAIN = 1 };

/* Search settings.  start_quat is HOST memory, [restarts][4] quaternions
 * (w,x,y,z) (normalised by the library), copied during the call; restart r
 * of every ligand starts from orientation r.
 * mode: DOCK_MODE_BATCHED docks many ligands per launch (one wavefront per
 * (ligand, restart)); DOCK_MODE_PLAIN docks one ligand per launch sequence,
 * spreading that ligand over the whole GPU (the paper's latency form). */
typedef struct {
    int32_t restarts;          /* R in [1, 4096] */
    int32_t torsion_steps;     /* T in [1, DOCK_MAX_TORSION_STEPS] */
    int32_t sweep_passes;      /* P in [0, 16] */
    int32_t align_steps;       /* A in [1, DOCK_MAX_ALIGN_STEPS] */
    int32_t top_k;             /* K in [1, DOCK_MAX_TOP_K] */
    int32_t final_align;       /* 0 or 1 */
    int32_t bump_min_bonds;    /* >= 1; pairs closer in bonds are never checked */
    int32_t mode;              /* DOCK_MODE_* */
    int32_t bump_prune;        /* 1: prune the Bump Check (pairs that cannot come within
                                  bump_dist for any angle are skipped, and only
                                  candidates that pass it are scored); 0: no pruning,
                                  every eligible pair is tested against every candidate
                                  and every candidate is scored, the bump verdict applied
                                  afterwards.  The selected steps are the same either
                                  way; 0 is the no-early-exit ablation of the paper's
                                  workload analysis (Execution Profiling). */
    int32_t bin_mode;          /* batched form's work lists: 0 = one per size bin of 32
                                  heavy atoms; 1 = the paper's buckets (Batched
                                  Implementation): size bin x group of 4 rotatable
                                  bonds (0-3, 4-7, ..., 28 and more), a launch per
                                  bucket.  Results are the same either way. */
    float bump_dist;           /* Angstrom, >= 0 */
    float dedup_rmsd;          /* Angstrom, >= 0 (0: plain top-K) */
    const float *start_quat;   /* HOST [restarts][4] */
} dock_params;

/* Outputs.  Same memory kind as the library (device for dock_ligands_batch,
 * host for dock_submit).  Required: best_score, n_poses, status, pose_score,
 * pose_restart.  Optional (NULL to skip): pose_xyz (required with
 * pose_contacts), restart_score, trace, final_trace, pose_contacts.  Skipping
 * pose_xyz changes nothing else (a screening service that keeps only scores
 * saves its A*K*12 bytes of transfer per request).
 *   pose_score[l*K + s], pose_restart[l*K + s], final_trace[l*K + s] for the
 *     s-th output pose (s < n_poses[l]; later slots get -inf / -1 / 0);
 *   pose_xyz: ligand l's pose s starts at float index 3*(atom_off[l]*K + s*n_l)
 *     (slots s >= n_poses[l] are zero);
 *   restart_score[l*R + r]: score of restart r after its sweeps;
 *   trace: decisions of every restart, ligand l's block starts at
 *     R*(l + P*rot_off[l]) and holds, per restart, 1 + P*B_l entries: the
 *     alignment index o, then the applied torsion step of each decision
 *     (DOCK_TRACE_NONE when every candidate bumped);
 *   final_trace[l*K + s]: alignment index of the final step (0 if final_align=0);
 *   pose_contacts[l*K + s]: contact score of output pose s against the pocket's
 *     atoms (dock_pocket_set_atoms; the call fails with DOCK_EINVAL when the
 *     pocket has none); 0 for slots s >= n_poses[l].
 * For a ligand whose status is not DOCK_LIG_OK only best_score (-inf), n_poses
 * (0), status, pose_score (-inf), pose_restart (-1) and final_trace (0) are
 * written (and pose_contacts, 0); its pose_xyz, restart_score and trace entries
 * are left as they were. */
typedef struct {
    float *best_score;        /* [L] */
    int32_t *n_poses;         /* [L] */
    int32_t *status;          /* [L] dock_ligand_status */
    float *pose_score;        /* [L*K] */
    int32_t *pose_restart;    /* [L*K] */
    float *pose_xyz;          /* [n_atoms_total*K*3] or NULL */
    float *restart_score;     /* [L*R] or NULL */
    uint16_t *trace;          /* [R*(L + P*n_rot_total)] or NULL */
    uint16_t *final_trace;    /* [L*K] or NULL */
    int32_t *pose_contacts;   /* [L*K] or NULL */
} dock_results;

/* Dock a device-resident library; all work is enqueued on `stream` (a
 * hipStream_t, NULL = the null stream) and the call returns after enqueueing.
 * Results are valid once the stream reaches this point.  The library and the
 * results must stay allocated until then.  Internal workspace is allocated on
 * first use and kept per stream; growing it waits for that stream. */
int dock_ligands_batch(dock_ctx *ctx, int32_t pocket, const dock_library *lib,
                       const dock_params *params, dock_results *out, void *stream);

/* Size of the device scratch array behind dock_ligands_batch_noalloc: 64 MiB,
 * held on each device the library runs on until the process ends. */
#define DOCK_NOALLOC_SCRATCH_BYTES (64u << 20)

/* dock_ligands_batch for callers that cannot allocate device memory (code that
 * runs under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments, kernels and results as dock_ligands_batch with
 * mode DOCK_MODE_BATCHED, but its tables and workspace live in a fixed
 * per-device scratch array of DOCK_NOALLOC_SCRATCH_BYTES, so the call allocates
 * no device memory, captures no graph and records no phase timing.  It enqueues
 * on `stream` one host-to-device copy of its tables (from host memory the
 * context keeps) and the kernels.
 * Limits: DOCK_EINVAL (nothing enqueued) when mode is not DOCK_MODE_BATCHED or
 * when the request needs more scratch than DOCK_NOALLOC_SCRATCH_BYTES: the
 * tables (16*3R B of start rotations, 16*3A^2 B of alignment rotations, 8*T B
 * of torsion (cos, sin), 8*(A rounded up to 32) B of alignment (cos, sin)) plus
 * the workspace (per atom 32 B of bump-pair rows and 12*top_k B of kept poses;
 * per ligand 4*R B of restart scores, 32 B of work lists (256 B with bin_mode 1)
 * and 12*top_k + 4 B of selection records; 3 KiB of counters;
 * and, when out->trace is NULL, 2*R*(L + P*n_rot_total) B of decision trace),
 * each part rounded up to a multiple of 256 B.
 * Every call on a device shares that device's array and leaves its contents
 * there: calls that overlap on one device (different streams or contexts) race
 * and give wrong results; calls on one stream are ordered by it.  The array's
 * counters are cleared by the call's own first kernel. */
int dock_ligands_batch_noalloc(dock_ctx *ctx, int32_t pocket, const dock_library *lib,
                               const dock_params *params, dock_results *out, void *stream);

/* Asynchronous form on host memory (paper: the batched form's asynchronous
 * interface, Batched Implementation subsection).  The library and params are
 * copied before the call returns; `out` must stay valid until dock_poll reports
 * done (or dock_wait returns).  Admission: DOCK_EAGAIN when the request's device
 * memory does not fit in the context's budget (see dock_create) next to the work
 * already admitted, or, without a budget, in the device memory left free (less
 * a reserve); nothing is enqueued then: retry after polling. */
int dock_submit(dock_ctx *ctx, int32_t pocket, const dock_library *lib,
                const dock_params *params, dock_results *out, uint64_t *ticket);
/* Device bytes a dock_submit of this request needs on a stream that holds no
 * workspace yet: the copies of the library and the results, held until the
 * ticket retires, plus the docking workspace; the figure the admission check
 * compares with the budget.  Reads only the sizes in lib, params and which
 * optional outputs of out are requested (no device work, no context). */
int dock_request_bytes(const dock_library *lib, const dock_params *params,
                       const dock_results *out, uint64_t *bytes);
/* *done = 1 once the results of `ticket` are in `out` (the ticket is then
 * retired; polling it again gives DOCK_ENOENT). */
int dock_poll(dock_ctx *ctx, uint64_t ticket, int32_t *done);
/* Block until `ticket` is done, then retire it. */
int dock_wait(dock_ctx *ctx, uint64_t ticket);

/* Per-bin autotuning of the batched form's tiles (paper: the batched form sizes
 * its launches per size bucket from the GPU's occupancy; Batched Implementation
 * subsection).  Size bin b holds the ligands with 32b < atoms <= 32(b+1).  For
 * each bin the sample has ligands in, dock_autotune docks the sample once,
 * then times the torsion-sweep kernel with 2, 4 and 8 restarts (waves) per
 * workgroup, the pose-selection kernel with 4, 8 and 16 waves per workgroup,
 * and the final-alignment kernel with 2, 4 and 8 waves per workgroup at 1, 2,
 * 4 or all workgroups per CU that fit, with and without the per-XCD split of
 * the ligands, each the best of two runs on `stream`;
 * the fastest tile of each kernel is kept by the context for these search
 * settings (restarts, torsion_steps, align_steps, top_k, sweep_passes) and used
 * by every later batched call with them (results do not depend on the tiles).
 * `sample` is device memory, as for dock_ligands_batch; `out` (NULL to skip)
 * receives DOCK_NUM_BINS entries.  The call allocates its own result buffers,
 * waits for `stream` and returns when done. */
#define DOCK_NUM_BINS 8
typedef struct {
    int32_t ligands;         /* ligands of the sample in the bin (0: not tuned) */
    int32_t dock_waves;      /* torsion sweep: restarts (waves) per workgroup */
    int32_t select_waves;    /* pose selection: waves per workgroup */
    int32_t falign_waves;    /* final alignment: waves per workgroup */
    int32_t falign_per_cu;   /* final alignment: workgroups per CU (0: all that fit) */
    int32_t falign_xcd;      /* final alignment: 1 = the ligands are split into 8 contiguous
                                shares, one per XCD (workgroups go round-robin to the
                                8 XCDs), so a ligand's kept poses share one L2; 0 = the
                                grid's waves take (ligand, pose) items in turn */
    float dock_ms, select_ms, falign_ms;  /* the chosen tiles on the sample */
    float dock_ms_default, select_ms_default, falign_ms_default;  /* the default tiles
                                                (4, 4, 4 waves, all that fit) */
} dock_bin_tuning;

int dock_autotune(dock_ctx *ctx, int32_t pocket, const dock_library *sample,
                  const dock_params *params, dock_bin_tuning *out, void *stream);
/* Set the tiles used for these search settings from `table` (DOCK_NUM_BINS
 * entries; entries with ligands = 0 keep the defaults), e.g. a table saved from
 * an earlier dock_autotune on the same device; NULL restores the defaults. */
int dock_set_tuning(dock_ctx *ctx, const dock_params *params, const dock_bin_tuning *table);

/* Phase timing, for measurement.  While enabled, every dock_ligands_batch
 * call records HIP events on its own stream before its prep kernel, after it,
 * after the alignment kernels (batched form), after the docking kernels and
 * after the select/final kernels.
 * dock_get_timing waits for every recorded event, returns the summed
 * milliseconds of each phase, the number of calls and the number of torsion
 * samples the docking kernels scored since the last dock_get_timing, and starts
 * a new sum.  A torsion sample is one moving atom of one bump-free candidate
 * angle: as in Alg. 1 (Optimize Pose), a candidate that fails the Bump Check is
 * not scored. */
typedef struct {
    double prep_ms;   /* ligand checks, bump-pair rows, size binning */
    double dock_ms;   /* restarts: start pose, alignment, torsion sweeps */
    double align_ms;  /* the alignment kernels' part of dock_ms (batched form; 0 in the
                         plain form, whose restart kernel also aligns) */
    double final_ms;  /* pose selection, final rigid step, outputs */
    int64_t calls;
    int64_t scored_samples;  /* torsion samples scored in the docking phase */
} dock_timing;

int dock_set_timing(dock_ctx *ctx, int enable);
int dock_get_timing(dock_ctx *ctx, dock_timing *out);

#ifdef __cplusplus
}
#endif
#endif /* DOCK_H */
