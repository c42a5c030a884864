// dock_internal.h -- argument blocks shared by the HIP kernels (dock_device.hip)
// and the host runtime (dock_runtime.cpp).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dockgpu {

constexpr int kMaxAtoms = 256;      // 4 slots of 64 lanes
constexpr int kMaxRot = 64;
constexpr int kMaxTorsionSteps = 1024;  // matches DOCK_MAX_TORSION_STEPS
constexpr int kNumBins = 8;         // bin b holds ligands with 32b < n <= 32(b+1)
constexpr int kFarWords = 4;        // far-pair rows: 4 x 64 bits per atom
constexpr uint16_t kTraceNone = 0xFFFFu;
constexpr int kMaxGroups = 8;       // paper buckets: rotatable bonds in groups of 4 (last: 28+)
constexpr int kMaxLists = kNumBins * kMaxGroups;  // work lists (atom bin x bond group)

constexpr int kMaxTopK = 64;        // matches DOCK_MAX_TOP_K
constexpr int kXcds = 8;            // gfx950: workgroups go round-robin to 8 XCDs of 32 CUs
// per list: count, dock_next, select_next, (unused), then one alignment queue per XCD
constexpr int kNumCounters = (4 + kXcds) * kMaxLists;
#ifndef DOCK_ALIGN_J
#define DOCK_ALIGN_J 32
#endif
constexpr int kAlignJ = DOCK_ALIGN_J;  // k_align: y rotations per lane
constexpr int kAlignMaxGroup = 64;  // k_align: restarts per item at most

// The pocket is kept as cell cubes: cube (t,k,j,i) holds, for x = i and then
// x = i+1, the bilinear coefficients (a, b, c, d) of the (y,z) face with corners
// v00 = v(x,j,k), v10 = v(x,j+1,k), v01 = v(x,j,k+1), v11 = v(x,j+1,k+1) of
// type t: a = v00, b = v10 - v00, c = v01 - v00, d = (v11 - v10) - (v01 - v00)
// (32 bytes), so the trilinear cell sits in one cache line and its value is
// two bilinear evaluations and one x interpolation.
struct GridArgs {
    const float4 *cubes;   // [ntypes][nz][ny][nx] cubes, 2 float4 each
    uint32_t ncells;       // ntypes*nx*ny*nz
    uint32_t type_bytes;   // nx*ny*nz*32
    int ntypes, nx, ny, nz;
    float inv_h;
    float ox, oy, oz;      // origin
    float cx, cy, cz;      // grid centre
    float mx, my, mz;      // n-1 per axis
    float m2x, m2y, m2z;   // n-2 per axis
    float fnx, fslab;      // nx and nx*ny as floats
    // Shell atlas (see k_align): per radius band b < nbands, bands[2b] = (y0, z0,
    // rows in y, rows in z), bands[2b+1] = (rows, columns or -1, table bytes,
    // C1: the column at which the band's second chunk starts);
    // blob16[t*nbands + b] = float4 offset of type t's band in `atlas`.
    const float4 *atlas;
    const int4 *bands;
    const int *blob16;
    int nbands;
    float acx, acy, acz;   // grid centre in grid units
};

struct SearchArgs {
    int R, T, P, A, K, final_align, bmin;
    int prune;             // 1: prune the bump check and score only bump-free candidates
    int groups;            // work lists per atom bin: 1, or kMaxGroups (paper buckets)
    float bump2g;          // (bump_dist / spacing)^2, grid units
    float dedup2;          // dedup_rmsd^2, Angstrom^2
    const float4 *smat;    // [R][3] start rotation rows (x,y,z,0)
    const float4 *amat;    // [A*A][3] alignment rotation rows
    const float2 *acs;     // [ceil(A/kAlignJ)*kAlignJ] (cos, sin) of 2 pi k / A
    const float2 *tors;    // [T] (cos, sin) of 2 pi k / T
};

struct LibArgs {
    int L, mask_words;
    long long A_total, Nb_total, Nr_total;
    const int *atom_off;
    const float *xyz;
    const uint8_t *type;
    const int *bond_off;
    const int *bond;
    const int *rot_off;
    const int *rot_bond;
    const unsigned long long *rot_mask;
};

struct WorkArgs {
    unsigned long long *far;  // [A_total][kFarWords]
    int *counters;            // [kNumCounters]: [4][kMaxLists] count, dock_next, select_next,
                              // (unused) of each work list, then [kMaxLists][kXcds] the
                              // alignment queues of each list
    int *bin_list;            // [lists][L] ligands of each work list
    float *rscore;            // [L][R]
    uint16_t *rtrace;         // [R*(L + P*Nr_total)]
    float *acc_pose;          // [A_total*K*3] kept poses (aligned by the final step in place)
    int *sel;                 // [L*K] restart of each kept pose
    int *nsel;                // [L] kept poses
    float *fscore;            // [L*K] final score of each kept pose
    int *fo;                  // [L*K] final-step orientation of each kept pose
    unsigned long long *scored;  // torsion samples scored (measurement; null: not counted)
};

// Pocket atoms of the pairwise rescoring stand-in, sorted into a cell grid whose
// cell edge is at least the contact distance (plus a margin above rounding), so
// every contact pair lies in neighbouring cells.
constexpr int kMaxContactWeights = 1024;  // ligand types x pocket atom types
struct ContactArgs {
    const float4 *atoms;     // [n] (x, y, z, type as int bits), sorted by cell
    const int *cell_start;   // [cx*cy*cz + 1] first atom of each cell (x fastest)
    const int *weight;       // [ligand types][ntypes]
    int ntypes, nw;          // pocket atom types; weight entries
    int cx, cy, cz;          // cells per axis
    float lox, loy, loz;     // corner of cell (0,0,0)
    float inv_cell;          // 1 / cell edge
    float dc2;               // contact distance squared
};

struct OutArgs {
    float *best;
    int *npose;
    int *status;
    float *pscore;
    int *prestart;
    float *pxyz;
    float *rscore_user;       // optional copy of restart scores
    uint16_t *ftrace;         // optional
    int *pcontacts;           // optional: contact score of each output pose
};

// Shared-memory bytes of the docking kernel for a bin with at most nmax atoms
// and `waves` wavefronts per workgroup.
size_t dock_lds_bytes(int nmax, int waves);
size_t select_lds_bytes(int nmax, int waves, int R, int K, int sel_lds);
// Whether k_select keeps candidate and kept poses in LDS (parallel selection).
int select_sel_lds(int nmax, int waves, int R, int K);
size_t falign_lds_bytes(int nmax, int waves, int single);

// Launchers (return hipError_t of the launch).
hipError_t launch_build_cubes(const float *values, float4 *cubes, int ntypes, int nx, int ny,
                              int nz, hipStream_t s);
// Zero work-queue counters [first, first + count), within [0, kNumCounters).
hipError_t launch_reset(int *counters, int first, int count, hipStream_t s);
hipError_t launch_prep(const GridArgs &g, const SearchArgs &sa, const LibArgs &lib,
                       const WorkArgs &ws, const OutArgs &out, hipStream_t s);
// Stage launches over work list `lst` of atom bin `bin` (lst = bin with one list
// per bin, bin * kMaxGroups + group with the paper buckets).
hipError_t launch_dock(int bin, int lst, int blocks, int waves, const GridArgs &g,
                       const SearchArgs &sa, const LibArgs &lib, const WorkArgs &ws, hipStream_t s);
// Shell atlas of a pocket: pass 1 writes the geometry of kMaxBands bands into
// info[2*kMaxBands]; pass 2 fills nb bands of every type.
constexpr int kMaxBands = 240;
// Atlas bands occupy whole 64-float4 blocks (the alignment kernel copies them
// with one 16-byte load per lane).
__host__ __device__ inline int band_padded(int size16) { return (size16 + 63) & ~63; }
hipError_t launch_atlas_count(const GridArgs &g, int4 *info, hipStream_t s);
hipError_t launch_atlas_fill(const GridArgs &g, int4 *info, const int *blob16, float4 *atlas,
                             int nb, hipStream_t s);
// Batched alignment of a bin's ligands (k_align), `arena` bytes of LDS per
// workgroup.
hipError_t launch_align(int bin, int lst, int blocks, int arena, const GridArgs &g,
                        const SearchArgs &sa, const LibArgs &lib, const WorkArgs &ws,
                        hipStream_t s);
// Smallest arena k_align accepts for the bin (fixed part plus a minimal region).
size_t align_lds_min(int bin, int A, int R);
int align_blocks_per_cu(int bin, int R, int A, int arena);
// Final stage of a bin.  single >= 0: only that ligand (plain form; k_falign then
// runs one workgroup per kept pose), else the bin's queue.
hipError_t launch_select(int bin, int lst, int blocks, int waves, const GridArgs &g,
                         const SearchArgs &sa, const LibArgs &lib, const WorkArgs &ws,
                         const OutArgs &out, int single, hipStream_t s);
// xcds > 1: the bin's ligands are split into that many contiguous shares, share x
// taken by workgroups b with b % xcds == x (the XCD they are dispatched to).
hipError_t launch_falign(int bin, int lst, int blocks, int waves, const GridArgs &g,
                         const SearchArgs &sa, const LibArgs &lib, const WorkArgs &ws,
                         const OutArgs &out, int single, int xcds, hipStream_t s);
hipError_t launch_out(int bin, int lst, int blocks, const SearchArgs &sa, const LibArgs &lib,
                      const WorkArgs &ws, const OutArgs &out, int single, hipStream_t s);
// Contact score (pairwise rescoring stand-in) of every output pose: single >= 0:
// ligand `single` only, one workgroup per pose (grid top_k); else every ligand,
// one wave per (ligand, pose) over `blocks` workgroups.
hipError_t launch_rescore(const ContactArgs &ca, const SearchArgs &sa, const LibArgs &lib,
                          const OutArgs &out, int single, int blocks, hipStream_t s);
// Plain form: checks of ligand l only (no size binning), and its restarts
// (grid = R workgroups of `waves` waves).
hipError_t launch_prep_one(const GridArgs &g, const SearchArgs &sa, const LibArgs &lib,
                           const WorkArgs &ws, const OutArgs &out, int l, hipStream_t s);
hipError_t launch_plain(int l, int bin, int waves, const GridArgs &g, const SearchArgs &sa,
                        const LibArgs &lib, const WorkArgs &ws, const OutArgs &out,
                        hipStream_t s);
size_t plain_lds_bytes(int nmax, int waves);
// Max resident workgroups per CU for a launch shape (occupancy API).
int dock_blocks_per_cu(int bin, int waves, int T);
int select_blocks_per_cu(int bin, int waves, int R, int K);
int falign_blocks_per_cu(int bin, int waves);

}  // namespace dockgpu
