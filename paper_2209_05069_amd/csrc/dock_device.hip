// dock_device.hip -- gfx950 kernels of the geometric-docking hot path.
//
// Method: Alg. 1 of arXiv:2209.05069 (Application Description).  One
// wavefront docks one (ligand, restart): Generate_Starting_Pose, the A*A rigid
// alignment and the greedy torsion sweep (Optimize Pose).  A second kernel does
// Select Poses and the final rigid step per ligand.  Mapping choices for CDNA4:
//  * lanes hold atoms (atom i = lane + 64*slot) for every per-atom update, so a
//    pose lives in registers; a wave-uniform atom is fetched with readlane;
//  * the alignment spreads the A*A orientations over the 64 lanes, and the
//    torsion step spreads the T candidates over the lanes (T/64 per lane); each
//    lane scores its candidates over the moving atoms, whose rotation frames
//    sit once per wave in LDS (broadcast reads);
//  * only the moving fragment's score changes with the torsion angle, so the
//    candidates are ranked by that partial sum (same argmax as the full score);
//  * bump check in closed form: turning a moving atom about the bond axis makes
//    its squared distance to a static atom C + A cos(theta) + B sin(theta), so
//    lanes over static atoms compute (C, A, B) per pair, drop pairs whose
//    closest approach stays above the bump distance (ballot), and test the few
//    remaining pairs against every candidate with two FMAs; one 64-bit key max
//    (order-preserving score bits, then the lower index) over the bump-free
//    candidates picks the step;
//  * grid gathers are raw buffer loads of cell cubes (a cell's trilinear
//    coefficients in one 32-byte record): two 16-byte loads from one cache line
//    per sample, a 32-bit voffset for the cell and the atom type as scalar offset,
//    with the range checked by hardware;
//  * a persistent grid pops (ligand, restart-group) items from a per-bin queue;
//    the ligand's coordinates, bump-pair rows and masks are staged once per
//    item in LDS and shared by the workgroup's waves.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dock_internal.h"

namespace dockgpu {

typedef unsigned long long u64;

// ---------------------------------------------------------------------------
// wavefront helpers
__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Whole-wave reductions with DPP: row_shr 1, 2, 4, 8 leave in lane 15 of every
// 16-lane row the reduction of its row; row_bcast 15 and 31 carry the rows into
// lane 63, whose value is then read by every lane.  Lanes outside a shift read 0,
// the identity of the sum, the max of unsigned keys and the or.  Call with the
// whole wave active.
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_read(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWS, 0xF, true);
}

template <int CTRL, int ROWS>
__device__ __forceinline__ u64 dpp_read64(u64 v) {
    const uint32_t lo = (uint32_t)dpp_read<CTRL, ROWS>((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)dpp_read<CTRL, ROWS>((int)(uint32_t)(v >> 32));
    return ((u64)hi << 32) | lo;
}

__device__ __forceinline__ u64 read_lane64(u64 v, int lane) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
    return ((u64)hi << 32) | lo;
}

#define DOCK_DPP_STEPS(STEP) \
    STEP(0x111, 0xF) STEP(0x112, 0xF) STEP(0x114, 0xF) STEP(0x118, 0xF) STEP(0x142, 0xA) STEP(0x143, 0xC)

__device__ __forceinline__ float wave_sum(float v) {
#define DOCK_SUM_STEP(C, R) v += __int_as_float(dpp_read<C, R>(__float_as_int(v)));
    DOCK_DPP_STEPS(DOCK_SUM_STEP)
#undef DOCK_SUM_STEP
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

__device__ __forceinline__ u64 wave_max_u64(u64 v) {
#define DOCK_MAX_STEP(C, R)                 \
    {                                       \
        const u64 w = dpp_read64<C, R>(v);  \
        v = w > v ? w : v;                  \
    }
    DOCK_DPP_STEPS(DOCK_MAX_STEP)
#undef DOCK_MAX_STEP
    return read_lane64(v, 63);
}

__device__ __forceinline__ u64 wave_or_u64(u64 v) {
#define DOCK_OR_STEP(C, R) v |= dpp_read64<C, R>(v);
    DOCK_DPP_STEPS(DOCK_OR_STEP)
#undef DOCK_OR_STEP
    return read_lane64(v, 63);
}
#undef DOCK_DPP_STEPS

__device__ __forceinline__ int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ float read_lane(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// Order-preserving map of a float to uint32 (larger float -> larger integer).
__device__ __forceinline__ uint32_t ord_f32(float f) {
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float unord_f32(uint32_t u) {
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}
// Key of (score, index): the max key has the best score, then the lowest index.
__device__ __forceinline__ u64 make_key(float s, uint32_t idx) {
    return ((u64)ord_f32(s) << 32) | (u64)(0xFFFFFFFFu - idx);
}
__device__ __forceinline__ uint32_t key_index(u64 k) { return 0xFFFFFFFFu - (uint32_t)k; }
__device__ __forceinline__ float key_score(u64 k) { return unord_f32((uint32_t)(k >> 32)); }

// Make LDS writes of this wave visible to its own later LDS reads by other lanes.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------
// Trilinear interpolation.  (gx,gy,gz) are grid coordinates ((p - origin)/h);
// each is clamped to [0, n-1], the cell corner is min(floor, n-2).  The pocket
// is stored as cell cubes (see GridArgs): the two x-vertex columns of a cell,
// each as the bilinear coefficients of its (y,z) face, are one 32-byte record,
// read as two 16-byte loads from the same cache line.
// toff is the byte offset of the atom type's block.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

struct Tri {
    __amdgpu_buffer_rsrc_t rs;
    float mx, my, mz, m2x, m2y, m2z, fnx, fslab;
    uint32_t nx, slab;  // cells per row and per slab
};

__device__ __forceinline__ Tri make_tri(const GridArgs &g) {
    Tri t;
    t.rs = __builtin_amdgcn_make_buffer_rsrc((void *)g.cubes, (short)0,
                                             (int)(g.ncells * 32u), 0x00020000);
    t.mx = g.mx; t.my = g.my; t.mz = g.mz;
    t.m2x = g.m2x; t.m2y = g.m2y; t.m2z = g.m2z;
    t.fnx = g.fnx; t.fslab = g.fslab;
    t.nx = (uint32_t)g.nx;
    t.slab = (uint32_t)g.nx * (uint32_t)g.ny;
    return t;
}

// byte offset of the cell record within the type block, and the fractions
__device__ __forceinline__ uint32_t tri_cell(const Tri &t, float gx, float gy, float gz, float &fx,
                                             float &fy, float &fz) {
    const float cx = __builtin_amdgcn_fmed3f(gx, 0.0f, t.mx);
    const float cy = __builtin_amdgcn_fmed3f(gy, 0.0f, t.my);
    const float cz = __builtin_amdgcn_fmed3f(gz, 0.0f, t.mz);
    const float ix = floorf(__builtin_amdgcn_fmed3f(gx, 0.0f, t.m2x));
    const float iy = floorf(__builtin_amdgcn_fmed3f(gy, 0.0f, t.m2y));
    const float iz = floorf(__builtin_amdgcn_fmed3f(gz, 0.0f, t.m2z));
    fx = cx - ix;
    fy = cy - iy;
    fz = cz - iz;
    // element index < 2^24: exact in float
    const float e = fmaf(iz, t.fslab, fmaf(iy, t.fnx, ix));
    return ((uint32_t)e) << 5;
}

// 16-byte raw buffer load; the builtin returns the bits as integers.
__device__ __forceinline__ float4 ldq(__amdgpu_buffer_rsrc_t rs, uint32_t voff, int soff) {
    const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)voff, soff, 0);
    return make_float4(__uint_as_float(v.x), __uint_as_float(v.y), __uint_as_float(v.z),
                       __uint_as_float(v.w));
}

// Bilinear (y,z) form of one x-vertex column: q = (a, b, c, d) with
// v(fy,fz) = a + b*fy + c*fz + d*fy*fz.
__device__ __forceinline__ float col_bilin(const float4 q, float fy, float fz) {
    return fmaf(fz, fmaf(fy, q.w, q.z), fmaf(fy, q.y, q.x));
}

// q0, q1: the columns at x vertices i and i+1; the x interpolation comes last.
__device__ __forceinline__ float tri_blend(const float4 q0, const float4 q1, float fx, float fy,
                                           float fz) {
    const float b0 = col_bilin(q0, fy, fz), b1 = col_bilin(q1, fy, fz);
    return fmaf(fx, b1 - b0, b0);
}

// wave-uniform type offset (scalar offsets)
__device__ __forceinline__ float tri_u(const Tri &t, float gx, float gy, float gz, int toff) {
    float fx, fy, fz;
    const uint32_t off = tri_cell(t, gx, gy, gz, fx, fy, fz);
    const float4 q0 = ldq(t.rs, off, toff);
    const float4 q1 = ldq(t.rs, off, toff + 16);
    return tri_blend(q0, q1, fx, fy, fz);
}

// per-lane type offset
__device__ __forceinline__ float tri_v(const Tri &t, float gx, float gy, float gz, uint32_t toff) {
    float fx, fy, fz;
    const uint32_t off = tri_cell(t, gx, gy, gz, fx, fy, fz) + toff;
    const float4 q0 = ldq(t.rs, off, 0);
    const float4 q1 = ldq(t.rs, off, 16);
    return tri_blend(q0, q1, fx, fy, fz);
}

// Samples known to lie in [0, n-2] on every axis: the clamps of tri_u are then
// the identity, floor is truncation and the fraction is exact as v_fract, so
// this returns the same value with fewer instructions.
// Byte offset of the cube of a sample in [0, n-2] on every axis: truncation is
// floor there, and cell indices and sizes fit the 24-bit multipliers.
__device__ __forceinline__ uint32_t in_cell(const Tri &t, float gx, float gy, float gz) {
    return (__umul24((uint32_t)gz, t.slab) + __umul24((uint32_t)gy, t.nx) + (uint32_t)gx) << 5;
}
constexpr float kInsideMargin = 0.5f;  // grid cells, far above FP32 rounding of coordinates
__device__ __forceinline__ float tri_in(const Tri &t, float gx, float gy, float gz, int toff) {
    const float fx = __builtin_amdgcn_fractf(gx), fy = __builtin_amdgcn_fractf(gy),
                fz = __builtin_amdgcn_fractf(gz);
    const uint32_t off = in_cell(t, gx, gy, gz);
    const float4 q0 = ldq(t.rs, off, toff);
    const float4 q1 = ldq(t.rs, off, toff + 16);
    return tri_blend(q0, q1, fx, fy, fz);
}

// Flag of a listed torsion candidate that bumps (see score_free).
constexpr int kCandBumped = 0x8000;

// Radius for ball_inside from its square: the hardware square root (about one
// ulp).  Only the choice between tri_in and tri_u depends on it, the two give the
// same value inside [0, n-2], and kInsideMargin dwarfs the error.
__device__ __forceinline__ float ball_radius(float r2) { return __builtin_amdgcn_sqrtf(r2); }

// Whether the ball of radius rad (grid units) about (cx,cy,cz), widened by
// kInsideMargin, stays inside [0, n-2] on every axis.
__device__ __forceinline__ bool ball_inside(const Tri &t, float cx, float cy, float cz, float rad) {
    const float r = rad + kInsideMargin;
    return cx - r >= 0.0f && cy - r >= 0.0f && cz - r >= 0.0f && cx + r <= t.m2x &&
           cy + r <= t.m2y && cz + r <= t.m2z;
}

// Bilinear coefficients of the (y,z) face at x vertex i of cell (j,k): from
// its corners v00 = v(i,j,k), v10 = v(i,j+1,k), v01 = v(i,j,k+1),
// v11 = v(i,j+1,k+1), (a, b, c, d) = (v00, v10 - v00, v01 - v00,
// (v11 - v10) - (v01 - v00)).
__device__ __forceinline__ float4 face_coeffs(const float *b0, const float *b1, long long r0,
                                              long long r1, int i) {
    const float v00 = b0[r0 + i], v10 = b0[r1 + i], v01 = b1[r0 + i], v11 = b1[r1 + i];
    return make_float4(v00, v10 - v00, v01 - v00, (v11 - v10) - (v01 - v00));
}

// Cell cubes from the plain grid (one thread per cell).  Cells at i = nx-1,
// j = ny-1 or k = nz-1 are never read (the cell corner is at most n-2); they
// repeat the edge values.
__global__ void k_build_cubes(const float *__restrict__ v, float4 *__restrict__ q, int ntypes,
                              int nx, int ny, int nz) {
    const long long cells = (long long)nx * ny * nz;
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= cells * ntypes) return;
    const long long t = e / cells;
    long long r = e - t * cells;
    const int k = (int)(r / ((long long)nx * ny));
    r -= (long long)k * nx * ny;
    const int j = (int)(r / nx), i = (int)(r - (long long)j * nx);
    const int i1 = i + 1 < nx ? i + 1 : i, j1 = j + 1 < ny ? j + 1 : j, k1 = k + 1 < nz ? k + 1 : k;
    const float *b0 = v + t * cells + (long long)k * nx * ny;
    const float *b1 = v + t * cells + (long long)k1 * nx * ny;
    const long long r0 = (long long)j * nx, r1 = (long long)j1 * nx;
    q[2 * e] = face_coeffs(b0, b1, r0, r1, i);
    q[2 * e + 1] = face_coeffs(b0, b1, r0, r1, i1);
}

// ---------------------------------------------------------------------------
// Pose held across lanes: atom i = lane + 64*s in slot s.
template <int NS>
struct Pose {
    float x[NS], y[NS], z[NS];
};

template <int NS>
__device__ __forceinline__ void pick_atom(const Pose<NS> &Y, int i, float &px, float &py,
                                          float &pz) {
    const int l = i & 63, s = i >> 6;
    px = read_lane(Y.x[0], l);
    py = read_lane(Y.y[0], l);
    pz = read_lane(Y.z[0], l);
#pragma unroll
    for (int q = 1; q < NS; ++q) {
        if (s == q) {
            px = read_lane(Y.x[q], l);
            py = read_lane(Y.y[q], l);
            pz = read_lane(Y.z[q], l);
        }
    }
}

template <int NS>
__device__ __forceinline__ void centroid(const Pose<NS> &Y, int n, float &cx, float &cy,
                                         float &cz) {
    float sx = 0.f, sy = 0.f, sz = 0.f;
    const int lane = lane_id();
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        if (lane + 64 * s < n) {
            sx += Y.x[s];
            sy += Y.y[s];
            sz += Y.z[s];
        }
    }
    const float inv = 1.0f / (float)n;
    cx = wave_sum(sx) * inv;
    cy = wave_sum(sy) * inv;
    cz = wave_sum(sz) * inv;
}

// Generate_Starting_Pose: Y = S_r (X - c0) + grid centre.  X rows in LDS (x,y,z,toff).
template <int NS>
__device__ __forceinline__ void start_pose(Pose<NS> &Y, const float4 *xyzt, int n, int r,
                                           const GridArgs &g, const SearchArgs &sa) {
    const int lane = lane_id();
    Pose<NS> X;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int i = lane + 64 * s;
        const float4 v = i < n ? xyzt[i] : make_float4(0.f, 0.f, 0.f, 0.f);
        X.x[s] = v.x;
        X.y[s] = v.y;
        X.z[s] = v.z;
    }
    float c0x, c0y, c0z;
    centroid(X, n, c0x, c0y, c0z);
    const float4 m0 = sa.smat[3 * r + 0], m1 = sa.smat[3 * r + 1], m2 = sa.smat[3 * r + 2];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const float dx = X.x[s] - c0x, dy = X.y[s] - c0y, dz = X.z[s] - c0z;
        Y.x[s] = fmaf(m0.x, dx, fmaf(m0.y, dy, fmaf(m0.z, dz, g.cx)));
        Y.y[s] = fmaf(m1.x, dx, fmaf(m1.y, dy, fmaf(m1.z, dz, g.cy)));
        Y.z[s] = fmaf(m2.x, dx, fmaf(m2.y, dy, fmaf(m2.z, dz, g.cz)));
    }
}

// Apply alignment orientation o about the pose centroid.
template <int NS>
__device__ __forceinline__ void apply_align(Pose<NS> &Y, int n, int o, const SearchArgs &sa) {
    float cx, cy, cz;
    centroid(Y, n, cx, cy, cz);
    const float4 m0 = sa.amat[3 * o + 0], m1 = sa.amat[3 * o + 1], m2 = sa.amat[3 * o + 2];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const float dx = Y.x[s] - cx, dy = Y.y[s] - cy, dz = Y.z[s] - cz;
        Y.x[s] = fmaf(m0.x, dx, fmaf(m0.y, dy, fmaf(m0.z, dz, cx)));
        Y.y[s] = fmaf(m1.x, dx, fmaf(m1.y, dy, fmaf(m1.z, dz, cy)));
        Y.z[s] = fmaf(m2.x, dx, fmaf(m2.y, dy, fmaf(m2.z, dz, cz)));
    }
}

// How the candidates of one decision (alignment orientations, torsion steps) are
// spread and reduced.  WaveSplit: one wavefront holds them all (batched form).
// BlockSplit: the waves of a workgroup hold interleaved slices and the argmax
// goes through LDS with workgroup barriers (plain form; every wave keeps the
// same pose).
struct WaveSplit {
    __device__ __forceinline__ int first() const { return 0; }
    __device__ __forceinline__ int stride() const { return 64; }
    __device__ __forceinline__ u64 reduce(u64 k) const { return wave_max_u64(k); }
};

struct BlockSplit {
    int wave, waves;
    u64 *slots;  // LDS, [waves]
    __device__ __forceinline__ int first() const { return 64 * wave; }
    __device__ __forceinline__ int stride() const { return 64 * waves; }
    __device__ __forceinline__ u64 reduce(u64 k) const {
        k = wave_max_u64(k);
        if (lane_id() == 0) slots[wave] = k;
        __syncthreads();
        u64 r = slots[0];
        for (int w = 1; w < waves; ++w) r = slots[w] > r ? slots[w] : r;
        __syncthreads();
        return r;
    }
};

// Read-only (cos, sin) table in the constant address space: wave-uniform
// indices load through the scalar cache into SGPRs.
typedef const __attribute__((address_space(4))) float *cfloat2_p;
__device__ __forceinline__ float2 ld_cs(cfloat2_p p, int k) {
    return make_float2(p[2 * k], p[2 * k + 1]);
}

// Alignment orientation o = i*A + j is R_y(2 pi j / A) R_x(2 pi i / A) about the
// pose centroid, applied in two stages to the centred grid-unit offset r of an
// atom.  The x rotation (per atom and i) gives the final y coordinate and the
// rotated z; the y rotation (per j) the final x and z.  (cos, sin) of 2 pi k / A
// come from the acs table; e is the centroid in grid units.
struct XStage {
    float rx, qz, gy;
};
__device__ __forceinline__ XStage align_x(float rx, float ry, float rz, float2 ci, float ey) {
    XStage s;
    s.rx = rx;
    s.qz = fmaf(ci.y, ry, ci.x * rz);
    s.gy = fmaf(ci.x, ry, fmaf(-ci.y, rz, ey));
    return s;
}
__device__ __forceinline__ float align_gx(const XStage &s, float2 cj, float ex) {
    return fmaf(cj.x, s.rx, fmaf(cj.y, s.qz, ex));
}
__device__ __forceinline__ float align_gz(const XStage &s, float2 cj, float ez) {
    return fmaf(-cj.y, s.rx, fmaf(cj.x, s.qz, ez));
}

// Alignment (Rigid Rotation): lanes over the A*A orientations, loop over atoms.
// rec: per-wave LDS, >= n float4.  toff[s]: type byte offset of this lane's atoms.
// Applies and returns the best orientation; *best_out = its score.
template <int NS, class Split>
__device__ int align_pose(Pose<NS> &Y, int n, const int (&toff)[NS], float4 *rec, const Tri &tr,
                          const GridArgs &g, const SearchArgs &sa, float *best_out,
                          const Split &sp) {
    const int lane = lane_id();
    float cx, cy, cz;
    centroid(Y, n, cx, cy, cz);
    const float ex = (cx - g.ox) * g.inv_h, ey = (cy - g.oy) * g.inv_h, ez = (cz - g.oz) * g.inv_h;
    // record: centred grid-unit offset and type offset; all_in: every orientation
    // of every atom samples inside the grid (spheres about the centroid)
    bool out_any = false;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int i = lane + 64 * s;
        if (i < n) {
            const float rx = (Y.x[s] - cx) * g.inv_h, ry = (Y.y[s] - cy) * g.inv_h,
                        rz = (Y.z[s] - cz) * g.inv_h;
            out_any = out_any ||
                      !ball_inside(tr, ex, ey, ez, ball_radius(fmaf(rx, rx, fmaf(ry, ry, rz * rz))));
            rec[i] = make_float4(rx, ry, rz, __int_as_float(toff[s]));
        }
    }
    const bool all_in = __ballot(out_any) == 0ull;
    wave_lds_sync();
    const int NO = sa.A * sa.A;
    u64 best = 0;
    for (int base = sp.first(); base < NO; base += sp.stride()) {
        const int o = base + lane;
        const bool ov = o < NO;
        const int oo = ov ? o : 0;
        const int oi = oo / sa.A;
        const float2 ci = sa.acs[oi], cj = sa.acs[oo - oi * sa.A];
        float acc = 0.f;
        if (all_in) {
            for (int a = 0; a < n; ++a) {
                const float4 r = rec[a];
                const int to = uniform_int(__float_as_int(r.w));
                const XStage xs = align_x(r.x, r.y, r.z, ci, ey);
                acc += tri_in(tr, align_gx(xs, cj, ex), xs.gy, align_gz(xs, cj, ez), to);
            }
        } else {
            for (int a = 0; a < n; ++a) {
                const float4 r = rec[a];
                const int to = uniform_int(__float_as_int(r.w));
                const XStage xs = align_x(r.x, r.y, r.z, ci, ey);
                acc += tri_u(tr, align_gx(xs, cj, ex), xs.gy, align_gz(xs, cj, ez), to);
            }
        }
        const u64 key = ov ? make_key(acc, (uint32_t)o) : 0ull;
        best = key > best ? key : best;
    }
    best = sp.reduce(best);
    const int ob = (int)key_index(best);
    if (best_out) *best_out = key_score(best);
    wave_lds_sync();  // rec is rewritten by the caller next
    apply_align(Y, n, ob, sa);
    return ob;
}

// Rotation frame of bond (a,b) for this lane's atoms: p = a + u(u.v),
// vp = v - u(u.v), w = u x v, with v = Y_i - a; a rotation by theta sends Y_i to
// p + cos(theta) vp + sin(theta) w.
struct Axis {
    float ax, ay, az, ux, uy, uz;
};

template <int NS>
__device__ __forceinline__ Axis bond_axis(const Pose<NS> &Y, int a, int b) {
    Axis A;
    float bx, by, bz;
    pick_atom(Y, a, A.ax, A.ay, A.az);
    pick_atom(Y, b, bx, by, bz);
    const float dx = bx - A.ax, dy = by - A.ay, dz = bz - A.az;
    // unit axis from the hardware reciprocal square root (about one ulp, as
    // against two roundings for a square root and a divide)
    const float inv = __builtin_amdgcn_rsqf(dx * dx + dy * dy + dz * dz);
    A.ux = dx * inv;
    A.uy = dy * inv;
    A.uz = dz * inv;
    return A;
}

__device__ __forceinline__ void torsion_frame(const Axis &A, float x, float y, float z, float &px,
                                              float &py, float &pz, float &vx, float &vy,
                                              float &vz, float &wx, float &wy, float &wz) {
    const float dx = x - A.ax, dy = y - A.ay, dz = z - A.az;
    const float ud = A.ux * dx + A.uy * dy + A.uz * dz;
    px = fmaf(A.ux, ud, A.ax);
    py = fmaf(A.uy, ud, A.ay);
    pz = fmaf(A.uz, ud, A.az);
    vx = fmaf(-A.ux, ud, dx);
    vy = fmaf(-A.uy, ud, dy);
    vz = fmaf(-A.uz, ud, dz);
    wx = A.uy * dz - A.uz * dy;
    wy = A.uz * dx - A.ux * dz;
    wz = A.ux * dy - A.uy * dx;
}

// Turn the moving atoms (mask row mrow) by (c, sn) = (cos, sin) about axis A.
template <int NS>
__device__ __forceinline__ void apply_torsion(Pose<NS> &Y, const u64 *mrow, const Axis &A,
                                              float c, float sn) {
    const int lane = lane_id();
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const bool mv = (mrow[s] >> lane) & 1ull;
        if (mv) {
            float px, py, pz, vx, vy, vz, wx, wy, wz;
            torsion_frame(A, Y.x[s], Y.y[s], Y.z[s], px, py, pz, vx, vy, vz, wx, wy, wz);
            Y.x[s] = fmaf(sn, wx, fmaf(c, vx, px));
            Y.y[s] = fmaf(sn, wy, fmaf(c, vy, py));
            Y.z[s] = fmaf(sn, wz, fmaf(c, vz, pz));
        }
    }
}

// One torsion decision (Optimize Pose, inner angle loop) for rotatable bond with
// moving-mask row mrow (NS words), axis atoms (a,b).  cs[c] = (cos,sin) of this
// lane's candidates k = lane + 64c.  Returns the applied step or kTraceNone.
// Best key (score, candidate) among the nfree candidates of a torsion step
// listed in cand, scored on the moving fragment (frames of m moving atoms in
// rec): lanes take the listed candidates in P passes of 64, each candidate's sum
// runs over the atoms in order, as when every candidate is scored in place.  An
// entry is the step index, with kCandBumped set when the candidate is listed
// although it bumps (no-pruning mode): it is scored but cannot win.
// Inside: every candidate position lies in [0, n-2] on every axis.
template <int P, bool Inside>
__device__ __forceinline__ u64 score_free(int nfree, const uint16_t *cand, const float4 *rec,
                                          int m, const float2 *tors, const Tri &tr) {
    const int lane = lane_id();
    int kp[P];
    bool ok[P];
    float2 csp[P];
    float acc[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int idx = lane + 64 * p;
        const int e = cand[idx < nfree ? idx : 0];
        kp[p] = e & (kCandBumped - 1);
        ok[p] = idx < nfree && !(e & kCandBumped);
        csp[p] = tors[kp[p]];
        acc[p] = 0.f;
    }
    int q = 0;
    // U atoms at a time (up to four (atom, pass) cube loads): their loads are in
    // flight together; the sums still take the atoms in order
    constexpr int U = P == 1 ? 4 : (P == 2 ? 2 : 1);
    if (Inside && U > 1) {
        for (; q + U - 1 < m; q += U) {
            float f[U][P][3];
            float4 c0[U][P], c1[U][P];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const float4 r0 = rec[3 * (q + u) + 0], r1 = rec[3 * (q + u) + 1],
                             r2 = rec[3 * (q + u) + 2];
                const int to = uniform_int(__float_as_int(r0.w));
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    const float gx = fmaf(csp[p].y, r2.x, fmaf(csp[p].x, r1.x, r0.x));
                    const float gy = fmaf(csp[p].y, r2.y, fmaf(csp[p].x, r1.y, r0.y));
                    const float gz = fmaf(csp[p].y, r2.z, fmaf(csp[p].x, r1.z, r0.z));
                    f[u][p][0] = __builtin_amdgcn_fractf(gx);
                    f[u][p][1] = __builtin_amdgcn_fractf(gy);
                    f[u][p][2] = __builtin_amdgcn_fractf(gz);
                    const uint32_t off = in_cell(tr, gx, gy, gz);
                    c0[u][p] = ldq(tr.rs, off, to);
                    c1[u][p] = ldq(tr.rs, off, to + 16);
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int p = 0; p < P; ++p)
                    acc[p] += tri_blend(c0[u][p], c1[u][p], f[u][p][0], f[u][p][1], f[u][p][2]);
        }
    }
    for (; q < m; ++q) {
        const float4 r0 = rec[3 * q + 0], r1 = rec[3 * q + 1], r2 = rec[3 * q + 2];
        const int to = uniform_int(__float_as_int(r0.w));
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const float gx = fmaf(csp[p].y, r2.x, fmaf(csp[p].x, r1.x, r0.x));
            const float gy = fmaf(csp[p].y, r2.y, fmaf(csp[p].x, r1.y, r0.y));
            const float gz = fmaf(csp[p].y, r2.z, fmaf(csp[p].x, r1.z, r0.z));
            acc[p] += Inside ? tri_in(tr, gx, gy, gz, to) : tri_u(tr, gx, gy, gz, to);
        }
    }
    u64 best = 0ull;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const u64 key = ok[p] ? make_key(acc[p], (uint32_t)kp[p]) : 0ull;
        best = key > best ? key : best;
    }
    return best;
}

// score_free with the pass count rounded up to a quarter of C (uniform branch).
template <int C, bool Inside>
__device__ __forceinline__ u64 score_free_any(int nfree, const uint16_t *cand, const float4 *rec,
                                              int m, const float2 *tors, const Tri &tr) {
    constexpr int Q = C >= 4 ? C / 4 : 1;
    constexpr int P2 = 2 * Q <= C ? 2 * Q : C, P3 = 3 * Q <= C ? 3 * Q : C;
    const int np = (nfree + 63) >> 6;
    if (np <= Q) return score_free<Q, Inside>(nfree, cand, rec, m, tors, tr);
    if (np <= P2) return score_free<P2, Inside>(nfree, cand, rec, m, tors, tr);
    if (np <= P3) return score_free<P3, Inside>(nfree, cand, rec, m, tors, tr);
    return score_free<C, Inside>(nfree, cand, rec, m, tors, tr);
}

template <int NS, int C, class Split>
__device__ int torsion_decide(Pose<NS> &Y, int n, const u64 *mrow, int a, int b,
                              const u64 *far, const int (&toff)[NS], float4 *rec,
                              uint16_t *cand, const float2 (&cs)[C], const Tri &tr,
                              const GridArgs &g, const SearchArgs &sa, const Split &sp,
                              long long &nscored) {
    const int lane = lane_id();
    const Axis A = bond_axis(Y, a, b);
    u64 mw[NS];
    int m = 0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        mw[s] = mrow[s];
        m += __popcll(mw[s]);
    }
    // moving-atom frames -> LDS (grid units), static atoms -> registers
    float sgx[NS], sgy[NS], sgz[NS];
    bool st[NS];
    bool out_any = false;  // a moving atom's circle leaves [0, n-2]
    int before = 0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int i = lane + 64 * s;
        const bool mv = (mw[s] >> lane) & 1ull;
        st[s] = !mv && i < n;
        sgx[s] = (Y.x[s] - g.ox) * g.inv_h;
        sgy[s] = (Y.y[s] - g.oy) * g.inv_h;
        sgz[s] = (Y.z[s] - g.oz) * g.inv_h;
        if (mv) {
            float px, py, pz, vx, vy, vz, wx, wy, wz;
            torsion_frame(A, Y.x[s], Y.y[s], Y.z[s], px, py, pz, vx, vy, vz, wx, wy, wz);
            const int q = before + (int)__builtin_amdgcn_mbcnt_hi(
                                       (uint32_t)(mw[s] >> 32),
                                       __builtin_amdgcn_mbcnt_lo((uint32_t)mw[s], 0u));
            rec[3 * q + 0] = make_float4((px - g.ox) * g.inv_h, (py - g.oy) * g.inv_h,
                                         (pz - g.oz) * g.inv_h, __int_as_float(toff[s]));
            rec[3 * q + 1] = make_float4(vx * g.inv_h, vy * g.inv_h, vz * g.inv_h,
                                         __int_as_float(i));
            // every candidate of this atom lies on the circle of radius |V| about P0
            const bool in = ball_inside(tr, (px - g.ox) * g.inv_h, (py - g.oy) * g.inv_h,
                                        (pz - g.oz) * g.inv_h,
                                        ball_radius(fmaf(vx, vx, fmaf(vy, vy, vz * vz))) * g.inv_h);
            rec[3 * q + 2] = make_float4(wx * g.inv_h, wy * g.inv_h, wz * g.inv_h, 0.f);
            out_any = out_any || !in;
        }
        before += __popcll(mw[s]);
    }
    const bool all_in = __ballot(out_any) == 0ull;
    wave_lds_sync();

    // Bump Check of every candidate at once.  For moving atom i (frame P0, V, W)
    // and static atom j, the squared distance after a turn by theta is
    //   d2(theta) = Cq + Aq cos(theta) + Bq sin(theta),
    //   Cq = |P0 - Y_j|^2 + |V|^2, Aq = 2 (P0 - Y_j).V, Bq = 2 (P0 - Y_j).W
    // (V and W are orthogonal with |V| = |W|).  Its minimum over theta is
    // Cq - sqrt(Aq^2 + Bq^2); pairs that cannot come closer than the bump distance
    // are skipped, and each remaining pair is tested against every candidate of
    // the lane with two FMAs.  Distances are in grid units.
    // bumped candidates as wave masks (bit = lane) per candidate slot c
    u64 bumped[C];
#pragma unroll
    for (int c = 0; c < C; ++c) bumped[c] = 0ull;
    const float lim = sa.bump2g;
    const float lim_in = lim * (1.0f + 1e-4f);  // filter margin: keeps borderline pairs
    // static atoms of each slot as wave masks (bit = lane)
    u64 stm[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) stm[s] = __ballot(st[s]);
    for (int q = 0; q < m; ++q) {
        const float4 r0 = rec[3 * q + 0], r1 = rec[3 * q + 1], r2 = rec[3 * q + 2];
        const int i = uniform_int(__float_as_int(r1.w));
        const float vv = fmaf(r1.x, r1.x, fmaf(r1.y, r1.y, r1.z * r1.z));
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            // static atoms of slot s at least bmin bonds from moving atom i
            const u64 elm = far[i * NS + s] & stm[s];
            if (elm == 0ull) continue;
            const float dx = r0.x - sgx[s], dy = r0.y - sgy[s], dz = r0.z - sgz[s];
            const float cq = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, vv)));
            const float aq = 2.0f * fmaf(dx, r1.x, fmaf(dy, r1.y, dz * r1.z));
            const float bq = 2.0f * fmaf(dx, r2.x, fmaf(dy, r2.y, dz * r2.z));
            const float e = cq - lim_in;
            u64 bal = sa.prune ? elm & (__builtin_amdgcn_ballot_w64(e < 0.0f) |
                                        __builtin_amdgcn_ballot_w64(e * e < fmaf(aq, aq, bq * bq)))
                               : elm;
            while (bal != 0ull) {
                const int src = __ffsll((long long)bal) - 1;
                bal &= bal - 1ull;
                const float c0 = read_lane(cq, src), a0 = read_lane(aq, src),
                            b0 = read_lane(bq, src);
#pragma unroll
                for (int c = 0; c < C; ++c)
                    bumped[c] |= __ballot(fmaf(b0, cs[c].y, fmaf(a0, cs[c].x, c0)) < lim);
            }
        }
    }
    // Only the bump-free candidates are scored (on the paper's workloads more than
    // half are bumped): list them for this wave, then score the list.  Without
    // pruning every candidate is listed and scored, the bumped ones flagged.
    int nfree = 0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int k = sp.first() + lane + sp.stride() * c;
        const bool bmp = (bumped[c] >> lane) & 1ull;
        const bool listed = k < sa.T && (!sa.prune || !bmp);
        const u64 bm = __ballot(listed);
        if (listed)
            cand[nfree + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bm >> 32),
                                                        __builtin_amdgcn_mbcnt_lo((uint32_t)bm, 0u))] =
                (uint16_t)(bmp ? k | kCandBumped : k);
        nfree += __popcll(bm);
    }
    wave_lds_sync();
    nscored += (long long)nfree * m;
    u64 best = 0ull;
    if (nfree > 0)
        best = all_in ? score_free_any<C, true>(nfree, cand, rec, m, sa.tors, tr)
                      : score_free_any<C, false>(nfree, cand, rec, m, sa.tors, tr);
    best = sp.reduce(best);
    const int kstar = best == 0ull ? (int)kTraceNone : (int)key_index(best);
    wave_lds_sync();  // rec is rewritten next
    if (kstar != (int)kTraceNone) {
        const float2 t = sa.tors[kstar];
        apply_torsion(Y, mrow, A, t.x, t.y);  // the pose is unchanged since A was taken
    }
    return kstar;
}

// Score of the pose: sum over atoms of the grid of the atom's type.
template <int NS>
__device__ __forceinline__ float pose_score(const Pose<NS> &Y, int n, const int (&toff)[NS],
                                            const Tri &tr, const GridArgs &g) {
    const int lane = lane_id();
    float s = 0.f;
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        if (lane + 64 * q < n)
            s += tri_v(tr, (Y.x[q] - g.ox) * g.inv_h, (Y.y[q] - g.oy) * g.inv_h,
                       (Y.z[q] - g.oz) * g.inv_h, (uint32_t)toff[q]);
    }
    return wave_sum(s);
}

// ---------------------------------------------------------------------------
// Shared-memory layout (bytes), identical for host and device.
struct Lds {
    static __host__ __device__ size_t xyzt(int nmax) { return 0; }
    static __host__ __device__ size_t far(int nmax) { return (size_t)nmax * 16; }
    static __host__ __device__ size_t mask(int nmax, int nw) {
        return far(nmax) + (size_t)nmax * nw * 8;
    }
    static __host__ __device__ size_t rot(int nmax, int nw) {
        return mask(nmax, nw) + (size_t)kMaxRot * nw * 8;
    }
    static __host__ __device__ size_t misc(int nmax, int nw) {
        return rot(nmax, nw) + (size_t)kMaxRot * 8;
    }
    static __host__ __device__ size_t rec(int nmax, int nw) { return misc(nmax, nw) + 16; }
    // per wave: moving-atom frames (3 float4 per atom), then the list of
    // bump-free torsion candidates (u16, up to kMaxTorsionSteps)
    static __host__ __device__ size_t rec_stride(int nmax) {
        return (size_t)nmax * 48 + (size_t)kMaxTorsionSteps * 2;
    }
    static __host__ __device__ size_t cand(int nmax) { return (size_t)nmax * 48; }
};

static inline __host__ __device__ int bin_nmax(int bin) { return 32 * (bin + 1); }
static inline __host__ __device__ int bin_slots(int bin) { return (bin_nmax(bin) + 63) / 64; }

size_t dock_lds_bytes(int nmax, int waves) {
    const int nw = (nmax + 63) / 64;
    return Lds::rec(nmax, nw) + (size_t)waves * Lds::rec_stride(nmax);
}

// Stage ligand l into LDS (whole workgroup).
template <int NS>
__device__ void stage_ligand(unsigned char *smem, int nmax, int l, const LibArgs &lib,
                             const WorkArgs &ws, const GridArgs &g, bool with_far) {
    float4 *xyzt = (float4 *)(smem + Lds::xyzt(nmax));
    u64 *far = (u64 *)(smem + Lds::far(nmax));
    u64 *mask = (u64 *)(smem + Lds::mask(nmax, NS));
    int2 *rot = (int2 *)(smem + Lds::rot(nmax, NS));
    int *misc = (int *)(smem + Lds::misc(nmax, NS));
    const int a0 = lib.atom_off[l], n = lib.atom_off[l + 1] - a0;
    const int r0 = lib.rot_off[l], B = lib.rot_off[l + 1] - r0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const float *p = lib.xyz + 3 * (size_t)(a0 + i);
        const uint32_t toff = (uint32_t)lib.type[a0 + i] * g.type_bytes;
        xyzt[i] = make_float4(p[0], p[1], p[2], __uint_as_float(toff));
    }
    if (with_far) {
        for (int e = threadIdx.x; e < n * NS; e += blockDim.x) {
            const int i = e / NS, w = e - i * NS;
            far[e] = ws.far[(size_t)(a0 + i) * kFarWords + w];
        }
    }
    for (int e = threadIdx.x; e < B * NS; e += blockDim.x) {
        const int b = e / NS, w = e - b * NS;
        mask[e] = w < lib.mask_words ? lib.rot_mask[(size_t)(r0 + b) * lib.mask_words + w] : 0ull;
    }
    for (int b = threadIdx.x; b < B; b += blockDim.x)
        rot[b] = make_int2(lib.rot_bond[2 * (size_t)(r0 + b)], lib.rot_bond[2 * (size_t)(r0 + b) + 1]);
    if (threadIdx.x == 0) {
        misc[1] = n;
        misc[2] = B;
    }
}

template <int NS>
__device__ __forceinline__ void lane_toff(const float4 *xyzt, int n, int (&toff)[NS]) {
    const int lane = lane_id();
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int i = lane + 64 * s;
        toff[s] = i < n ? __float_as_int(xyzt[i].w) : 0;
    }
}

static __device__ __forceinline__ size_t trace_base(const LibArgs &lib, const SearchArgs &sa, int l) {
    return (size_t)sa.R * ((size_t)l + (size_t)sa.P * (size_t)lib.rot_off[l]);
}

// ---------------------------------------------------------------------------
// Docking kernel: persistent workgroups pop (ligand, restart-group) items of one
// size bin; each wave docks one restart from the orientation k_align chose.
template <int NS, int C>
__global__ __launch_bounds__(512) void k_dock(GridArgs g, SearchArgs sa, LibArgs lib, WorkArgs ws,
                                              int bin, int lst) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int nmax = bin_nmax(bin);
    const int W = blockDim.x >> 6, wave = threadIdx.x >> 6, lane = lane_id();
    float4 *xyzt = (float4 *)(smem + Lds::xyzt(nmax));
    const u64 *far = (const u64 *)(smem + Lds::far(nmax));
    const u64 *mask = (const u64 *)(smem + Lds::mask(nmax, NS));
    const int2 *rot = (const int2 *)(smem + Lds::rot(nmax, NS));
    int *misc = (int *)(smem + Lds::misc(nmax, NS));
    float4 *rec = (float4 *)(smem + Lds::rec(nmax, NS) + (size_t)wave * Lds::rec_stride(nmax));
    uint16_t *cand = (uint16_t *)((unsigned char *)rec + Lds::cand(nmax));
    const Tri tr = make_tri(g);

    float2 cs[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int k = lane + 64 * c;
        cs[c] = k < sa.T ? sa.tors[k] : make_float2(1.f, 0.f);
    }
    const int groups = (sa.R + W - 1) / W;
    const long long total = (long long)ws.counters[lst] * groups;
    int cur = -1;
    for (;;) {
        if (threadIdx.x == 0) misc[0] = atomicAdd(&ws.counters[kMaxLists + lst], 1);
        __syncthreads();
        const int item = misc[0];
        if ((long long)item >= total) break;
        const int li = item / groups, grp = item - li * groups;
        const int l = ws.bin_list[(size_t)lst * lib.L + li];
        if (l != cur) {
            stage_ligand<NS>(smem, nmax, l, lib, ws, g, true);
            cur = l;
        }
        __syncthreads();
        const int r = grp * W + wave;
        if (r < sa.R) {
            const int n = misc[1], B = misc[2];
            int toff[NS];
            lane_toff(xyzt, n, toff);
            Pose<NS> Y;
            start_pose(Y, xyzt, n, r, g, sa);
            uint16_t *tr_out = ws.rtrace + trace_base(lib, sa, l) + (size_t)r * (1 + sa.P * B);
            // the alignment step was taken by k_align (first trace entry)
            const int o = uniform_int((int)tr_out[0]);
            apply_align(Y, n, o < sa.A * sa.A ? o : 0, sa);
            int d = 1;
            long long nsc = 0;
            for (int p = 0; p < sa.P; ++p) {
                for (int b = 0; b < B; ++b, ++d) {
                    const int2 ab = rot[b];
                    const int k = torsion_decide<NS, C>(Y, n, mask + b * NS, uniform_int(ab.x),
                                                        uniform_int(ab.y), far, toff, rec, cand,
                                                        cs, tr, g, sa, WaveSplit(), nsc);
                    if (lane == 0) tr_out[d] = (uint16_t)k;
                }
            }
            if (ws.scored && lane == 0) atomicAdd(ws.scored, (unsigned long long)nsc);
            const float sc = pose_score(Y, n, toff, tr, g);
            if (lane == 0) ws.rscore[(size_t)l * sa.R + r] = sc;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Batched rigid alignment (Rigid Rotation of Alg. 1) from sphere shells in LDS.
//
// Every alignment sample of atom a lies on the sphere of radius |Y_a - c| about
// the pose centroid c, and Generate_Starting_Pose puts c at the grid centre for
// every restart and every ligand.  So the grid cells a sample can fall in
// depend only on the atom type and that radius.  At pocket load the shell
// atlas stores, per type and per radius band of kBandWidth cells (thickened by
// kShellPad on both sides), the cells the band crosses as face columns: for
// vertex x-position i of cell row (j,k) the bilinear coefficients of the face
// with corners v(i,j,k), v(i,j+1,k), v(i,j,k+1), v(i,j+1,k+1) (the first half
// of cube (i,j,k)); cell (i,j,k) is the two consecutive columns i and i+1.  A
// row table indexed by (j,k) gives each row's cell range on the low-x and the
// high-x side of the centre.  A workgroup of k_align aligns GR restarts of one
// ligand: per atom one wave streams that atom's band into LDS while the others
// sample the previous one, and all GR * A * A samples of the atom read LDS.  A
// sample whose cell is not in the band reads its cube from global memory; both
// give the same values, and the transform, blend and atom-order sum are those
// of align_pose, so the scores are bit-identical.
// The pad covers the rounding of a sample's distance from the grid centre (the
// pose centroid lands there up to ~1e-5 cells, the turn keeps |r| up to a few
// ulps): ~1e-4 cells at most, 200 times less than the pad.
constexpr float kShellPad = 0.02f;
constexpr float kBandWidth = 0.125f;
constexpr int kShellRowsPerThread = 4;  // atlas kernels: rows per thread of 1024
#ifndef DOCK_SHELL_BATCH
#define DOCK_SHELL_BATCH 2
#endif
constexpr int kShellBatch = DOCK_SHELL_BATCH;  // samples scheduled together

// Of the JM y-rotation slots of a k_align lane, align_global_count(JM) take
// their samples from the cubes in global memory (through L1/L2) instead of the
// LDS band: the value is the same, and the two paths run on separate hardware
// (the LDS versus the vector-memory pipeline), so their sample rates add.  The
// global slots are spread evenly over the JM (is_global_slot).
#ifndef DOCK_ALIGN_GLOBAL_32THS
#define DOCK_ALIGN_GLOBAL_32THS 0
#endif
__host__ __device__ constexpr int align_global_count(int G) {
    return G * DOCK_ALIGN_GLOBAL_32THS / 32;
}
__host__ __device__ constexpr bool is_global_slot(int G, int gg) {
    return (gg + 1) * align_global_count(G) / G != gg * align_global_count(G) / G;
}

// Side entry of a row: bits 0-15 first column (relative to the band's columns)
// minus the first cell x plus kEntryBias, so that cell ix of the segment is
// column (e & 0xFFFF) - kEntryBias + ix; bits 16-23 first cell x, 24-31 number
// of cells (0: empty side).
constexpr int kEntryBias = 512;
__device__ __forceinline__ int seg_entry(int base, int lo, int len) {
    return len > 0 ? ((base - lo + kEntryBias) | (lo << 16) | (len << 24)) : kEntryBias;
}

struct RowShell {
    int nlo, nhi, plo, phi;  // cell x ranges, low and high side; empty: lo > hi
    bool merged;             // one segment serves both sides
    __device__ int cols_n() const { return nhi >= nlo ? nhi - nlo + 2 : 0; }
    __device__ int cols_p() const { return (!merged && phi >= plo) ? phi - plo + 2 : 0; }
};

// Cells of row (iy, iz) crossed by the shell rlo <= |p - ec| <= rhi (grid units).
__device__ RowShell shell_row(int iy, int iz, float ecx, float ecy, float ecz, float rlo2,
                              float rhi2, const GridArgs &g) {
    RowShell r{1, 0, 1, 0, false};
    if (iy < 0 || iy > g.ny - 2 || iz < 0 || iz > g.nz - 2) return r;
    const float ya = (float)iy - ecy, yb = ya + 1.0f;
    const float za = (float)iz - ecz, zb = za + 1.0f;
    const float dy0 = ya > 0.0f ? ya : (yb < 0.0f ? -yb : 0.0f);
    const float dz0 = za > 0.0f ? za : (zb < 0.0f ? -zb : 0.0f);
    const float dy1 = fmaxf(fabsf(ya), fabsf(yb)), dz1 = fmaxf(fabsf(za), fabsf(zb));
    const float dmin2 = dy0 * dy0 + dz0 * dz0, dmax2 = dy1 * dy1 + dz1 * dz1;
    if (dmin2 > rhi2) return r;
    const float xa = sqrtf(fmaxf(rlo2 - dmax2, 0.0f)), xb = sqrtf(rhi2 - dmin2);
    r.nlo = max((int)floorf(ecx - xb), 0);
    r.nhi = min((int)floorf(ecx - xa), g.nx - 2);
    r.plo = max((int)floorf(ecx + xa), 0);
    r.phi = min((int)floorf(ecx + xb), g.nx - 2);
    if (r.nlo > r.nhi) {  // only the high side: keep it as the segment of both sides
        r.nlo = r.plo;
        r.nhi = r.phi;
        r.merged = true;
    } else if (r.plo > r.phi) {
        r.merged = true;
    } else if (r.nhi + 1 >= r.plo) {
        r.nhi = max(r.nhi, r.phi);
        r.merged = true;
    }
    return r;
}

struct BandGeom {
    int y0, z0, thy, thz;
    float rlo2, rhi2;
};

__device__ __forceinline__ BandGeom band_geom(int b, float ecy, float ecz) {
    BandGeom q;
    const float rlo = fmaxf((float)b * kBandWidth - kShellPad, 0.0f);
    const float rhi = (float)(b + 1) * kBandWidth + kShellPad;
    q.rlo2 = rlo * rlo;
    q.rhi2 = rhi * rhi;
    q.y0 = (int)floorf(ecy - rhi) - 1;
    q.z0 = (int)floorf(ecz - rhi) - 1;
    q.thy = (int)floorf(ecy + rhi) + 1 - q.y0 + 1;
    q.thz = (int)floorf(ecz + rhi) + 1 - q.z0 + 1;
    return q;
}

// Atlas pass 1 (one workgroup of 1024 per band): band geometry and column count.
// info[2b] = (y0, z0, thy, thz), info[2b+1] = (rows, ncols or -1, table bytes, 0);
// pass 2 sets info[2b+1].w to the band's row split (see k_atlas_fill).
__global__ __launch_bounds__(1024) void k_atlas_count(GridArgs g, int4 *info) {
    __shared__ int wsum[16];
    const int b = blockIdx.x, tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    const BandGeom q = band_geom(b, g.acy, g.acz);
    const int rows = q.thy * q.thz;
    const int per = (rows + (int)blockDim.x - 1) / (int)blockDim.x;
    int local = 0;
    if (per <= kShellRowsPerThread) {
        for (int k = 0; k < per; ++k) {
            const int t = tid * per + k;
            if (t < rows) {
                const RowShell r = shell_row(q.y0 + t / q.thz, q.z0 + t % q.thz, g.acx, g.acy,
                                             g.acz, q.rlo2, q.rhi2, g);
                local += r.cols_n() + r.cols_p();
            }
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) local += __shfl_xor(local, o, 64);
    if (lane == 0) wsum[wave] = local;
    __syncthreads();
    if (tid == 0) {
        int total = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) total += wsum[w];
        // entries hold (first column - first cell + kEntryBias) in 16 bits
        const bool ok = per <= kShellRowsPerThread && total < (1 << 15);
        info[2 * b] = make_int4(q.y0, q.z0, q.thy, q.thz);
        info[2 * b + 1] = make_int4(rows, ok ? total : -1, (rows * 8 + 15) & ~15, 0);
    }
}

// Atlas pass 2 (one workgroup of 1024 per (type, band)): the row table and the
// face columns of the band, from the cell cubes.  blob16[t*nb + b] is the
// band's offset in float4 units.  The columns are stored row by row, so the
// column index C1 at which the first row starts whose columns begin at or past
// half the band splits it into two chunks, each a run of whole rows (both
// columns of every cell in one chunk); the type-0 workgroup writes C1 into
// info[2b+1].w (k_align streams a band larger than its LDS region in two
// chunks of the same table).
__global__ __launch_bounds__(1024) void k_atlas_fill(GridArgs g, int4 *info,
                                                     const int *blob16, float4 *atlas, int nb) {
    __shared__ int pre[kShellRowsPerThread * 1024 + 1];
    __shared__ int wsum[16];
    const int t = blockIdx.x / nb, b = blockIdx.x - t * nb;
    const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6, BD = blockDim.x;
    const int4 i1 = info[2 * b + 1];
    if (i1.y < 0) return;
    const BandGeom q = band_geom(b, g.acy, g.acz);
    const int rows = i1.x, per = (rows + BD - 1) / BD;
    int2 *table = (int2 *)(atlas + blob16[blockIdx.x]);
    float4 *col = atlas + blob16[blockIdx.x] + i1.z / 16;
    int cnt[kShellRowsPerThread];
    int local = 0;
#pragma unroll
    for (int k = 0; k < kShellRowsPerThread; ++k) {
        cnt[k] = 0;
        const int r = tid * per + k;
        if (k < per && r < rows) {
            const RowShell s = shell_row(q.y0 + r / q.thz, q.z0 + r % q.thz, g.acx, g.acy, g.acz,
                                         q.rlo2, q.rhi2, g);
            cnt[k] = s.cols_n() + s.cols_p();
        }
        local += cnt[k];
    }
    int incl = local;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int v = __shfl_up(incl, o, 64);
        if (lane >= o) incl += v;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int run = incl - local;
    for (int w = 0; w < wave; ++w) run += wsum[w];
#pragma unroll
    for (int k = 0; k < kShellRowsPerThread; ++k) {
        const int r = tid * per + k;
        if (k < per && r < rows) {
            pre[r] = run;
            const RowShell s = shell_row(q.y0 + r / q.thz, q.z0 + r % q.thz, g.acx, g.acy, g.acz,
                                         q.rlo2, q.rhi2, g);
            const int cn = s.cols_n();
            const int en = seg_entry(run, s.nlo, cn > 0 ? s.nhi - s.nlo + 1 : 0);
            const int ep = s.merged ? en
                                    : seg_entry(run + cn, s.plo, s.phi >= s.plo ? s.phi - s.plo + 1 : 0);
            table[r] = make_int2(en, ep);
            run += cnt[k];
        }
    }
    __syncthreads();
    if (t == 0) {
        // C1 = pre[r] for the first row r with pre[r] >= ncols / 2 (a row boundary)
        for (int r = tid; r < rows; r += BD) {
            const bool first = pre[r] >= i1.y / 2 && (r == 0 || pre[r - 1] < i1.y / 2);
            if (first) info[2 * b + 1].w = pre[r];
        }
    }
    for (int v = tid; v < i1.y; v += BD) {
        int lo = 0, hi = rows - 1;  // last row whose first column is <= v
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (pre[mid] <= v) lo = mid;
            else hi = mid - 1;
        }
        const int iy = q.y0 + lo / q.thz, iz = q.z0 + lo % q.thz;
        const RowShell s = shell_row(iy, iz, g.acx, g.acy, g.acz, q.rlo2, q.rhi2, g);
        const int u = v - pre[lo], cn = s.cols_n();
        const int i = u < cn ? s.nlo + u : s.plo + (u - cn);
        const size_t e = ((size_t)t * g.nz * g.ny + (size_t)iz * g.ny + iy) * g.nx + i;
        col[v] = g.cubes[2 * e];
    }
}

// Shared-memory layout of k_align (bytes); GR restarts per item.
struct AlignLds {
    static __host__ __device__ size_t xyzt() { return 0; }                  // [nmax] x,y,z,toff
    static __host__ __device__ size_t dxyz(int nmax) { return (size_t)nmax * 16; }  // X - c0, toff
    static __host__ __device__ size_t ectr(int nmax) { return dxyz(nmax) + (size_t)nmax * 16; }
    static __host__ __device__ size_t ainf(int nmax, int GR) {
        return ectr(nmax) + (size_t)GR * 32;  // [GR] centroid (world), centroid (grid units)
    }
    static __host__ __device__ size_t misc(int nmax, int GR) { return ainf(nmax, GR) + (size_t)nmax * 32; }
    static __host__ __device__ size_t best(int nmax, int GR) { return misc(nmax, GR) + 128; }
    static __host__ __device__ size_t region(int nmax, int GR) {
        return (best(nmax, GR) + (size_t)GR * 8 + 15) & ~(size_t)15;
    }
};

struct Shell {
    int y0, z0, thy, thz, rows, maxcol;
    float cx;             // centre x (grid units): side of a sample
    unsigned koff;        // absolute row index y0*thz + z0 of the first row
    const int2 *table;    // [thy*thz] (low-side entry, high-side entry)
    const float4 *col;    // face columns
    const float4 *zero;   // two zero columns: a miss blends to +0
    // The same band as LDS byte addresses, for the in-grid sample paths (unsigned
    // arithmetic, so an address below the region start wraps and wraps back):
    uint32_t t0b;         // absolute row 0 (the table's first row less koff rows)
    uint32_t tlob, thib;  // the table's first and last rows
    uint32_t colb;        // column c at colb + 16 (c + kEntryBias)
    uint32_t cmaxb;       // maxcol + kEntryBias
    uint32_t zerob;       // the zero pair
};

// LDS byte address of a pointer into shared memory, and loads from one.
typedef int lds_i32x2 __attribute__((ext_vector_type(2)));
typedef float lds_f32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint32_t lds_addr(const void *p) {
    return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) void *)p;
}
__device__ __forceinline__ int2 lds_ld_int2(uint32_t a) {
    const lds_i32x2 v = *(const __attribute__((address_space(3))) lds_i32x2 *)a;
    return make_int2(v.x, v.y);
}
__device__ __forceinline__ float4 lds_ld_float4(uint32_t a) {
    const lds_f32x4 v = *(const __attribute__((address_space(3))) lds_f32x4 *)a;
    return make_float4(v.x, v.y, v.z, v.w);
}

// Byte-address fields of a shell whose table starts at LDS address table_b and
// whose column c lies at col_b + 16 c (rows, koff, maxcol already set).
__device__ __forceinline__ void shell_bytes(Shell &s, uint32_t table_b, uint32_t col_b) {
    s.tlob = table_b;
    s.thib = table_b + 8u * (uint32_t)(s.rows - 1);
    s.t0b = table_b - 8u * s.koff;
    // wave-uniform and opaque, so that a column address stays one shift-and-add
    // of the index
    s.colb = (uint32_t)uniform_int((int)(col_b - 16u * (uint32_t)kEntryBias));
    asm volatile("" : "+s"(s.colb));
    s.cmaxb = (uint32_t)(s.maxcol + kEntryBias);
}

// x clamped to [lo, hi] in one instruction (lo <= hi).
__device__ __forceinline__ uint32_t med3_u32(uint32_t x, uint32_t lo, uint32_t hi) {
    uint32_t r;
    asm("v_med3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "v"(lo), "v"(hi));
    return r;
}

// Low 16 bits of a row entry pair's entry on the sample's side of the centre
// (e.x when gx < cx, else e.y; cx wave-uniform): the compare, then one
// sub-dword select that takes the low halves of both operands.
__device__ __forceinline__ uint32_t side_lo16(int2 e, float gx, float cx) {
    uint32_t r;
    asm("v_cmp_gt_f32 vcc, %3, %4\n\t"
        "v_cndmask_b32_sdwa %0, %2, %1, vcc dst_sel:DWORD dst_unused:UNUSED_PAD "
        "src0_sel:WORD_0 src1_sel:WORD_0"
        : "=v"(r)
        : "v"(e.x), "v"(e.y), "s"(cx), "v"(gx)
        : "vcc");
    return r;
}

__device__ __forceinline__ float lerp_cell(const float4 *p, float fx, float fy, float fz) {
    return tri_blend(p[0], p[1], fx, fy, fz);
}

// Column pair of cell x index ix in row entry pair e2 (side by gx), or the zero
// pair when the cell is not in the shell.
__device__ __forceinline__ const float4 *shell_cols(const Shell &s, int2 e2, float gx, int ix,
                                                    bool &hit) {
    const unsigned e = (unsigned)(gx < s.cx ? e2.x : e2.y);
    const int d = ix - (int)((e >> 16) & 255u);
    hit = (unsigned)d < (e >> 24);
    return hit ? s.col + ((int)(e & 0xFFFFu) - kEntryBias + ix) : s.zero;
}

// Trilinear sample of grid coordinates (gx,gy,gz) from the shell, for an atom
// whose sphere may leave the grid: the clamps of tri_u, the row range and the
// segment are checked, and a cell not in the shell gives +0 and hit = false.
// Same arithmetic as tri_u.
__device__ __forceinline__ float shell_sample(const Shell &s, const Tri &t, float gx, float gy,
                                              float gz, bool &hit) {
    const float cx = __builtin_amdgcn_fmed3f(gx, 0.0f, t.mx);
    const float cy = __builtin_amdgcn_fmed3f(gy, 0.0f, t.my);
    const float cz = __builtin_amdgcn_fmed3f(gz, 0.0f, t.mz);
    const float ix = floorf(__builtin_amdgcn_fmed3f(gx, 0.0f, t.m2x));
    const float iy = floorf(__builtin_amdgcn_fmed3f(gy, 0.0f, t.m2y));
    const float iz = floorf(__builtin_amdgcn_fmed3f(gz, 0.0f, t.m2z));
    const int jy = (int)iy - s.y0, kz = (int)iz - s.z0;
    const bool rin = (unsigned)jy < (unsigned)s.thy && (unsigned)kz < (unsigned)s.thz;
    const unsigned ri = min((unsigned)(__mul24(jy, s.thz) + kz), (unsigned)s.rows - 1u);
    int2 e2 = s.table[ri];
    e2.x &= 0 - (int)rin;
    e2.y &= 0 - (int)rin;
    return lerp_cell(shell_cols(s, e2, gx, (int)ix, hit), cx - ix, cy - iy, cz - iz);
}

// One batch of kShellBatch samples (y slots j0..) of a sphere inside the grid,
// in phases so that a wave keeps every sample's reads in flight together:
// fractions and row entries, then the cell columns (LDS band, or the cube in
// global memory for the slots is_global_slot picks), then the blends.  Each
// value is the one tri_in gives.  Every sample lies in [0, n-2] on each axis, so
// the clamps of tri_u are the identity, floor is truncation and the fraction is
// exact as v_fract.  A sample's distance to the grid centre differs from the
// atom's radius by FP32 rounding only (~1e-4 cells, against kShellPad), so by
// construction of the band its row lies in the table and its cell in the row's
// segment on its side of the centre (two separate segments are more than a cell
// apart): the row and column indices are only clamped, to keep reads in bounds.
// fy is the fraction of gy and rowy the byte address of row (int) gy * thz of
// the table (both per atom); the indices are LDS byte addresses.
template <int JM>
__device__ __forceinline__ void shell_batch_in(float (&v)[kShellBatch], int j0, const Shell &s,
                                               const Tri &t, const float (&gx)[kShellBatch],
                                               float gy, float fy, uint32_t rowy,
                                               const float (&gz)[kShellBatch], int to) {
    float fx[kShellBatch], fz[kShellBatch];
    uint32_t off[kShellBatch];
    int2 e2[kShellBatch];
#pragma unroll
    for (int k = 0; k < kShellBatch; ++k) {
        fx[k] = __builtin_amdgcn_fractf(gx[k]);
        fz[k] = __builtin_amdgcn_fractf(gz[k]);
        if (is_global_slot(JM, j0 + k)) {
            off[k] = in_cell(t, gx[k], gy, gz[k]);
        } else {
            // absolute row iy*thz + iz, clamped to the table's rows
            e2[k] = lds_ld_int2(med3_u32(rowy + ((uint32_t)(int)gz[k] << 3), s.tlob, s.thib));
        }
    }
    // every row read is issued before the first column address waits for one
    __builtin_amdgcn_sched_barrier(0);
    float4 q0[kShellBatch], q1[kShellBatch];
#pragma unroll
    for (int k = 0; k < kShellBatch; ++k) {
        if (is_global_slot(JM, j0 + k)) {
            q0[k] = ldq(t.rs, off[k], to);
            q1[k] = ldq(t.rs, off[k], to + 16);
        } else {
            const uint32_t c = min(side_lo16(e2[k], gx[k], s.cx) + (uint32_t)(int)gx[k], s.cmaxb);
            const uint32_t a = s.colb + (c << 4);
            q0[k] = lds_ld_float4(a);
            q1[k] = lds_ld_float4(a + 16u);
        }
    }
    // every column read is issued before the first blend waits for one
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < kShellBatch; ++k) v[k] = tri_blend(q0[k], q1[k], fx[k], fy, fz[k]);
}

// Per-atom inputs of shell_batch_in / shell_batch_part: the fraction of gy and
// the byte address of table row (int) gy * thz.
__device__ __forceinline__ uint32_t shell_rowy(const Shell &s, float gy) {
    return s.t0b + (__umul24((uint32_t)(int)gy, (uint32_t)s.thz) << 3);
}

// The JM samples of one atom for one lane's strip (restart, x-rotation i, y
// rotations j0 .. j0+JM-1; cj = the (cos, sin) entries from j0), added to acc in
// slot order.  Slots from jw on are past A for every lane of the wave and are
// skipped in whole batches.  A sample whose cell is not in the shell adds +0
// (the exact identity: a sum that starts at +0 never becomes -0) and is redone
// from global memory before any later addition to its accumulator, so every sum
// keeps atom order.
template <int JM, bool Inside>
__device__ __forceinline__ void shell_atom(float (&acc)[JM], const Shell &sh, const Tri &tr,
                                           const XStage &xs, cfloat2_p cj, int jw, float ex,
                                           float ez, int to) {
    if constexpr (Inside) {
        const float fy = __builtin_amdgcn_fractf(xs.gy);
        const uint32_t rowy = shell_rowy(sh, xs.gy);
        // (cos, sin) of the next batch's y rotations, loaded one batch ahead
        float2 cn[kShellBatch];
#pragma unroll
        for (int k = 0; k < kShellBatch; ++k) cn[k] = ld_cs(cj, k);
#pragma unroll
        for (int j0 = 0; j0 < JM; j0 += kShellBatch) {
            if (j0 < jw) {
                float gx[kShellBatch], gz[kShellBatch], v[kShellBatch];
                float2 cc[kShellBatch];
#pragma unroll
                for (int k = 0; k < kShellBatch; ++k) cc[k] = cn[k];
                if (j0 + kShellBatch < JM) {
#pragma unroll
                    for (int k = 0; k < kShellBatch; ++k) cn[k] = ld_cs(cj, j0 + kShellBatch + k);
                }
#pragma unroll
                for (int k = 0; k < kShellBatch; ++k) {
                    gx[k] = align_gx(xs, cc[k], ex);
                    gz[k] = align_gz(xs, cc[k], ez);
                }
                shell_batch_in<JM>(v, j0, sh, tr, gx, xs.gy, fy, rowy, gz, to);
#pragma unroll
                for (int k = 0; k < kShellBatch; ++k) acc[j0 + k] += v[k];
            }
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int jj = 0; jj < JM; ++jj) asm volatile("" : "+v"(acc[jj]));
        return;
    } else {
    bool miss = false;
#pragma unroll
    for (int j0 = 0; j0 < JM; j0 += kShellBatch) {
        if (j0 < jw) {
#pragma unroll
            for (int jj = j0; jj < j0 + kShellBatch; ++jj) {
                const float2 c = ld_cs(cj, jj);
                const float gx = align_gx(xs, c, ex), gz = align_gz(xs, c, ez);
                if (is_global_slot(JM, jj)) {
                    acc[jj] += tri_u(tr, gx, xs.gy, gz, to);
                } else {
                    bool hit;
                    acc[jj] += shell_sample(sh, tr, gx, xs.gy, gz, hit);
                    miss = miss || !hit;
                }
            }
        }
        // keep the scheduler from hoisting every sample's loads (register spills)
        __builtin_amdgcn_sched_barrier(0);
    }
    // materialise the sums here (else the compiler defers them past the branch
    // below and keeps every sample's inputs live)
#pragma unroll
    for (int jj = 0; jj < JM; ++jj) asm volatile("" : "+v"(acc[jj]));
    if (__ballot(miss) != 0ull) {
        // recompute rather than keep the first pass's coordinates live across it
        // (an opaque zero offset stops the compiler merging the two passes)
        int z = 0;
        asm volatile("" : "+v"(z));
#pragma unroll
        for (int jj = 0; jj < JM; ++jj) {
            if (is_global_slot(JM, jj) || jj >= jw) continue;
            const float2 c = ld_cs(cj, jj + z);
            const float gx = align_gx(xs, c, ex), gz = align_gz(xs, c, ez);
            bool hit;
            (void)shell_sample(sh, tr, gx, xs.gy, gz, hit);
            if (!hit) acc[jj] += tri_u(tr, gx, xs.gy, gz, to);
        }
    }
    }
}

// shell_batch_in for a band of which only columns [lo, hi) are resident (a band
// streamed in two chunks of whole rows): a sample whose column lies in the
// resident chunk reads it, the others read the zero pair and add +0.  Each
// sample's column lies in exactly one chunk and the two passes of an atom run
// before the next atom, so every accumulator gets each sample once, in atom
// order, and +0 never changes a sum (sums start at +0 and never become -0).
// plo = lo + kEntryBias and pn = hi - lo: the chunk in biased column indices;
// the chunk test replaces the column clamp of shell_batch_in.
template <int JM>
__device__ __forceinline__ void shell_batch_part(float (&v)[kShellBatch], const Shell &s,
                                                 const float (&gx)[kShellBatch], float fy,
                                                 uint32_t rowy, const float (&gz)[kShellBatch],
                                                 uint32_t plo, uint32_t pn) {
    static_assert(align_global_count(JM) == 0, "no global slots in a chunked band");
    float fx[kShellBatch], fz[kShellBatch];
    int2 e2[kShellBatch];
#pragma unroll
    for (int k = 0; k < kShellBatch; ++k) {
        fx[k] = __builtin_amdgcn_fractf(gx[k]);
        fz[k] = __builtin_amdgcn_fractf(gz[k]);
        e2[k] = lds_ld_int2(med3_u32(rowy + ((uint32_t)(int)gz[k] << 3), s.tlob, s.thib));
    }
    float4 q0[kShellBatch], q1[kShellBatch];
#pragma unroll
    for (int k = 0; k < kShellBatch; ++k) {
        const uint32_t c = side_lo16(e2[k], gx[k], s.cx) + (uint32_t)(int)gx[k];
        const uint32_t a = c - plo < pn ? s.colb + (c << 4) : s.zerob;
        q0[k] = lds_ld_float4(a);
        q1[k] = lds_ld_float4(a + 16u);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < kShellBatch; ++k) v[k] = tri_blend(q0[k], q1[k], fx[k], fy, fz[k]);
}

// shell_atom<JM, true> over the resident chunk [lo, hi) of the atom's band.
template <int JM>
__device__ __forceinline__ void shell_atom_part(float (&acc)[JM], const Shell &sh,
                                                const XStage &xs, cfloat2_p cj, int jw, float ex,
                                                float ez, int lo, int hi) {
    const float fy = __builtin_amdgcn_fractf(xs.gy);
    const uint32_t rowy = shell_rowy(sh, xs.gy);
    const uint32_t plo = (uint32_t)(lo + kEntryBias), pn = (uint32_t)(hi - lo);
#pragma unroll
    for (int j0 = 0; j0 < JM; j0 += kShellBatch) {
        if (j0 < jw) {
            float gx[kShellBatch], gz[kShellBatch], v[kShellBatch];
#pragma unroll
            for (int k = 0; k < kShellBatch; ++k) {
                const float2 c = ld_cs(cj, j0 + k);
                gx[k] = align_gx(xs, c, ex);
                gz[k] = align_gz(xs, c, ez);
            }
            shell_batch_part<JM>(v, sh, gx, fy, rowy, gz, plo, pn);
#pragma unroll
            for (int k = 0; k < kShellBatch; ++k) acc[j0 + k] += v[k];
        }
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int jj = 0; jj < JM; ++jj) asm volatile("" : "+v"(acc[jj]));
}

// Copy by every wave of the workgroup (wave: its wave-uniform index of W): n16
// float4 (a whole number of 64-float4 instructions) from src in global memory to
// dst in LDS with direct global-to-LDS loads, all in flight before one wait; the
// caller's barrier then publishes them.
__device__ __forceinline__ void lds_fill(float4 *dst, const float4 *src, int n16, int wave, int W) {
    const float4 *sl = src + lane_id();
    for (int c = 64 * wave; c < n16; c += 64 * W)
        __builtin_amdgcn_global_load_lds((const void *)(sl + c),
                                         (__attribute__((address_space(3))) void *)(dst + c), 16, 0,
                                         0);
    __builtin_amdgcn_s_waitcnt(0);
}

// Float4 count of the first copy of an atom's band (c0, c1 from k_align's ainf):
// the whole band, or for a band in two chunks its table and first chunk.
__device__ __forceinline__ int band_copy16(const int4 &c0, const int4 &c1) {
    const int C1 = c1.w >> 1;
    return C1 > 0 ? band_padded(c1.z + C1) : band_padded(c0.y);
}

// Persistent workgroups pop (ligand, group of GR restarts) items of one size bin
// and write each restart's best orientation as the first entry of its decision
// trace; k_dock then starts from it.  A lane holds a strip: one restart, one x
// rotation i and JM consecutive y rotations, with JM score accumulators; strips
// are ordered (part of the y range, restart, i).  Per atom a lane rebuilds its
// restart's start-pose offset from the ligand-centred coordinates (the same
// arithmetic as start_pose), applies the x rotation once and then samples the JM
// y rotations.  The last wave streams the next atom's band into LDS.
template <int NS, int JM>
__global__ __launch_bounds__(1024) void k_align(GridArgs g, SearchArgs sa, LibArgs lib, WorkArgs ws,
                                                int bin, int lst, int arena, int GR) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int nmax = bin_nmax(bin);
    const int BD = blockDim.x, W = BD >> 6, tid = threadIdx.x, wave = tid >> 6, lane = lane_id();
    const int A = sa.A, parts = (A + JM - 1) / JM;
    float4 *xyzt = (float4 *)(smem + AlignLds::xyzt());
    float4 *dxyz = (float4 *)(smem + AlignLds::dxyz(nmax));
    float4 *ectr = (float4 *)(smem + AlignLds::ectr(nmax));
    int4 *ainf = (int4 *)(smem + AlignLds::ainf(nmax, GR));  // per atom: band copy, band rows
    int *misc = (int *)(smem + AlignLds::misc(nmax, GR));    // [0] item, bytes 64..95 zero pair
    float4 *zero2 = (float4 *)(smem + AlignLds::misc(nmax, GR) + 64);
    u64 *bestk = (u64 *)(smem + AlignLds::best(nmax, GR));
    float4 *region = (float4 *)(smem + AlignLds::region(nmax, GR));
    const int region16 = (arena - (int)AlignLds::region(nmax, GR)) / 16;
    const uint32_t region_b = lds_addr(region), zero_b = lds_addr(zero2);
    const int wave_u = uniform_int(wave);
    const Tri tr = make_tri(g);
    const int groups = (sa.R + GR - 1) / GR;
    const int Ws = W - 1;  // sampling waves; wave Ws copies bands
    const bool sampler = wave < Ws;
    // strips of one part padded to whole waves, so that j0 is wave-uniform
    const int spp = (GR * A + 63) & ~63, strips = parts * spp;
    if (tid < 2) zero2[tid] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    // Items (ligand of the list, group of GR restarts), one queue per XCD: XCD x
    // (workgroup b runs on XCD b % kXcds, the round-robin dispatch) takes the
    // x-th contiguous share of the list's ligands with all their restart groups,
    // so the groups of a ligand, which copy the same bands, read them through one
    // L2.  A workgroup whose queue is empty takes items from the next queues.
    const long long nl = ws.counters[lst];
    int *qc = ws.counters + 4 * kMaxLists + lst * kXcds;
    int qcur = (int)(blockIdx.x % kXcds), qleft = kXcds;  // thread 0's cursor
    for (;;) {
        if (tid == 0) {
            int qli = -1, qgrp = 0;
            while (qleft > 0) {
                const long long l0 = nl * qcur / kXcds, l1 = nl * (qcur + 1) / kXcds;
                const int got = atomicAdd(&qc[qcur], 1);
                if ((long long)got < (l1 - l0) * groups) {
                    qli = (int)(l0 + got / groups);
                    qgrp = got % groups;
                    break;
                }
                qcur = qcur + 1 == kXcds ? 0 : qcur + 1;
                --qleft;
            }
            misc[0] = qli;
            misc[1] = qgrp;
        }
        __syncthreads();
        const int li = misc[0], grp = misc[1];
        if (li < 0) break;
        const int l = ws.bin_list[(size_t)lst * lib.L + li];
        const int a0 = lib.atom_off[l], n = lib.atom_off[l + 1] - a0;
        const int B = lib.rot_off[l + 1] - lib.rot_off[l];
        const int rbase = grp * GR;
        for (int i = tid; i < n; i += BD) {
            const float *p = lib.xyz + 3 * (size_t)(a0 + i);
            const uint32_t toff = (uint32_t)lib.type[a0 + i] * g.type_bytes;
            xyzt[i] = make_float4(p[0], p[1], p[2], __uint_as_float(toff));
        }
        if (tid < GR) bestk[tid] = 0ull;
        __syncthreads();
        if (wave == W - 1) {
            // ligand-centred coordinates X - c0, with the c0 of start_pose
            Pose<NS> X;
#pragma unroll
            for (int q = 0; q < NS; ++q) {
                const int i = lane + 64 * q;
                const float4 v = i < n ? xyzt[i] : make_float4(0.f, 0.f, 0.f, 0.f);
                X.x[q] = v.x;
                X.y[q] = v.y;
                X.z[q] = v.z;
            }
            float c0x, c0y, c0z;
            centroid(X, n, c0x, c0y, c0z);
#pragma unroll
            for (int q = 0; q < NS; ++q) {
                const int i = lane + 64 * q;
                if (i < n)
                    dxyz[i] = make_float4(X.x[q] - c0x, X.y[q] - c0y, X.z[q] - c0z, xyzt[i].w);
            }
        }
        for (int gg = wave; gg < GR; gg += W) {
            // restarts past R (last group) repeat the group's first restart
            const int r = rbase + gg < sa.R ? rbase + gg : rbase;
            Pose<NS> Y;
            start_pose(Y, xyzt, n, r, g, sa);
            float cx, cy, cz;
            centroid(Y, n, cx, cy, cz);
            const float ex = (cx - g.ox) * g.inv_h, ey = (cy - g.oy) * g.inv_h,
                        ez = (cz - g.oz) * g.inv_h;
            if (lane == 0) {
                ectr[2 * gg] = make_float4(cx, cy, cz, 0.0f);
                ectr[2 * gg + 1] = make_float4(ex, ey, ez, 0.0f);
            }
            if (gg != 0) continue;
            // each atom's band in the atlas (radius from the group's first restart)
#pragma unroll
            for (int q = 0; q < NS; ++q) {
                const int a = lane + 64 * q;
                if (a >= n) continue;
                const float rx = (Y.x[q] - cx) * g.inv_h, ry = (Y.y[q] - cy) * g.inv_h,
                            rz = (Y.z[q] - cz) * g.inv_h;
                const float rg = sqrtf(fmaf(rx, rx, fmaf(ry, ry, rz * rz)));
                const int b = (int)(rg * (1.0f / kBandWidth));
                // clamps are the identity when the sphere stays inside [0, n-2]
                const bool inside = ball_inside(tr, ex, ey, ez, rg);
                int4 c0 = make_int4(-1, 0, 0, 0), c1 = make_int4(0, 0, 0, inside ? 1 : 0);
                if (b < g.nbands) {
                    const int4 gi = g.bands[2 * b], gj = g.bands[2 * b + 1];
                    const int size16 = gj.z / 16 + gj.y;
                    const int t = (int)(lib.type[a0 + a]);
                    if (gj.y >= 0 && band_padded(size16) <= region16) {
                        c0 = make_int4(g.blob16[t * g.nbands + b], size16, gi.x, gi.y);
                        c1 = make_int4(gi.z, gi.w, gj.z / 16, inside ? 1 : 0);
                    } else if (gj.y >= 0 && inside && gj.w > 0 &&
                               band_padded(gj.z / 16 + gj.w) <= region16 &&
                               gj.z / 16 + band_padded(gj.y - gj.w) <= region16) {
                        // too large for the region: two chunks of whole rows, columns
                        // [0, C1) and [C1, ncols), each resident with the table
                        // (c1.w: bit 0 inside, bits 1.. C1)
                        c0 = make_int4(g.blob16[t * g.nbands + b], size16, gi.x, gi.y);
                        c1 = make_int4(gi.z, gi.w, gj.z / 16, 1 | (gj.w << 1));
                    }
                }
                ainf[2 * a] = c0;
                ainf[2 * a + 1] = c1;
            }
        }
        __syncthreads();
        for (int sbase = 0; sbase < strips; sbase += Ws * 64) {
            const int wbase = __builtin_amdgcn_readfirstlane(sbase + 64 * wave);
            const int part = wbase / spp, rem = sbase + tid - part * spp;
            const bool sv = sampler && wbase < strips && rem < GR * A;
            const int rr = sv ? rem : 0;  // padding lanes repeat the part's first strip
            const int gg = rr / A, i = rr - gg * A, j0 = part * JM;
            const bool won = sampler && wbase < strips;
            const int jw_part = min(JM, A - j0);
            const int r = rbase + gg < sa.R ? rbase + gg : rbase;
            const float4 m0 = sa.smat[3 * r + 0], m1 = sa.smat[3 * r + 1], m2 = sa.smat[3 * r + 2];
            const float4 cw = ectr[2 * gg], ce = ectr[2 * gg + 1];
            const float2 ci = sa.acs[i];
            const cfloat2_p cj = (cfloat2_p)sa.acs + 2 * j0;
            float acc[JM];
#pragma unroll
            for (int jj = 0; jj < JM; ++jj) acc[jj] = 0.0f;
            // the first atom's band, at the start of the region
            int offA = 0;
            {
                const int4 c0 = ainf[0];
                if (c0.x >= 0) {
                    const int sz = band_copy16(c0, ainf[1]);
                    lds_fill(region, g.atlas + c0.x, sz, wave_u, W);
                }
            }
            __syncthreads();
            for (int a = 0; a < n; ++a) {
                const int4 cn = a + 1 < n ? ainf[2 * (a + 1)] : make_int4(-1, 0, 0, 0);
                const int4 cn1 = a + 1 < n ? ainf[2 * (a + 1) + 1] : make_int4(0, 0, 0, 0);
                const int4 c0 = ainf[2 * a], c1 = ainf[2 * a + 1];
                // A band in two chunks fills the region (its first chunk and table at
                // the start, the second chunk after the table) and is never double
                // buffered.  Where the next band (or first chunk) goes: when both fit,
                // at the other end of the region, streamed by the copier wave while
                // this atom is sampled; else at the start, copied by everyone after the
                // barrier.
                const int C1 = c1.w >> 1;
                const bool two = c0.x >= 0 && C1 > 0;
                const bool next_two = cn.x >= 0 && (cn1.w >> 1) > 0;
                const int sa_ = c0.x >= 0 ? band_padded(c0.y) : 0;
                const int sn = cn.x >= 0 ? band_copy16(cn, cn1) : 0;
                const bool dbl = cn.x >= 0 && !two && !next_two && sa_ + sn <= region16;
                const int offN = dbl ? (offA == 0 ? region16 - sn : 0) : 0;
                if (won) {
                    const float4 d = dxyz[a];
                    const int to = uniform_int(__float_as_int(d.w));
                    // the batch tests j0 < jw are made here, per atom, in scalar
                    // registers (hoisted out of the atom loop they are spilled)
                    int jw = jw_part;
                    asm volatile("" : "+s"(jw));
                    // start-pose offset of this atom for the lane's restart
                    const float yx = fmaf(m0.x, d.x, fmaf(m0.y, d.y, fmaf(m0.z, d.z, g.cx)));
                    const float yy = fmaf(m1.x, d.x, fmaf(m1.y, d.y, fmaf(m1.z, d.z, g.cy)));
                    const float yz = fmaf(m2.x, d.x, fmaf(m2.y, d.y, fmaf(m2.z, d.z, g.cz)));
                    const XStage xs = align_x((yx - cw.x) * g.inv_h, (yy - cw.y) * g.inv_h,
                                              (yz - cw.z) * g.inv_h, ci, ce.y);
                    if (c0.x >= 0) {
                        Shell sh;
                        sh.y0 = c0.z;
                        sh.z0 = c0.w;
                        sh.thy = c1.x;
                        sh.thz = c1.y;
                        sh.rows = c1.x * c1.y;
                        sh.maxcol = c0.y - c1.z - 2;  // last column pair of the band
                        sh.cx = g.acx;
                        sh.koff = (unsigned)(c0.z * c1.y + c0.w);
                        sh.table = (const int2 *)(region + offA);
                        sh.col = region + offA + c1.z;
                        sh.zero = zero2;
                        sh.zerob = zero_b;
                        shell_bytes(sh, region_b + 16u * (uint32_t)offA,
                                    region_b + 16u * (uint32_t)(offA + c1.z));
                        if (two) shell_atom_part<JM>(acc, sh, xs, cj, jw, ce.x, ce.z, 0, C1);
                        else if (c1.w) shell_atom<JM, true>(acc, sh, tr, xs, cj, jw, ce.x, ce.z, to);
                        else shell_atom<JM, false>(acc, sh, tr, xs, cj, jw, ce.x, ce.z, to);
                    } else if (c1.w) {
#pragma unroll
                        for (int jj = 0; jj < JM; ++jj) {
                            if (jj >= jw) break;
                            const float2 c = ld_cs(cj, jj);
                            acc[jj] += tri_in(tr, align_gx(xs, c, ce.x), xs.gy,
                                              align_gz(xs, c, ce.z), to);
                        }
                    } else {
#pragma unroll
                        for (int jj = 0; jj < JM; ++jj) {
                            if (jj >= jw) break;
                            const float2 c = ld_cs(cj, jj);
                            acc[jj] += tri_u(tr, align_gx(xs, c, ce.x), xs.gy,
                                             align_gz(xs, c, ce.z), to);
                        }
                    }
                } else if (wave == Ws && dbl) {
                    // copier wave: global -> LDS loads, 64 float4 per instruction (band
                    // sizes are padded to whole instructions, so every lane stays in
                    // the band's slot), then wait for them before the barrier
                    const float4 *src = g.atlas + cn.x + lane;
                    for (int c = 0; c < sn; c += 64)
                        __builtin_amdgcn_global_load_lds(
                            (const void *)(src + c),
                            (__attribute__((address_space(3))) void *)(region + offN + c), 16, 0, 0);
                    __builtin_amdgcn_s_waitcnt(0);
                }
                __syncthreads();  // every sample of atom a has read the region
                if (two) {
                    // second chunk: columns [C1, ncols) after the table, then the
                    // samples whose columns lie there
                    const int nB = band_padded(c0.y - c1.z - C1);
                    lds_fill(region + c1.z, g.atlas + c0.x + c1.z + C1, nB, wave_u, W);
                    __syncthreads();
                    if (won) {
                        const float4 d = dxyz[a];
                        int jw = jw_part;
                        asm volatile("" : "+s"(jw));
                        const float yx = fmaf(m0.x, d.x, fmaf(m0.y, d.y, fmaf(m0.z, d.z, g.cx)));
                        const float yy = fmaf(m1.x, d.x, fmaf(m1.y, d.y, fmaf(m1.z, d.z, g.cy)));
                        const float yz = fmaf(m2.x, d.x, fmaf(m2.y, d.y, fmaf(m2.z, d.z, g.cz)));
                        const XStage xs = align_x((yx - cw.x) * g.inv_h, (yy - cw.y) * g.inv_h,
                                                  (yz - cw.z) * g.inv_h, ci, ce.y);
                        Shell sh;
                        sh.y0 = c0.z;
                        sh.z0 = c0.w;
                        sh.thy = c1.x;
                        sh.thz = c1.y;
                        sh.rows = c1.x * c1.y;
                        sh.maxcol = c0.y - c1.z - 2;
                        sh.cx = g.acx;
                        sh.koff = (unsigned)(c0.z * c1.y + c0.w);
                        sh.table = (const int2 *)region;
                        sh.col = region + c1.z - C1;  // column c >= C1 at region + c1.z + (c - C1)
                        sh.zero = zero2;
                        sh.zerob = zero_b;
                        shell_bytes(sh, region_b, region_b + 16u * (uint32_t)(c1.z - C1));
                        shell_atom_part<JM>(acc, sh, xs, cj, jw, ce.x, ce.z, C1, c0.y - c1.z);
                    }
                    __syncthreads();
                }
                if (cn.x >= 0 && !dbl) {  // the next atom's band, at the start
                    lds_fill(region, g.atlas + cn.x, sn, wave_u, W);
                    __syncthreads();
                }
                offA = offN;
            }
            if (sv) {
                // best (score, then lowest index) of the strip, into its restart's slot
                u64 best = 0ull;
#pragma unroll
                for (int jj = 0; jj < JM; ++jj) {
                    const int j = j0 + jj;
                    const u64 key = j < A ? make_key(acc[jj], (uint32_t)(i * A + j)) : 0ull;
                    best = key > best ? key : best;
                }
                atomicMax(&bestk[gg], best);
            }
        }
        __syncthreads();
        if (tid < GR && rbase + tid < sa.R) {
            const int r = rbase + tid;
            ws.rtrace[trace_base(lib, sa, l) + (size_t)r * (1 + sa.P * B)] =
                (uint16_t)key_index(bestk[tid]);
        }
        __syncthreads();
    }
}

// Plain (latency) form: one ligand per launch sequence.  Workgroup r docks
// restart r; its waves split the orientations and the torsion candidates and
// agree on every decision through LDS and workgroup barriers.
template <int NS, int C>
__global__ __launch_bounds__(256) void k_plain(GridArgs g, SearchArgs sa, LibArgs lib, WorkArgs ws,
                                               const int *__restrict__ status, int l, int bin) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int nmax = bin_nmax(bin);
    const int W = blockDim.x >> 6, wave = threadIdx.x >> 6, lane = lane_id();
    if (status[l] != 0) return;
    float4 *xyzt = (float4 *)(smem + Lds::xyzt(nmax));
    const u64 *far = (const u64 *)(smem + Lds::far(nmax));
    const u64 *mask = (const u64 *)(smem + Lds::mask(nmax, NS));
    const int2 *rot = (const int2 *)(smem + Lds::rot(nmax, NS));
    int *misc = (int *)(smem + Lds::misc(nmax, NS));
    float4 *rec = (float4 *)(smem + Lds::rec(nmax, NS) + (size_t)wave * Lds::rec_stride(nmax));
    uint16_t *cand = (uint16_t *)((unsigned char *)rec + Lds::cand(nmax));
    u64 *slots = (u64 *)(smem + Lds::rec(nmax, NS) + (size_t)W * Lds::rec_stride(nmax));
    const Tri tr = make_tri(g);
    const BlockSplit sp{wave, W, slots};
    float2 cs[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int k = sp.first() + lane + sp.stride() * c;
        cs[c] = k < sa.T ? sa.tors[k] : make_float2(1.f, 0.f);
    }
    stage_ligand<NS>(smem, nmax, l, lib, ws, g, true);
    __syncthreads();
    const int r = blockIdx.x;
    const int n = misc[1], B = misc[2];
    int toff[NS];
    lane_toff(xyzt, n, toff);
    Pose<NS> Y;
    start_pose(Y, xyzt, n, r, g, sa);
    uint16_t *tr_out = ws.rtrace + trace_base(lib, sa, l) + (size_t)r * (1 + sa.P * B);
    const bool writer = threadIdx.x == 0;
    const int o = align_pose(Y, n, toff, rec, tr, g, sa, nullptr, sp);
    if (writer) tr_out[0] = (uint16_t)o;
    int d = 1;
    long long nsc = 0;  // this wave's share of the scored torsion samples
    for (int p = 0; p < sa.P; ++p) {
        for (int b = 0; b < B; ++b, ++d) {
            const int2 ab = rot[b];
            const int k = torsion_decide<NS, C>(Y, n, mask + b * NS, uniform_int(ab.x),
                                                uniform_int(ab.y), far, toff, rec, cand, cs, tr,
                                                g, sa, sp, nsc);
            if (writer) tr_out[d] = (uint16_t)k;
        }
    }
    if (ws.scored && lane == 0) atomicAdd(ws.scored, (unsigned long long)nsc);
    const float sc = pose_score(Y, n, toff, tr, g);
    if (writer) ws.rscore[(size_t)l * sa.R + r] = sc;
}

// Replay restart r of ligand l from its decision trace (same arithmetic as k_dock).
template <int NS>
__device__ void replay_pose(Pose<NS> &Y, const float4 *xyzt, const u64 *mask, const int2 *rot,
                            int n, int B, int r, const uint16_t *trace, const GridArgs &g,
                            const SearchArgs &sa) {
    const int lane = lane_id();
    start_pose(Y, xyzt, n, r, g, sa);
    // The trace and each step's (cos, sin) are loaded 64 entries at a time, one
    // entry per lane, so the replay waits for one round of loads per 64 steps
    // instead of one per step; entry 0 is the alignment, entry 1 + p*B + b the
    // step of bond b in pass p.
    const int D = 1 + sa.P * B;
    for (int base = 0; base < D; base += 64) {
        const int e = base + lane;
        const int kl = e < D ? (int)trace[e] : (int)kTraceNone;
        const float2 tl = e > 0 && kl < sa.T ? sa.tors[kl] : make_float2(1.f, 0.f);
        const int cnt = D - base < 64 ? D - base : 64;
        for (int u = 0; u < cnt; ++u) {
            const int d = base + u;
            const int k = __builtin_amdgcn_readlane(kl, u);
            if (d == 0) {
                apply_align(Y, n, k < sa.A * sa.A ? k : 0, sa);  // from k_dock; bound anyway
            } else if (k < sa.T) {
                const int b = (d - 1) % B;
                const float c = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(tl.x), u));
                const float sn = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(tl.y), u));
                const int2 ab = rot[b];
                apply_torsion(Y, mask + b * NS, bond_axis(Y, uniform_int(ab.x), uniform_int(ab.y)),
                              c, sn);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Final stage (Select Poses, then the final rigid step and score of every kept
// pose, then the outputs), as three kernels per size bin:
//   k_select: one workgroup per ligand (persistent over the bin list): ranks the
//     restarts, rebuilds candidates from their traces and keeps them greedily;
//     writes the kept poses (workspace acc_pose), their restarts and count;
//   k_falign: one wave per (ligand, kept pose) item (the grid's waves take the
//     bin's items in turn), or in the plain form one workgroup per kept pose
//     with the orientations split over its waves: alignment again about the
//     pose centroid, final score and orientation;
//   k_out: one workgroup per ligand: output order (final score desc, restart
//     asc), scores, restarts, final-step indices, and the kept poses turned by
//     their final-step orientation.
// k_select's shared memory: staged ligand, restart keys and order, selection
// scratch, then (sel_lds) the batch of candidate poses and the kept poses.

static __host__ __device__ size_t select_sel_offset(int nmax, int waves, int R, int K) {
    const int nw = (nmax + 63) / 64;
    const size_t b = Lds::rec(nmax, nw) + (size_t)R * 12 + (size_t)K * 4 + 4 +
                     (size_t)(2 * waves + 1) * 4;
    return (b + 15) & ~(size_t)15;
}

size_t select_lds_bytes(int nmax, int waves, int R, int K, int sel_lds) {
    return select_sel_offset(nmax, waves, R, K) +
           (sel_lds ? (size_t)(waves + K) * (size_t)nmax * 12 : 0);
}

int select_sel_lds(int nmax, int waves, int R, int K) {
    return select_lds_bytes(nmax, waves, R, K, 1) <= (size_t)160 * 1024 ? 1 : 0;
}

template <int NS>
__global__ __launch_bounds__(1024) void k_select(GridArgs g, SearchArgs sa, LibArgs lib,
                                                WorkArgs ws, OutArgs out, int bin, int lst, int single,
                                                int sel_lds) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int nmax = bin_nmax(bin);
    const int W = blockDim.x >> 6, wave = threadIdx.x >> 6, lane = lane_id();
    const int R = sa.R, K = sa.K;
    float4 *xyzt = (float4 *)(smem + Lds::xyzt(nmax));
    const u64 *mask = (const u64 *)(smem + Lds::mask(nmax, NS));
    const int2 *rot = (const int2 *)(smem + Lds::rot(nmax, NS));
    int *misc = (int *)(smem + Lds::misc(nmax, NS));
    unsigned char *p = smem + Lds::rec(nmax, NS);
    u64 *rkey = (u64 *)p;                     // [R]
    int *order = (int *)(p + (size_t)R * 8);  // [R]
    int *sel = (int *)(p + (size_t)R * 12);   // [K]
    int *nsel = sel + K;                      // [1]
    int *cflag = nsel + 1;                    // [W] candidate conflicts
    int *kinfo = cflag + W;                   // [1 + W] kept count, slot of each wave's candidate
    float *candL = (float *)(smem + select_sel_offset(nmax, W, R, K));  // [W][n][3]
    float *keptL = candL + (size_t)W * nmax * 3;                         // [K][n][3]

    if (single >= 0 && out.status[single] != 0) return;
    for (int pass = 0;; ++pass) {
        int l;
        if (single >= 0) {
            // plain form: exactly one ligand, given by the launch
            if (pass > 0) break;
            l = single;
        } else {
            if (threadIdx.x == 0) misc[0] = atomicAdd(&ws.counters[2 * kMaxLists + lst], 1);
            __syncthreads();
            const int li = misc[0];
            if (li >= ws.counters[lst]) break;
            l = ws.bin_list[(size_t)lst * lib.L + li];
        }
        stage_ligand<NS>(smem, nmax, l, lib, ws, g, false);
        for (int r = threadIdx.x; r < R; r += blockDim.x) {
            const float s = ws.rscore[(size_t)l * R + r];
            rkey[r] = make_key(s, (uint32_t)r);
            if (out.rscore_user) out.rscore_user[(size_t)l * R + r] = s;
        }
        __syncthreads();
        // order restarts by (score desc, restart asc): rank = number of larger keys
        for (int r = threadIdx.x; r < R; r += blockDim.x) {
            const u64 kr = rkey[r];
            int rk = 0;
            for (int q = 0; q < R; ++q) rk += rkey[q] > kr;
            order[rk] = r;
        }
        __syncthreads();
        const int n = misc[1], B = misc[2];
        const int a0 = lib.atom_off[l];
        float *accp = ws.acc_pose + (size_t)a0 * K * 3;
        const uint16_t *trl = ws.rtrace + trace_base(lib, sa, l);
        const int D = 1 + sa.P * B;
        if (sel_lds) {
            // Select Poses with every wave: per round, wave w replays the restart
            // ranked t0 + w and tests it against the poses kept so far (lanes over
            // kept poses) and against the round's earlier candidates (lanes over
            // atoms); one thread then takes the round's candidates in rank order,
            // which is the greedy rule.
            const float lim = sa.dedup2 * (float)n;
            int ns = 0;
            for (int t0 = 0; t0 < R && ns < K; t0 += W) {
                const int t = t0 + wave;
                float *cp = candL + (size_t)wave * n * 3;
                int flag = 1;  // bit 0: conflicts with a kept pose (or no candidate)
                if (t < R) {
                    const int r = order[t];
                    Pose<NS> Y;
                    replay_pose(Y, xyzt, mask, rot, n, B, r, trl + (size_t)r * D, g, sa);
#pragma unroll
                    for (int q = 0; q < NS; ++q) {
                        const int i = lane + 64 * q;
                        if (i < n) {
                            cp[3 * i + 0] = Y.x[q];
                            cp[3 * i + 1] = Y.y[q];
                            cp[3 * i + 2] = Y.z[q];
                        }
                    }
                    wave_lds_sync();
                    bool conflict = false;
                    if (sa.dedup2 > 0.f && ns > 0) {
                        const bool ks = lane < ns;
                        const float *kq = keptL + (size_t)(ks ? lane : 0) * n * 3;
                        float ssd = 0.f;
                        for (int i = 0; i < n; ++i) {
                            const float dx = cp[3 * i + 0] - kq[3 * i + 0];
                            const float dy = cp[3 * i + 1] - kq[3 * i + 1];
                            const float dz = cp[3 * i + 2] - kq[3 * i + 2];
                            ssd = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, ssd)));
                        }
                        conflict = __ballot(ks && ssd < lim) != 0ull;
                    }
                    flag = conflict ? 1 : 0;
                }
                __syncthreads();  // the round's candidates are in LDS
                if (t < R && sa.dedup2 > 0.f) {
                    for (int v = 0; v < wave; ++v) {
                        const float *vp = candL + (size_t)v * n * 3;
                        float ssd = 0.f;
#pragma unroll
                        for (int q = 0; q < NS; ++q) {
                            const int i = lane + 64 * q;
                            if (i < n) {
                                const float dx = cp[3 * i + 0] - vp[3 * i + 0];
                                const float dy = cp[3 * i + 1] - vp[3 * i + 1];
                                const float dz = cp[3 * i + 2] - vp[3 * i + 2];
                                ssd = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, ssd)));
                            }
                        }
                        if (wave_sum(ssd) < lim) flag |= 2 << v;
                    }
                }
                if (lane == 0) cflag[wave] = flag;
                __syncthreads();
                if (threadIdx.x == 0) {
                    int nn = ns, kept = 0;
                    for (int w = 0; w < W; ++w) {
                        kinfo[1 + w] = -1;
                        const int f = cflag[w];
                        if (nn >= K || (f & 1) || ((f >> 1) & kept)) continue;
                        kept |= 1 << w;
                        kinfo[1 + w] = nn;
                        sel[nn++] = order[t0 + w];
                    }
                    kinfo[0] = nn;
                }
                __syncthreads();
                const int slot = kinfo[1 + wave];
                if (slot >= 0) {
                    float *kd = keptL + (size_t)slot * n * 3;
                    for (int e = lane; e < 3 * n; e += 64) kd[e] = cp[e];
                }
                ns = kinfo[0];
                __syncthreads();
            }
            if (threadIdx.x == 0) *nsel = ns;
            // kept poses to the workspace, for k_falign
            for (int e = threadIdx.x; e < ns * n * 3; e += blockDim.x) accp[e] = keptL[e];
        } else if (wave == 0) {
            // greedy selection with plain-RMSD dedup; poses rebuilt from traces
            int ns = 0;
            const float lim = sa.dedup2 * (float)n;
            for (int t = 0; t < R && ns < K; ++t) {
                const int r = order[t];
                Pose<NS> Y;
                replay_pose(Y, xyzt, mask, rot, n, B, r, trl + (size_t)r * D, g, sa);
                bool keep = true;
                if (sa.dedup2 > 0.f) {
                    for (int s = 0; s < ns && keep; ++s) {
                        float ssd = 0.f;
#pragma unroll
                        for (int q = 0; q < NS; ++q) {
                            const int i = lane + 64 * q;
                            if (i < n) {
                                const float *P = accp + ((size_t)s * n + i) * 3;
                                const float dx = Y.x[q] - P[0], dy = Y.y[q] - P[1],
                                            dz = Y.z[q] - P[2];
                                ssd += dx * dx + dy * dy + dz * dz;
                            }
                        }
                        ssd = wave_sum(ssd);
                        if (ssd < lim) keep = false;
                    }
                }
                if (keep) {
#pragma unroll
                    for (int q = 0; q < NS; ++q) {
                        const int i = lane + 64 * q;
                        if (i < n) {
                            float *P = accp + ((size_t)ns * n + i) * 3;
                            P[0] = Y.x[q];
                            P[1] = Y.y[q];
                            P[2] = Y.z[q];
                        }
                    }
                    if (lane == 0) sel[ns] = r;
                    ++ns;
                }
            }
            if (lane == 0) *nsel = ns;
        }
        __syncthreads();
        const int ns = *nsel;
        for (int s = threadIdx.x; s < ns; s += blockDim.x) ws.sel[(size_t)l * K + s] = sel[s];
        if (threadIdx.x == 0) ws.nsel[l] = ns;
        __syncthreads();
    }
}

// Final rigid step and score of kept pose s of ligand l (Rescore Pose stand-in):
// the alignment about the pose centroid (if final_align), then the grid score,
// written to fscore / fo by the lead wave.  The kept pose itself is left as it
// is (k_out applies the chosen orientation), so the kernel can be run again on
// the same inputs.  rec: LDS for >= n float4.
template <int NS, class Split>
__device__ void final_item(int l, int s, float4 *rec, const Tri &tr, const GridArgs &g,
                           const SearchArgs &sa, const LibArgs &lib, const WorkArgs &ws,
                           const Split &sp, bool lead_wave) {
    const int lane = lane_id();
    const int a0 = lib.atom_off[l], n = lib.atom_off[l + 1] - a0;
    const float *P = ws.acc_pose + ((size_t)a0 * sa.K + (size_t)s * n) * 3;
    Pose<NS> Y;
    int toff[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        const int i = lane + 64 * q;
        const int ii = i < n ? i : 0;
        Y.x[q] = P[3 * ii + 0];
        Y.y[q] = P[3 * ii + 1];
        Y.z[q] = P[3 * ii + 2];
        toff[q] = i < n ? (int)((uint32_t)lib.type[a0 + i] * g.type_bytes) : 0;
    }
    int o = 0;
    if (sa.final_align) o = align_pose(Y, n, toff, rec, tr, g, sa, nullptr, sp);
    const float sc = pose_score(Y, n, toff, tr, g);
    if (lead_wave && lane == 0) {
        ws.fscore[(size_t)l * sa.K + s] = sc;
        ws.fo[(size_t)l * sa.K + s] = o;
    }
}

// Final step of kept poses s0 and s0 + 1 (when s0 + 1 < ns) of ligand l in one
// wave, for A <= 32 with final_align: lane (h, i) = (lane / 32, lane % 32) holds
// the strip of pose h, x rotation i and the A y rotations, one accumulator each.
// Per atom the x rotation is applied once (align_x) and each y rotation costs 4
// FMAs, and the cube loads of kFalignBatch samples are issued before the first
// blend waits for them.  Every sample, the atom-order sums and the tie rule
// (first maximum in o = i*A + j) are those of align_pose, and the chosen
// orientation is applied and scored as there, so fscore / fo are bit-identical
// to final_item's.  rec: LDS for 2 * nmax float4.
constexpr int kFalignBatch = 4;

template <int NS>
__device__ void final_pair(int l, int s0, int ns, float4 *rec, int nmax, const Tri &tr,
                           const GridArgs &g, const SearchArgs &sa, const LibArgs &lib,
                           const WorkArgs &ws) {
    const int lane = lane_id(), h = lane >> 5, i = lane & 31;
    const int a0 = lib.atom_off[l], n = lib.atom_off[l + 1] - a0, K = sa.K, A = sa.A;
    const int np = s0 + 1 < ns ? 2 : 1;
    int toff[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        const int ia = lane + 64 * q;
        toff[q] = ia < n ? (int)((uint32_t)lib.type[a0 + ia] * g.type_bytes) : 0;
    }
    // records of both poses: centred grid-unit offsets and type offsets, as in
    // align_pose; every sample inside the grid unless some atom's sphere may leave it
    float ex[2] = {0.f, 0.f}, ey[2] = {0.f, 0.f}, ez[2] = {0.f, 0.f};
    bool out_any = false;
    for (int p = 0; p < np; ++p) {
        const float *P = ws.acc_pose + ((size_t)a0 * K + (size_t)(s0 + p) * n) * 3;
        Pose<NS> Y;
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            const int ia = lane + 64 * q, ii = ia < n ? ia : 0;
            Y.x[q] = P[3 * ii + 0];
            Y.y[q] = P[3 * ii + 1];
            Y.z[q] = P[3 * ii + 2];
        }
        float cx, cy, cz;
        centroid(Y, n, cx, cy, cz);
        ex[p] = (cx - g.ox) * g.inv_h;
        ey[p] = (cy - g.oy) * g.inv_h;
        ez[p] = (cz - g.oz) * g.inv_h;
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            const int ia = lane + 64 * q;
            if (ia < n) {
                const float rx = (Y.x[q] - cx) * g.inv_h, ry = (Y.y[q] - cy) * g.inv_h,
                            rz = (Y.z[q] - cz) * g.inv_h;
                out_any = out_any || !ball_inside(tr, ex[p], ey[p], ez[p],
                                                  ball_radius(fmaf(rx, rx, fmaf(ry, ry, rz * rz))));
                rec[p * nmax + ia] = make_float4(rx, ry, rz, __int_as_float(toff[q]));
            }
        }
    }
    const bool all_in = __ballot(out_any) == 0ull;
    wave_lds_sync();
    // strips; lanes without one (i >= A, or the second pose missing) mirror a valid
    // strip so that their reads stay in range, and take no part in the maximum
    const bool valid = h < np && i < A;
    const int hp = h < np ? h : 0;
    const float pex = hp ? ex[1] : ex[0], pey = hp ? ey[1] : ey[0], pez = hp ? ez[1] : ez[0];
    const float2 ci = sa.acs[i < A ? i : 0];
    const cfloat2_p cj = (cfloat2_p)sa.acs;  // padded to 32 entries (k >= A wraps)
    const float4 *rp = rec + hp * nmax;
    float acc[32];
#pragma unroll
    for (int jj = 0; jj < 32; ++jj) acc[jj] = 0.0f;
    for (int a = 0; a < n; ++a) {
        const float4 r = rp[a];
        const int to = uniform_int(__float_as_int(rec[a].w));  // same atom, same type in both
        const XStage xs = align_x(r.x, r.y, r.z, ci, pey);
#pragma unroll
        for (int j0 = 0; j0 < 32; j0 += kFalignBatch) {
            if (j0 < A) {
                float fx[kFalignBatch], fy[kFalignBatch], fz[kFalignBatch];
                uint32_t off[kFalignBatch];
#pragma unroll
                for (int k = 0; k < kFalignBatch; ++k) {
                    const float2 c = ld_cs(cj, j0 + k);
                    const float gx = align_gx(xs, c, pex), gz = align_gz(xs, c, pez);
                    if (all_in) {
                        // tri_in's cell and fractions
                        fx[k] = __builtin_amdgcn_fractf(gx);
                        fy[k] = __builtin_amdgcn_fractf(xs.gy);
                        fz[k] = __builtin_amdgcn_fractf(gz);
                        off[k] = in_cell(tr, gx, xs.gy, gz);
                    } else {
                        // tri_u's clamped cell and fractions
                        off[k] = tri_cell(tr, gx, xs.gy, gz, fx[k], fy[k], fz[k]);
                    }
                }
                float4 q0[kFalignBatch], q1[kFalignBatch];
#pragma unroll
                for (int k = 0; k < kFalignBatch; ++k) {
                    q0[k] = ldq(tr.rs, off[k], to);
                    q1[k] = ldq(tr.rs, off[k], to + 16);
                }
                // every load of the batch is issued before the first blend waits
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int k = 0; k < kFalignBatch; ++k)
                    acc[j0 + k] += tri_blend(q0[k], q1[k], fx[k], fy[k], fz[k]);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    // best (score, then lowest index) of each pose: lane maxima, then a max over
    // each half wave (rows 0-1 into lane 31, rows 2-3 into lane 63)
    u64 best = 0ull;
#pragma unroll
    for (int jj = 0; jj < 32; ++jj) {
        const u64 key = valid && jj < A ? make_key(acc[jj], (uint32_t)(i * A + jj)) : 0ull;
        best = key > best ? key : best;
    }
#define DOCK_HALF_MAX_STEP(C, R)            \
    {                                       \
        const u64 w = dpp_read64<C, R>(best); \
        best = w > best ? w : best;         \
    }
    DOCK_HALF_MAX_STEP(0x111, 0xF)
    DOCK_HALF_MAX_STEP(0x112, 0xF)
    DOCK_HALF_MAX_STEP(0x114, 0xF)
    DOCK_HALF_MAX_STEP(0x118, 0xF)
    DOCK_HALF_MAX_STEP(0x142, 0xA)
#undef DOCK_HALF_MAX_STEP
    const u64 bk[2] = {read_lane64(best, 31), read_lane64(best, 63)};
    wave_lds_sync();  // rec is rewritten by the wave's next item
    for (int p = 0; p < np; ++p) {
        const int ob = (int)key_index(bk[p]);
        const float *P = ws.acc_pose + ((size_t)a0 * K + (size_t)(s0 + p) * n) * 3;
        Pose<NS> Y;
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            const int ia = lane + 64 * q, ii = ia < n ? ia : 0;
            Y.x[q] = P[3 * ii + 0];
            Y.y[q] = P[3 * ii + 1];
            Y.z[q] = P[3 * ii + 2];
        }
        apply_align(Y, n, ob, sa);
        const float sc = pose_score(Y, n, toff, tr, g);
        if (lane == 0) {
            ws.fscore[(size_t)l * K + s0 + p] = sc;
            ws.fo[(size_t)l * K + s0 + p] = ob;
        }
    }
}

size_t falign_lds_bytes(int nmax, int waves, int single) {
    return single ? (size_t)nmax * 16 + (size_t)waves * 8 : (size_t)waves * 2 * nmax * 16;
}

template <int NS>
__global__ __launch_bounds__(512) void k_falign(GridArgs g, SearchArgs sa, LibArgs lib,
                                               WorkArgs ws, const int *__restrict__ status,
                                               int bin, int lst, int single, int xcds) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int nmax = bin_nmax(bin);
    // every lane is active here, so the wave index is read from the first lane
    const int W = blockDim.x >> 6, wave = uniform_int((int)(threadIdx.x >> 6));
    const Tri tr = make_tri(g);
    if (single >= 0) {
        // plain form: workgroup s takes kept pose s of the ligand, its waves split
        // the orientations and agree on the best through LDS
        const int l = single, s = blockIdx.x;
        if (status[l] != 0 || s >= ws.nsel[l]) return;
        float4 *rec = (float4 *)smem;
        u64 *slots = (u64 *)(smem + (size_t)nmax * 16);
        final_item<NS>(l, s, rec, tr, g, sa, lib, ws, BlockSplit{wave, W, slots}, wave == 0);
        return;
    }
    // batched form: the waves of the grid take the bin's (ligand, kept pose)
    // items in turn (item = global wave index + k * waves in the grid).  The
    // item index is scalar arithmetic only: no lane-dependent branch precedes
    // the loop test, so every lane of a wave runs the same items.
    // With xcds > 1 the workgroups are taken as dispatched round-robin over that
    // many XCDs (workgroup b on XCD b % xcds): XCD x takes a contiguous x-th share
    // of the bin's ligands, so the kept poses of a ligand share one L2.
    // An item is a pair of kept poses (s0 = 2 * pair, s0 + 1) of one ligand.
    float4 *rec = (float4 *)(smem + (size_t)wave * 2 * nmax * 16);
    const long long nl = ws.counters[lst];
    const int x = xcds > 1 ? (int)(blockIdx.x % xcds) : 0;
    const int bx = xcds > 1 ? (int)(blockIdx.x / xcds) : (int)blockIdx.x;
    const int nbx = xcds > 1 ? (int)((gridDim.x - x + xcds - 1) / xcds) : (int)gridDim.x;
    const int nx = xcds > 1 ? xcds : 1;
    const int pairs = (sa.K + 1) / 2;
    const bool strips = sa.final_align && sa.A <= 32;
    const long long li0 = nl * x / nx, li1 = nl * (x + 1) / nx;
    const long long total = (li1 - li0) * pairs;
    const long long nwaves = (long long)nbx * W;
    for (long long item = (long long)bx * W + wave; item < total; item += nwaves) {
        const int li = (int)(li0 + item / pairs), s0 = 2 * (int)(item % pairs);
        const int l = ws.bin_list[(size_t)lst * lib.L + li];
        const int ns = ws.nsel[l];
        if (s0 >= ns) continue;
        if (strips) {
            final_pair<NS>(l, s0, ns, rec, nmax, tr, g, sa, lib, ws);
        } else {
            final_item<NS>(l, s0, rec, tr, g, sa, lib, ws, WaveSplit(), true);
            if (s0 + 1 < ns) final_item<NS>(l, s0 + 1, rec, tr, g, sa, lib, ws, WaveSplit(), true);
        }
    }
}

// Outputs of a ligand's kept poses, ordered by (final score desc, restart asc):
// each wave takes kept poses in turn, turns it by its final-step orientation
// (the same arithmetic as the alignment's own apply step) and writes it to its
// output slot.
template <int NS>
__global__ __launch_bounds__(256) void k_out(SearchArgs sa, LibArgs lib, WorkArgs ws,
                                             OutArgs out, int bin, int lst, int single) {
    __shared__ int rank[kMaxTopK];
    const int K = sa.K;
    const int W = blockDim.x >> 6, wave = threadIdx.x >> 6, lane = lane_id();
    for (int li = blockIdx.x;; li += gridDim.x) {
        int l;
        if (single >= 0) {
            if (li > 0 || out.status[single] != 0) break;
            l = single;
        } else {
            if (li >= ws.counters[lst]) break;
            l = ws.bin_list[(size_t)lst * lib.L + li];
        }
        const int a0 = lib.atom_off[l], n = lib.atom_off[l + 1] - a0;
        const int ns = ws.nsel[l];
        const float *fsc = ws.fscore + (size_t)l * K;
        const int *sel = ws.sel + (size_t)l * K;
        const int *fo = ws.fo + (size_t)l * K;
        for (int s = threadIdx.x; s < ns; s += blockDim.x) {
            const u64 ks = make_key(fsc[s], (uint32_t)sel[s]);
            int rk = 0;
            for (int q = 0; q < ns; ++q) rk += make_key(fsc[q], (uint32_t)sel[q]) > ks;
            rank[s] = rk;
            out.pscore[(size_t)l * K + rk] = fsc[s];
            out.prestart[(size_t)l * K + rk] = sel[s];
            if (out.ftrace) out.ftrace[(size_t)l * K + rk] = (uint16_t)fo[s];
            if (rk == 0) out.best[l] = fsc[s];
        }
        __syncthreads();
        const float *acc = ws.acc_pose + (size_t)a0 * K * 3;
        for (int s = wave; s < ns && out.pxyz; s += W) {
            Pose<NS> Y;
#pragma unroll
            for (int q = 0; q < NS; ++q) {
                const int i = lane + 64 * q;
                const float *P = acc + ((size_t)s * n + (i < n ? i : 0)) * 3;
                Y.x[q] = P[0];
                Y.y[q] = P[1];
                Y.z[q] = P[2];
            }
            if (sa.final_align) apply_align(Y, n, fo[s], sa);
            float *O = out.pxyz + ((size_t)a0 * K + (size_t)rank[s] * n) * 3;
#pragma unroll
            for (int q = 0; q < NS; ++q) {
                const int i = lane + 64 * q;
                if (i < n) {
                    O[3 * i + 0] = Y.x[q];
                    O[3 * i + 1] = Y.y[q];
                    O[3 * i + 2] = Y.z[q];
                }
            }
        }
        const int per = 3 * n;
        for (int e = threadIdx.x; out.pxyz && e < (K - ns) * per; e += blockDim.x)
            out.pxyz[((size_t)a0 * K + (size_t)ns * n) * 3 + e] = 0.f;
        for (int s = ns + (int)threadIdx.x; s < K; s += blockDim.x) {
            out.pscore[(size_t)l * K + s] = -INFINITY;
            out.prestart[(size_t)l * K + s] = -1;
            if (out.ftrace) out.ftrace[(size_t)l * K + s] = 0;
        }
        if (threadIdx.x == 0) {
            out.npose[l] = ns;
            if (ns == 0) out.best[l] = -INFINITY;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Pairwise rescoring stand-in (Rescore Pose): the paper evaluates every ligand
// atom against every pocket atom and accumulates the pair terms per pose; here
// the pair term is weight[ligand type][pocket atom type] for pairs closer than
// the contact distance, summed as an integer.  Pairs beyond the neighbouring
// cells of the pocket-atom cell grid are farther apart than the contact
// distance, so only the 3 x 3 rows of 3 cells around the atom are visited.

__device__ __forceinline__ int wave_sum_int(int v) {
    v += dpp_read<0x111, 0xf>(v);  // row_shr:1
    v += dpp_read<0x112, 0xf>(v);  // row_shr:2
    v += dpp_read<0x114, 0xf>(v);  // row_shr:4
    v += dpp_read<0x118, 0xf>(v);  // row_shr:8
    v += dpp_read<0x142, 0xa>(v);  // row_bcast:15
    v += dpp_read<0x143, 0xc>(v);  // row_bcast:31
    return __builtin_amdgcn_readlane(v, 63);
}

__device__ int atom_contacts(const ContactArgs &ca, const int *wrow, float px, float py,
                             float pz) {
    // cell of the atom; coordinates are clamped to one cell beyond the grid, which
    // only adds pocket atoms that fail the distance test
    const float fx = fminf(fmaxf((px - ca.lox) * ca.inv_cell, -1.f), (float)ca.cx);
    const float fy = fminf(fmaxf((py - ca.loy) * ca.inv_cell, -1.f), (float)ca.cy);
    const float fz = fminf(fmaxf((pz - ca.loz) * ca.inv_cell, -1.f), (float)ca.cz);
    const int ix = (int)floorf(fx), iy = (int)floorf(fy), iz = (int)floorf(fz);
    const int x0 = ix - 1 < 0 ? 0 : ix - 1, x1 = ix + 1 >= ca.cx ? ca.cx - 1 : ix + 1;
    int v = 0;
    if (x0 > x1) return 0;
    for (int z = iz - 1; z <= iz + 1; ++z) {
        if (z < 0 || z >= ca.cz) continue;
        for (int y = iy - 1; y <= iy + 1; ++y) {
            if (y < 0 || y >= ca.cy) continue;
            const int row = (z * ca.cy + y) * ca.cx;
            const int j1 = ca.cell_start[row + x1 + 1];
            for (int j = ca.cell_start[row + x0]; j < j1; ++j) {
                const float4 a = ca.atoms[j];
                const float dx = px - a.x, dy = py - a.y, dz = pz - a.z;
                const float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                if (d2 < ca.dc2) v += wrow[__float_as_int(a.w)];
            }
        }
    }
    return v;
}

__global__ __launch_bounds__(256) void k_rescore(ContactArgs ca, SearchArgs sa, LibArgs lib,
                                                 OutArgs out, int single) {
    __shared__ int wt[kMaxContactWeights];
    __shared__ int part[4];
    for (int e = threadIdx.x; e < ca.nw; e += blockDim.x) wt[e] = ca.weight[e];
    __syncthreads();
    const int K = sa.K;
    // every lane is active here, so the wave index is read from the first lane
    const int W = blockDim.x >> 6, wave = uniform_int((int)(threadIdx.x >> 6)), lane = lane_id();
    if (single >= 0) {
        // plain form: workgroup s scores output pose s of the ligand, its threads
        // over the ligand's atoms
        const int l = single, s = blockIdx.x;
        int v = 0;
        if (s < out.npose[l]) {
            const int a0 = lib.atom_off[l], n = lib.atom_off[l + 1] - a0;
            const float *P = out.pxyz + ((size_t)a0 * K + (size_t)s * n) * 3;
            for (int i = threadIdx.x; i < n; i += blockDim.x)
                v += atom_contacts(ca, wt + (int)lib.type[a0 + i] * ca.ntypes, P[3 * i],
                                   P[3 * i + 1], P[3 * i + 2]);
        }
        v = wave_sum_int(v);
        if (lane == 0) part[wave] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            int t = 0;
            for (int w = 0; w < W; ++w) t += part[w];
            out.pcontacts[(size_t)l * K + s] = t;
        }
        return;
    }
    // batched form: the grid's waves take the (ligand, output pose) items in turn
    const long long total = (long long)lib.L * K;
    const long long nwaves = (long long)gridDim.x * W;
    for (long long item = (long long)blockIdx.x * W + wave; item < total; item += nwaves) {
        const int l = (int)(item / K), s = (int)(item - (long long)l * K);
        int v = 0;
        if (s < out.npose[l]) {
            const int a0 = lib.atom_off[l], n = lib.atom_off[l + 1] - a0;
            const float *P = out.pxyz + ((size_t)a0 * K + (size_t)s * n) * 3;
            for (int i = lane; i < n; i += 64)
                v += atom_contacts(ca, wt + (int)lib.type[a0 + i] * ca.ntypes, P[3 * i],
                                   P[3 * i + 1], P[3 * i + 2]);
        }
        v = wave_sum_int(v);
        if (lane == 0) out.pcontacts[item] = v;
    }
}

// ---------------------------------------------------------------------------
// Preparation: one wavefront per ligand.  Checks the ligand, builds its
// bump-pair rows (pairs at least bmin bonds apart), and appends it to its size
// bin.  A ligand that fails a check gets a status and empty outputs.
__global__ __launch_bounds__(64) void k_prep(GridArgs g, SearchArgs sa, LibArgs lib, WorkArgs ws,
                                             OutArgs out, int first, int do_bin) {
    __shared__ u64 adj[kMaxAtoms * 4];   // adjacency + self rows
    const int l = first + (int)blockIdx.x;
    const int lane = lane_id();
    if (l >= lib.L) return;
    int status = 0;
    const int a0 = lib.atom_off[l], a1 = lib.atom_off[l + 1];
    const int b0 = lib.bond_off[l], b1 = lib.bond_off[l + 1];
    const int r0 = lib.rot_off[l], r1 = lib.rot_off[l + 1];
    const int n = a1 - a0, nb = b1 - b0, B = r1 - r0;
    if (a0 < 0 || a1 < a0 || (long long)a1 > lib.A_total || b0 < 0 || b1 < b0 ||
        (long long)b1 > lib.Nb_total || r0 < 0 || r1 < r0 || (long long)r1 > lib.Nr_total)
        status = 5;
    else if (n < 1 || n > kMaxAtoms || B > kMaxRot || nb > 8 * n || n > 64 * lib.mask_words)
        status = 1;
    const int NW = (n + 63) >> 6;
    if (status == 0) {
        bool bad = false;
        for (int i = lane; i < n; i += 64) bad |= (int)lib.type[a0 + i] >= g.ntypes;
        if (__ballot(bad)) status = 2;
    }
    if (status == 0) {
        for (int e = lane; e < 4 * n; e += 64) adj[e] = 0ull;
        __syncthreads();
        for (int i = lane; i < n; i += 64) atomicOr(&adj[i * 4 + (i >> 6)], 1ull << (i & 63));
        bool bad = false;
        for (int e = lane; e < nb; e += 64) {
            const int u = lib.bond[2 * (size_t)(b0 + e)], v = lib.bond[2 * (size_t)(b0 + e) + 1];
            if (u < 0 || v < 0 || u >= n || v >= n || u == v) {
                bad = true;
            } else {
                atomicOr(&adj[u * 4 + (v >> 6)], 1ull << (v & 63));
                atomicOr(&adj[v * 4 + (u >> 6)], 1ull << (u & 63));
            }
        }
        for (int e = lane; e < B; e += 64) {
            const int a = lib.rot_bond[2 * (size_t)(r0 + e)], b = lib.rot_bond[2 * (size_t)(r0 + e) + 1];
            if (a < 0 || b < 0 || a >= n || b >= n || a == b) bad = true;
        }
        if (__ballot(bad)) status = 3;
        __syncthreads();
    }
    if (status == 0) {
        // every rotatable bond is a bond
        bool bad = false;
        for (int e = lane; e < B; e += 64) {
            const int a = lib.rot_bond[2 * (size_t)(r0 + e)], b = lib.rot_bond[2 * (size_t)(r0 + e) + 1];
            bad |= !((adj[a * 4 + (b >> 6)] >> (b & 63)) & 1ull);
        }
        if (__ballot(bad)) status = 3;
    }
    if (status == 0) {
        // connected: closure of {0} under adjacency
        u64 reach[4] = {1ull, 0ull, 0ull, 0ull};
        for (int it = 0; it < n; ++it) {
            u64 nr[4] = {0ull, 0ull, 0ull, 0ull};
            for (int i = lane; i < n; i += 64)
                if ((reach[i >> 6] >> (i & 63)) & 1ull)
                    for (int w = 0; w < NW; ++w) nr[w] |= adj[i * 4 + w];
            bool changed = false;
            for (int w = 0; w < NW; ++w) {
                nr[w] = wave_or_u64(nr[w]) | reach[w];
                changed |= nr[w] != reach[w];
                reach[w] = nr[w];
            }
            if (!changed) break;
        }
        int cnt = 0;
        for (int w = 0; w < NW; ++w) cnt += __popcll(reach[w]);
        if (cnt != n) status = 4;
    }
    if (status == 0) {
        // each mask: contains b, not a, no bit >= n, and no bond other than a-b crosses it
        bool bad = false;
        for (int rb = 0; rb < B && !bad; ++rb) {
            const int a = lib.rot_bond[2 * (size_t)(r0 + rb)], b = lib.rot_bond[2 * (size_t)(r0 + rb) + 1];
            u64 m[4] = {0ull, 0ull, 0ull, 0ull};
            for (int w = 0; w < lib.mask_words && w < 4; ++w)
                m[w] = lib.rot_mask[(size_t)(r0 + rb) * lib.mask_words + w];
            for (int w = NW; w < lib.mask_words; ++w)
                if (lib.rot_mask[(size_t)(r0 + rb) * lib.mask_words + w] != 0ull) bad = true;
            if ((n & 63) != 0 && (m[NW - 1] >> (n & 63)) != 0ull) bad = true;
            if (!((m[b >> 6] >> (b & 63)) & 1ull) || ((m[a >> 6] >> (a & 63)) & 1ull)) bad = true;
            bool cross = false;
            for (int e = lane; e < nb; e += 64) {
                const int u = lib.bond[2 * (size_t)(b0 + e)], v = lib.bond[2 * (size_t)(b0 + e) + 1];
                if ((u == a && v == b) || (u == b && v == a)) continue;
                const bool su = (m[u >> 6] >> (u & 63)) & 1ull, sv = (m[v >> 6] >> (v & 63)) & 1ull;
                cross |= su != sv;
            }
            if (__ballot(cross)) bad = true;
        }
        if (bad) status = 4;
    }
    if (status == 0) {
        // rows of atoms within bmin-1 bonds, complemented: the bump-checked pairs
        for (int i = lane; i < n; i += 64) {
            u64 near[4] = {0ull, 0ull, 0ull, 0ull};
            near[i >> 6] = 1ull << (i & 63);
            for (int step = 1; step < sa.bmin; ++step) {
                u64 nx[4] = {near[0], near[1], near[2], near[3]};
                for (int w = 0; w < NW; ++w) {
                    u64 bits = near[w];
                    while (bits) {
                        const int j = 64 * w + __ffsll((long long)bits) - 1;
                        bits &= bits - 1;
                        for (int v = 0; v < NW; ++v) nx[v] |= adj[j * 4 + v];
                    }
                }
                for (int w = 0; w < 4; ++w) near[w] = nx[w];
            }
            for (int w = 0; w < kFarWords; ++w) {
                u64 valid = 0ull;
                if (w < NW) valid = (w == NW - 1 && (n & 63)) ? ((1ull << (n & 63)) - 1) : ~0ull;
                ws.far[(size_t)(a0 + i) * kFarWords + w] = ~near[w] & valid;
            }
        }
        if (lane == 0 && do_bin) {
            // work list: the atom bin, or with sa.groups > 1 the paper's bucket of
            // (atom bin, group of 4 rotatable bonds; the last group takes the rest)
            const int bin = (n - 1) >> 5;
            const int grp = B / 4 < sa.groups - 1 ? B / 4 : sa.groups - 1;
            const int lst = bin * sa.groups + grp;
            const int pos = atomicAdd(&ws.counters[lst], 1);
            ws.bin_list[(size_t)lst * lib.L + pos] = l;
        }
    } else {
        for (int s = lane; s < sa.K; s += 64) {
            out.pscore[(size_t)l * sa.K + s] = -INFINITY;
            out.prestart[(size_t)l * sa.K + s] = -1;
            if (out.ftrace) out.ftrace[(size_t)l * sa.K + s] = 0;
        }
        if (lane == 0) {
            out.best[l] = -INFINITY;
            out.npose[l] = 0;
        }
    }
    if (lane == 0) out.status[l] = status;
}

hipError_t launch_rescore(const ContactArgs &ca, const SearchArgs &sa, const LibArgs &lib,
                          const OutArgs &out, int single, int blocks, hipStream_t s) {
    if (single >= 0) blocks = sa.K;
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rescore, dim3(blocks), dim3(256), 0, s, ca, sa, lib, out, single);
    return hipGetLastError();
}

// Zero counters [first, first + count): work-queue counters are cleared by a
// kernel, not a memset, so the sequence can be captured in a graph.
__global__ void k_reset(int *counters, int first, int count) {
    for (int i = threadIdx.x; i < count; i += blockDim.x) counters[first + i] = 0;
}

// ---------------------------------------------------------------------------
// launchers
hipError_t launch_build_cubes(const float *values, float4 *cubes, int ntypes, int nx, int ny,
                              int nz, hipStream_t s) {
    const long long n = (long long)ntypes * nx * ny * nz;
    const int threads = 256;
    const long long blocks = (n + threads - 1) / threads;
    hipLaunchKernelGGL(k_build_cubes, dim3((unsigned)blocks), dim3(threads), 0, s, values, cubes,
                       ntypes, nx, ny, nz);
    return hipGetLastError();
}

hipError_t launch_atlas_count(const GridArgs &g, int4 *info, hipStream_t s) {
    hipLaunchKernelGGL(k_atlas_count, dim3(kMaxBands), dim3(1024), 0, s, g, info);
    return hipGetLastError();
}

hipError_t launch_atlas_fill(const GridArgs &g, int4 *info, const int *blob16, float4 *atlas,
                             int nb, hipStream_t s) {
    if (nb <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_atlas_fill, dim3(nb * g.ntypes), dim3(1024), 0, s, g, info, blob16, atlas,
                       nb);
    return hipGetLastError();
}

hipError_t launch_reset(int *counters, int first, int count, hipStream_t s) {
    if (first < 0 || count < 0 || first + count > kNumCounters) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(256), 0, s, counters, first, count);
    return hipGetLastError();
}

hipError_t launch_prep(const GridArgs &g, const SearchArgs &sa, const LibArgs &lib,
                       const WorkArgs &ws, const OutArgs &out, hipStream_t s) {
    if (lib.L <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_prep, dim3(lib.L), dim3(64), 0, s, g, sa, lib, ws, out, 0, 1);
    return hipGetLastError();
}

hipError_t launch_prep_one(const GridArgs &g, const SearchArgs &sa, const LibArgs &lib,
                           const WorkArgs &ws, const OutArgs &out, int l, hipStream_t s) {
    hipLaunchKernelGGL(k_prep, dim3(1), dim3(64), 0, s, g, sa, lib, ws, out, l, 0);
    return hipGetLastError();
}

size_t plain_lds_bytes(int nmax, int waves) { return dock_lds_bytes(nmax, waves) + (size_t)waves * 8; }

template <int NS, int C>
static hipError_t launch_plain_t(int l, int bin, int waves, const GridArgs &g,
                                 const SearchArgs &sa, const LibArgs &lib, const WorkArgs &ws,
                                 const OutArgs &out, hipStream_t s) {
    const size_t lds = plain_lds_bytes(bin_nmax(bin), waves);
    hipFuncSetAttribute((const void *)k_plain<NS, C>, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)lds);
    hipLaunchKernelGGL((k_plain<NS, C>), dim3(sa.R), dim3(64 * waves), lds, s, g, sa, lib, ws,
                       (const int *)out.status, l, bin);
    return hipGetLastError();
}

template <int NS>
static hipError_t launch_plain_c(int l, int bin, int waves, const GridArgs &g,
                                 const SearchArgs &sa, const LibArgs &lib, const WorkArgs &ws,
                                 const OutArgs &out, hipStream_t s) {
    const int C = (sa.T + 64 * waves - 1) / (64 * waves);
    if (C <= 1) return launch_plain_t<NS, 1>(l, bin, waves, g, sa, lib, ws, out, s);
    if (C <= 2) return launch_plain_t<NS, 2>(l, bin, waves, g, sa, lib, ws, out, s);
    return launch_plain_t<NS, 4>(l, bin, waves, g, sa, lib, ws, out, s);
}

hipError_t launch_plain(int l, int bin, int waves, const GridArgs &g, const SearchArgs &sa,
                        const LibArgs &lib, const WorkArgs &ws, const OutArgs &out,
                        hipStream_t s) {
    switch (bin_slots(bin)) {
        case 1: return launch_plain_c<1>(l, bin, waves, g, sa, lib, ws, out, s);
        case 2: return launch_plain_c<2>(l, bin, waves, g, sa, lib, ws, out, s);
        case 3: return launch_plain_c<3>(l, bin, waves, g, sa, lib, ws, out, s);
        default: return launch_plain_c<4>(l, bin, waves, g, sa, lib, ws, out, s);
    }
}

template <int NS, int C>
static hipError_t launch_dock_t(int bin, int lst, int blocks, int waves, const GridArgs &g,
                                const SearchArgs &sa, const LibArgs &lib, const WorkArgs &ws,
                                hipStream_t s) {
    const size_t lds = dock_lds_bytes(bin_nmax(bin), waves);
    hipFuncSetAttribute((const void *)k_dock<NS, C>, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)lds);
    hipLaunchKernelGGL((k_dock<NS, C>), dim3(blocks), dim3(64 * waves), lds, s, g, sa, lib, ws, bin,
                       lst);
    return hipGetLastError();
}

template <int NS>
static hipError_t launch_dock_c(int bin, int lst, int blocks, int waves, const GridArgs &g,
                                const SearchArgs &sa, const LibArgs &lib, const WorkArgs &ws,
                                hipStream_t s) {
    const int C = (sa.T + 63) / 64;
    if (C <= 1) return launch_dock_t<NS, 1>(bin, lst, blocks, waves, g, sa, lib, ws, s);
    if (C <= 2) return launch_dock_t<NS, 2>(bin, lst, blocks, waves, g, sa, lib, ws, s);
    if (C <= 4) return launch_dock_t<NS, 4>(bin, lst, blocks, waves, g, sa, lib, ws, s);
    if (C <= 8) return launch_dock_t<NS, 8>(bin, lst, blocks, waves, g, sa, lib, ws, s);
    return launch_dock_t<NS, 16>(bin, lst, blocks, waves, g, sa, lib, ws, s);
}

hipError_t launch_dock(int bin, int lst, int blocks, int waves, const GridArgs &g,
                       const SearchArgs &sa, const LibArgs &lib, const WorkArgs &ws, hipStream_t s) {
    switch (bin_slots(bin)) {
        case 1: return launch_dock_c<1>(bin, lst, blocks, waves, g, sa, lib, ws, s);
        case 2: return launch_dock_c<2>(bin, lst, blocks, waves, g, sa, lib, ws, s);
        case 3: return launch_dock_c<3>(bin, lst, blocks, waves, g, sa, lib, ws, s);
        default: return launch_dock_c<4>(bin, lst, blocks, waves, g, sa, lib, ws, s);
    }
}

template <int NS>
static hipError_t launch_select_t(int bin, int lst, int blocks, int waves, const GridArgs &g,
                                  const SearchArgs &sa, const LibArgs &lib, const WorkArgs &ws,
                                  const OutArgs &out, int single, hipStream_t s) {
    const int sel = select_sel_lds(bin_nmax(bin), waves, sa.R, sa.K);
    const size_t lds = select_lds_bytes(bin_nmax(bin), waves, sa.R, sa.K, sel);
    hipFuncSetAttribute((const void *)k_select<NS>, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)lds);
    hipLaunchKernelGGL((k_select<NS>), dim3(blocks), dim3(64 * waves), lds, s, g, sa, lib, ws, out,
                       bin, lst, single, sel);
    return hipGetLastError();
}

hipError_t launch_select(int bin, int lst, int blocks, int waves, const GridArgs &g,
                         const SearchArgs &sa, const LibArgs &lib, const WorkArgs &ws,
                         const OutArgs &out, int single, hipStream_t s) {
    switch (bin_slots(bin)) {
        case 1: return launch_select_t<1>(bin, lst, blocks, waves, g, sa, lib, ws, out, single, s);
        case 2: return launch_select_t<2>(bin, lst, blocks, waves, g, sa, lib, ws, out, single, s);
        case 3: return launch_select_t<3>(bin, lst, blocks, waves, g, sa, lib, ws, out, single, s);
        default: return launch_select_t<4>(bin, lst, blocks, waves, g, sa, lib, ws, out, single, s);
    }
}

template <int NS>
static hipError_t launch_falign_t(int bin, int lst, int blocks, int waves, const GridArgs &g,
                                  const SearchArgs &sa, const LibArgs &lib, const WorkArgs &ws,
                                  const OutArgs &out, int single, int xcds, hipStream_t s) {
    const size_t lds = falign_lds_bytes(bin_nmax(bin), waves, single >= 0 ? 1 : 0);
    hipFuncSetAttribute((const void *)k_falign<NS>, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)lds);
    hipLaunchKernelGGL((k_falign<NS>), dim3(blocks), dim3(64 * waves), lds, s, g, sa, lib, ws,
                       (const int *)out.status, bin, lst, single, xcds);
    return hipGetLastError();
}

hipError_t launch_falign(int bin, int lst, int blocks, int waves, const GridArgs &g,
                         const SearchArgs &sa, const LibArgs &lib, const WorkArgs &ws,
                         const OutArgs &out, int single, int xcds, hipStream_t s) {
    switch (bin_slots(bin)) {
        case 1: return launch_falign_t<1>(bin, lst, blocks, waves, g, sa, lib, ws, out, single, xcds, s);
        case 2: return launch_falign_t<2>(bin, lst, blocks, waves, g, sa, lib, ws, out, single, xcds, s);
        case 3: return launch_falign_t<3>(bin, lst, blocks, waves, g, sa, lib, ws, out, single, xcds, s);
        default: return launch_falign_t<4>(bin, lst, blocks, waves, g, sa, lib, ws, out, single, xcds, s);
    }
}

hipError_t launch_out(int bin, int lst, int blocks, const SearchArgs &sa, const LibArgs &lib,
                      const WorkArgs &ws, const OutArgs &out, int single, hipStream_t s) {
#define DOCK_OUT_LAUNCH(NS) \
    hipLaunchKernelGGL(k_out<NS>, dim3(blocks), dim3(256), 0, s, sa, lib, ws, out, bin, lst, single)
    switch (bin_slots(bin)) {
        case 1: DOCK_OUT_LAUNCH(1); break;
        case 2: DOCK_OUT_LAUNCH(2); break;
        case 3: DOCK_OUT_LAUNCH(3); break;
        default: DOCK_OUT_LAUNCH(4); break;
    }
#undef DOCK_OUT_LAUNCH
    return hipGetLastError();
}

// k_align geometry: JM = kAlignJ y rotations per lane, the y range in
// parts = ceil(A / JM) pieces, GR restarts per item so that the parts, each of
// GR*A strips padded to whole waves, fill the 15 sampling waves (GR at most
// kAlignMaxGroup and R, at least 1).
static int align_parts(int A) { return (A + kAlignJ - 1) / kAlignJ; }

int align_group(int A, int R) {
    const int parts = align_parts(A);
    int GR = 1;
    while (GR < kAlignMaxGroup && GR < R && parts * (((GR + 1) * A + 63) & ~63) <= 15 * 64) ++GR;
    return GR;
}

// Sampling waves (enough for the strips, at most 15) plus the copier wave.
static int align_waves(int A, int R) {
    const int strips = align_parts(A) * ((align_group(A, R) * A + 63) & ~63);
    const int w = strips / 64;
    return (w > 15 ? 15 : w) + 1;
}

size_t align_lds_min(int bin, int A, int R) {
    return AlignLds::region(bin_nmax(bin), align_group(A, R)) + 1024;
}

template <int NS>
static hipError_t launch_align_t(int bin, int lst, int blocks, int arena, const GridArgs &g,
                                 const SearchArgs &sa, const LibArgs &lib, const WorkArgs &ws,
                                 hipStream_t s) {
    hipFuncSetAttribute((const void *)k_align<NS, kAlignJ>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, arena);
    hipLaunchKernelGGL((k_align<NS, kAlignJ>), dim3(blocks), dim3(64 * align_waves(sa.A, sa.R)),
                       (size_t)arena, s, g, sa, lib, ws, bin, lst, arena, align_group(sa.A, sa.R));
    return hipGetLastError();
}

hipError_t launch_align(int bin, int lst, int blocks, int arena, const GridArgs &g,
                        const SearchArgs &sa, const LibArgs &lib, const WorkArgs &ws,
                        hipStream_t s) {
    switch (bin_slots(bin)) {
        case 1: return launch_align_t<1>(bin, lst, blocks, arena, g, sa, lib, ws, s);
        case 2: return launch_align_t<2>(bin, lst, blocks, arena, g, sa, lib, ws, s);
        case 3: return launch_align_t<3>(bin, lst, blocks, arena, g, sa, lib, ws, s);
        default: return launch_align_t<4>(bin, lst, blocks, arena, g, sa, lib, ws, s);
    }
}

template <int NS>
static int align_occ_t(int waves, int arena) {
    int nb = 0;
    hipFuncSetAttribute((const void *)k_align<NS, kAlignJ>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, arena);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_align<NS, kAlignJ>, 64 * waves,
                                                     (size_t)arena) != hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

int align_blocks_per_cu(int bin, int R, int A, int arena) {
    const int waves = align_waves(A, R);
    switch (bin_slots(bin)) {
        case 1: return align_occ_t<1>(waves, arena);
        case 2: return align_occ_t<2>(waves, arena);
        case 3: return align_occ_t<3>(waves, arena);
        default: return align_occ_t<4>(waves, arena);
    }
}

template <int NS, int C>
static int dock_occ(int bin, int waves) {
    int nb = 0;
    const size_t lds = dock_lds_bytes(bin_nmax(bin), waves);
    hipFuncSetAttribute((const void *)k_dock<NS, C>, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)lds);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_dock<NS, C>, 64 * waves, lds) !=
        hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

template <int NS>
static int dock_occ_c(int bin, int waves, int T) {
    const int C = (T + 63) / 64;
    if (C <= 1) return dock_occ<NS, 1>(bin, waves);
    if (C <= 2) return dock_occ<NS, 2>(bin, waves);
    if (C <= 4) return dock_occ<NS, 4>(bin, waves);
    if (C <= 8) return dock_occ<NS, 8>(bin, waves);
    return dock_occ<NS, 16>(bin, waves);
}

int dock_blocks_per_cu(int bin, int waves, int T) {
    switch (bin_slots(bin)) {
        case 1: return dock_occ_c<1>(bin, waves, T);
        case 2: return dock_occ_c<2>(bin, waves, T);
        case 3: return dock_occ_c<3>(bin, waves, T);
        default: return dock_occ_c<4>(bin, waves, T);
    }
}

template <int NS>
static int select_occ(int bin, int waves, int R, int K) {
    int nb = 0;
    const size_t lds = select_lds_bytes(bin_nmax(bin), waves, R, K,
                                        select_sel_lds(bin_nmax(bin), waves, R, K));
    hipFuncSetAttribute((const void *)k_select<NS>, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)lds);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_select<NS>, 64 * waves, lds) !=
        hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

int select_blocks_per_cu(int bin, int waves, int R, int K) {
    switch (bin_slots(bin)) {
        case 1: return select_occ<1>(bin, waves, R, K);
        case 2: return select_occ<2>(bin, waves, R, K);
        case 3: return select_occ<3>(bin, waves, R, K);
        default: return select_occ<4>(bin, waves, R, K);
    }
}

template <int NS>
static int falign_occ(int bin, int waves) {
    int nb = 0;
    const size_t lds = falign_lds_bytes(bin_nmax(bin), waves, 0);
    hipFuncSetAttribute((const void *)k_falign<NS>, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)lds);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_falign<NS>, 64 * waves, lds) !=
        hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

int falign_blocks_per_cu(int bin, int waves) {
    switch (bin_slots(bin)) {
        case 1: return falign_occ<1>(bin, waves);
        case 2: return falign_occ<2>(bin, waves);
        case 3: return falign_occ<3>(bin, waves);
        default: return falign_occ<4>(bin, waves);
    }
}

}  // namespace dockgpu
