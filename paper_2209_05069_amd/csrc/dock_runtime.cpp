// dock_runtime.cpp -- host side of the C ABI declared in include/dock.h.
//
// Responsibilities: argument checks, pocket residency (one device copy of each
// pocket's grids, shared by all work; the paper keeps the pocket read-only and
// shared by every host thread of a GPU), the small per-call tables (start
// rotations, alignment rotations, torsion cos/sin, computed in double and
// rounded to float), per-stream workspaces, the launch sequence
// (reset -> prep -> dock per size bin -> select/final per size bin), and the
// asynchronous submit/poll path with free-memory admission.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>
#include <array>
#include <chrono>
#include <thread>

#include "dock.h"
#include "dock_internal.h"

using namespace dockgpu;

// Scratch memory of dock_ligands_batch_noalloc (for callers that cannot
// allocate device memory): the call's tables and workspace live in this array.
// Host code never passes the array's name to a kernel or a copy (on the host it
// is only a stand-in for the symbol); dock_create looks up its address on each
// device once, and the entry point uses that address.
static __device__ __align__(256) unsigned char scratch[DOCK_NOALLOC_SCRATCH_BYTES];

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                \
    do {                                                                             \
        hipError_t e_ = (expr);                                                      \
        if (e_ != hipSuccess)                                                        \
            return fail(DOCK_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)


std::mutex g_scratch_mu;
std::map<int, char *> g_scratch_ptr;  // device -> address of its copy of `scratch`

// Address of `scratch` on `device` (the current device), looked up once.
int scratch_address(int device, char **out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    if (it == g_scratch_ptr.end()) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || ptr == nullptr) {
            (void)hipGetLastError();
            return fail(DOCK_EDEVICE, std::string("scratch symbol lookup failed: ") +
                                          hipGetErrorString(e));
        }
        it = g_scratch_ptr.emplace(device, (char *)ptr).first;
    }
    *out = it->second;
    return DOCK_OK;
}

struct Pocket {
    float4 *d_cubes = nullptr;
    float4 *d_atlas = nullptr;
    int4 *d_bands = nullptr;
    int *d_blob16 = nullptr;
    void *d_contacts = nullptr;  // pocket atoms, cell starts and weights (rescoring)
    GridArgs g{};
    ContactArgs ca{};
    bool has_atoms = false;
    int busy = 0;
    void release_atoms() {
        hipFree(d_contacts);
        d_contacts = nullptr;
        has_atoms = false;
        ca = ContactArgs{};
    }
    void release() {
        hipFree(d_cubes);
        hipFree(d_atlas);
        hipFree(d_bands);
        hipFree(d_blob16);
        release_atoms();
        d_cubes = d_atlas = nullptr;
        d_bands = nullptr;
        d_blob16 = nullptr;
    }
};

struct Workspace {
    void *base = nullptr;
    size_t bytes = 0;
};

struct Tables {
    void *d = nullptr;
    const float4 *smat = nullptr;
    const float4 *amat = nullptr;
    const float2 *tors = nullptr;
    const float2 *acs = nullptr;
};

// Tile choice of one size bin for the batched kernels (per-bin autotuner).
struct BinShape {
    int dock_waves = 4;     // k_dock: waves (restarts of one ligand) per workgroup
    int select_waves = 4;   // k_select: waves per workgroup
    int falign_waves = 4;   // k_falign: waves per workgroup
    int falign_per_cu = 0;  // k_falign: workgroups per CU (0: as many as fit)
    int falign_xcd = 0;     // k_falign: 1 = each XCD takes a contiguous share of ligands
};

// Host image of a Tables allocation (offsets relative to its start).
struct TableBlob {
    std::vector<char> bytes;
    size_t o_smat = 0, o_amat = 0, o_tors = 0, o_acs = 0;
};

struct Ticket {
    hipEvent_t done = nullptr;
    int32_t pocket = -1;
    dock_results user{};
    int L = 0, K = 0, R = 0;
    long long A = 0, trace_len = 0;
    void *pinned = nullptr;          // pinned inputs followed by the results
    size_t pinned_cap = 0;           // its capacity (it returns to the pinned pool)
    void *host_stage = nullptr;      // results part of `pinned`
    size_t dev_bytes = 0;            // device memory held until the ticket retires
    hipStream_t stream = nullptr;    // submit stream the request runs on
    size_t stage_bytes = 0;
    // offsets of the result arrays inside host_stage
    size_t o_best, o_np, o_st, o_ps, o_pr, o_xyz, o_rs, o_tr, o_ft, o_pc;
};

}  // namespace

struct dock_ctx {
    int device = 0;
    int num_cu = 0;
    int lds_arena = 0;  // LDS bytes per workgroup of the alignment kernel
    unsigned long long *d_scored = nullptr;  // scored torsion samples while timing is on
    std::mutex mu;
    std::map<int32_t, Pocket> pockets;
    int32_t next_pocket = 1;
    std::map<hipStream_t, Workspace> ws;
    std::map<std::string, Tables> tables;
    // dock_ligands_batch_noalloc: host images of the tables it copied into the
    // scratch array, kept until destroy so no asynchronous copy outlives its source
    std::map<std::string, TableBlob> noalloc_tables;
    char *scratch = nullptr;  // this device's copy of the scratch array
    std::map<std::string, int> occ;
    // per-bin tile choices of dock_autotune, by (R, T, A, K, P)
    std::map<std::string, std::array<BinShape, kNumBins>> tuned;
    std::vector<hipStream_t> submit_streams;  // dock_submit: requests round-robin over these
    size_t next_submit = 0;
    std::map<uint64_t, Ticket> tickets;
    // pinned staging buffers of retired tickets, kept for reuse: capacity -> buffer
    std::multimap<size_t, void *> pinned_pool;
    size_t pinned_pool_bytes = 0;
    uint64_t next_ticket = 1;
    size_t reserve_bytes = (size_t)1 << 30;
    size_t budget = 0;         // dock_submit admission budget (0: free memory less the reserve)
    size_t inflight = 0;       // device bytes of admitted tickets not yet retired
    std::map<hipStream_t, int> stream_tickets;  // tickets in flight per submit stream
    bool timing = false;
    // Batched launch sequences seen once (eager) and captured as graphs when they
    // repeat with identical arguments.
    std::map<std::string, int> seen_keys;
    std::map<std::string, hipGraphExec_t> graphs;
    std::vector<hipStream_t> plain_streams;  // plain form: ligands round-robin over these
    std::vector<hipEvent_t> plain_events;
    // per call: start, after prep, after the alignment kernels, after dock, end
    std::vector<std::array<hipEvent_t, 5>> marks;
};

namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int check_params(const dock_params *p) {
    if (!p) return fail(DOCK_EINVAL, "params is NULL");
    if (p->restarts < 1 || p->restarts > 4096) return fail(DOCK_EINVAL, "restarts must be in [1,4096]");
    if (p->torsion_steps < 1 || p->torsion_steps > DOCK_MAX_TORSION_STEPS)
        return fail(DOCK_EINVAL, "torsion_steps must be in [1,1024]");
    if (p->sweep_passes < 0 || p->sweep_passes > 16) return fail(DOCK_EINVAL, "sweep_passes must be in [0,16]");
    if (p->align_steps < 1 || p->align_steps > DOCK_MAX_ALIGN_STEPS)
        return fail(DOCK_EINVAL, "align_steps must be in [1,255]");
    if (p->top_k < 1 || p->top_k > DOCK_MAX_TOP_K) return fail(DOCK_EINVAL, "top_k must be in [1,64]");
    if (p->final_align != 0 && p->final_align != 1) return fail(DOCK_EINVAL, "final_align must be 0 or 1");
    if (p->bump_min_bonds < 1 || p->bump_min_bonds > DOCK_MAX_ATOMS)
        return fail(DOCK_EINVAL, "bump_min_bonds must be in [1,256]");
    if (!(p->bump_dist >= 0.f) || !std::isfinite(p->bump_dist)) return fail(DOCK_EINVAL, "bump_dist must be finite and >= 0");
    if (!(p->dedup_rmsd >= 0.f) || !std::isfinite(p->dedup_rmsd)) return fail(DOCK_EINVAL, "dedup_rmsd must be finite and >= 0");
    if (p->mode != DOCK_MODE_BATCHED && p->mode != DOCK_MODE_PLAIN) return fail(DOCK_EINVAL, "unknown mode");
    if (p->bump_prune != 0 && p->bump_prune != 1) return fail(DOCK_EINVAL, "bump_prune must be 0 or 1");
    if (p->bin_mode != 0 && p->bin_mode != 1) return fail(DOCK_EINVAL, "bin_mode must be 0 or 1");
    if (!p->start_quat) return fail(DOCK_EINVAL, "start_quat is NULL");
    for (int r = 0; r < p->restarts; ++r) {
        double s = 0;
        for (int a = 0; a < 4; ++a) {
            const double v = p->start_quat[4 * r + a];
            if (!std::isfinite(v)) return fail(DOCK_EINVAL, "start_quat has a non-finite value");
            s += v * v;
        }
        if (s < 1e-12) return fail(DOCK_EINVAL, "start_quat has a zero quaternion");
    }
    return DOCK_OK;
}

int check_library_shape(const dock_library *lib) {
    if (!lib) return fail(DOCK_EINVAL, "library is NULL");
    if (lib->n_ligands < 0) return fail(DOCK_EINVAL, "n_ligands < 0");
    if (lib->mask_words < 1 || lib->mask_words > 4) return fail(DOCK_EINVAL, "mask_words must be in [1,4]");
    if (lib->n_atoms_total < 0 || lib->n_bonds_total < 0 || lib->n_rot_total < 0)
        return fail(DOCK_EINVAL, "negative totals");
    if (lib->n_atoms_total >= ((long long)1 << 31) || lib->n_bonds_total >= ((long long)1 << 31) ||
        lib->n_rot_total >= ((long long)1 << 31))
        return fail(DOCK_EINVAL, "totals must be below 2^31 (int32 offsets)");
    if (lib->n_ligands > 0) {
        if (!lib->atom_off || !lib->bond_off || !lib->rot_off)
            return fail(DOCK_EINVAL, "offset array is NULL");
        if (lib->n_atoms_total > 0 && (!lib->xyz || !lib->type)) return fail(DOCK_EINVAL, "xyz/type is NULL");
        if (lib->n_bonds_total > 0 && !lib->bond) return fail(DOCK_EINVAL, "bond is NULL");
        if (lib->n_rot_total > 0 && (!lib->rot_bond || !lib->rot_mask))
            return fail(DOCK_EINVAL, "rot_bond/rot_mask is NULL");
    }
    return DOCK_OK;
}

int check_results(const dock_results *o, int n_ligands) {
    if (!o) return fail(DOCK_EINVAL, "results is NULL");
    if (n_ligands > 0 && (!o->best_score || !o->n_poses || !o->status || !o->pose_score ||
                          !o->pose_restart))
        return fail(DOCK_EINVAL, "a required result array is NULL");
    if (o->pose_contacts && !o->pose_xyz)
        return fail(DOCK_EINVAL, "pose_contacts needs pose_xyz (the contacts are of the output poses)");
    return DOCK_OK;
}

// Start rotations (quaternion -> matrix), alignment rotations R_y(beta_j) R_x(alpha_i),
// torsion (cos, sin): computed in double, rounded to float, in one host blob
// (offsets in `t`, relative to the blob's start).
std::string tables_key(const dock_params *p) {
    std::string key((const char *)p->start_quat, sizeof(float) * 4 * (size_t)p->restarts);
    key += "|" + std::to_string(p->restarts) + "|" + std::to_string(p->align_steps) + "|" +
           std::to_string(p->torsion_steps);
    return key;
}

void make_tables(const dock_params *p, TableBlob *out) {
    const int R = p->restarts, A = p->align_steps, T = p->torsion_steps;
    const size_t nS = (size_t)R * 3, nA = (size_t)A * A * 3;
    std::vector<float4> smat(nS), amat(nA);
    std::vector<float2> tors(T);
    for (int r = 0; r < R; ++r) {
        double w = p->start_quat[4 * r], x = p->start_quat[4 * r + 1], y = p->start_quat[4 * r + 2],
               z = p->start_quat[4 * r + 3];
        const double s = std::sqrt(w * w + x * x + y * y + z * z);
        w /= s; x /= s; y /= s; z /= s;
        const double M[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                             2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                             2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
        for (int a = 0; a < 3; ++a)
            smat[3 * r + a] = make_float4((float)M[3 * a], (float)M[3 * a + 1], (float)M[3 * a + 2], 0.f);
    }
    for (int i = 0; i < A; ++i)
        for (int j = 0; j < A; ++j) {
            const double al = 2.0 * M_PI * i / A, be = 2.0 * M_PI * j / A;
            const double ca = std::cos(al), sa = std::sin(al), cb = std::cos(be), sb = std::sin(be);
            // R_y(b) R_x(a) = [[cb, sb sa, sb ca], [0, ca, -sa], [-sb, cb sa, cb ca]]
            const double M[9] = {cb, sb * sa, sb * ca, 0.0, ca, -sa, -sb, cb * sa, cb * ca};
            const int o = i * A + j;
            for (int a = 0; a < 3; ++a)
                amat[3 * o + a] = make_float4((float)M[3 * a], (float)M[3 * a + 1], (float)M[3 * a + 2], 0.f);
        }
    for (int k = 0; k < T; ++k) {
        const double th = 2.0 * M_PI * k / T;
        tors[k] = make_float2((float)std::cos(th), (float)std::sin(th));
    }
    // (cos, sin) of 2 pi k / A, padded to whole k_align strips (k >= A wraps)
    const int nC = (A + kAlignJ - 1) / kAlignJ * kAlignJ;
    std::vector<float2> acs(nC);
    for (int k = 0; k < nC; ++k) {
        const double an = 2.0 * M_PI * k / A;
        acs[k] = make_float2((float)std::cos(an), (float)std::sin(an));
    }
    const size_t bS = align256(nS * sizeof(float4)), bA = align256(nA * sizeof(float4)),
                 bT = align256((size_t)T * sizeof(float2)), bC = align256((size_t)nC * sizeof(float2));
    out->o_smat = 0;
    out->o_amat = bS;
    out->o_tors = bS + bA;
    out->o_acs = bS + bA + bT;
    out->bytes.assign(bS + bA + bT + bC, 0);
    std::memcpy(out->bytes.data() + out->o_smat, smat.data(), nS * sizeof(float4));
    std::memcpy(out->bytes.data() + out->o_amat, amat.data(), nA * sizeof(float4));
    std::memcpy(out->bytes.data() + out->o_tors, tors.data(), (size_t)T * sizeof(float2));
    std::memcpy(out->bytes.data() + out->o_acs, acs.data(), (size_t)nC * sizeof(float2));
}

Tables tables_at(const TableBlob &b, char *d) {
    Tables t;
    t.d = d;
    t.smat = (const float4 *)(d + b.o_smat);
    t.amat = (const float4 *)(d + b.o_amat);
    t.tors = (const float2 *)(d + b.o_tors);
    t.acs = (const float2 *)(d + b.o_acs);
    return t;
}

// Device tables of the ordinary entry points: one allocation per distinct
// (start orientations, R, A, T), kept by the context.
int get_tables(dock_ctx *c, const dock_params *p, Tables *out) {
    const std::string key = tables_key(p);
    auto it = c->tables.find(key);
    if (it != c->tables.end()) {
        *out = it->second;
        return DOCK_OK;
    }
    TableBlob b;
    make_tables(p, &b);
    void *d = nullptr;
    HIP_TRY(hipMalloc(&d, b.bytes.size()));
    HIP_TRY(hipMemcpy(d, b.bytes.data(), b.bytes.size(), hipMemcpyHostToDevice));
    const Tables t = tables_at(b, (char *)d);
    c->tables[key] = t;
    *out = t;
    return DOCK_OK;
}

struct WsLayout {
    size_t far, counters, bin_list, rscore, rtrace, acc, sel, nsel, fscore, fo, total;
};

WsLayout ws_layout(const dock_library *lib, const dock_params *p, bool user_trace) {
    WsLayout w{};
    size_t o = 0;
    const size_t L = (size_t)lib->n_ligands, R = (size_t)p->restarts, K = (size_t)p->top_k;
    w.far = o; o += align256((size_t)lib->n_atoms_total * kFarWords * 8);
    w.counters = o; o += align256(kNumCounters * sizeof(int));
    const size_t lists = (size_t)kNumBins * (p->bin_mode ? kMaxGroups : 1);
    w.bin_list = o; o += align256(lists * L * sizeof(int));
    w.rscore = o; o += align256(L * R * sizeof(float));
    w.rtrace = o;
    if (!user_trace) o += align256(R * (L + (size_t)p->sweep_passes * lib->n_rot_total) * sizeof(uint16_t));
    w.acc = o; o += align256((size_t)lib->n_atoms_total * K * 3 * sizeof(float));
    w.sel = o; o += align256(L * K * sizeof(int));
    w.nsel = o; o += align256(L * sizeof(int));
    w.fscore = o; o += align256(L * K * sizeof(float));
    w.fo = o; o += align256(L * K * sizeof(int));
    w.total = o;
    return w;
}

// A workspace grows to a quarter more than asked, so that slightly larger later
// calls reuse it.
size_t ws_grown_bytes(size_t bytes) { return bytes + bytes / 4; }

int get_workspace(dock_ctx *c, hipStream_t s, size_t bytes, void **out) {
    Workspace &w = c->ws[s];
    if (w.bytes < bytes) {
        if (w.base) {
            HIP_TRY(hipStreamSynchronize(s));
            HIP_TRY(hipFree(w.base));
            w.base = nullptr;
            w.bytes = 0;
        }
        const size_t nb = ws_grown_bytes(bytes);
        if (hipMalloc(&w.base, nb) != hipSuccess) {
            w.base = nullptr;
            if (hipMalloc(&w.base, bytes) != hipSuccess) {
                w.base = nullptr;
                (void)hipGetLastError();
                return fail(DOCK_ENOMEM, "workspace allocation failed");
            }
            w.bytes = bytes;
        } else {
            w.bytes = nb;
        }
    }
    *out = w.base;
    return DOCK_OK;
}

// Device layout of a dock_submit request: the library copy (inputs, the same
// layout as the pinned staging buffer) followed by the results; t receives the
// result offsets.
struct SubmitLayout {
    size_t i_ao, i_xyz, i_ty, i_bo, i_b, i_ro, i_rb, i_rm, inputs, results;
};

SubmitLayout submit_layout(const dock_library *lib, const dock_params *p, const dock_results *o,
                           Ticket *t) {
    SubmitLayout sl{};
    const int L = lib->n_ligands;
    const long long A = lib->n_atoms_total, Nb = lib->n_bonds_total, Nr = lib->n_rot_total;
    const int K = p->top_k, R = p->restarts;
    const long long trace_len = o->trace ? (long long)R * (L + (long long)p->sweep_passes * Nr) : 0;
    size_t off = 0;
    auto take = [&](size_t b) { size_t r = off; off += align256(b); return r; };
    sl.i_ao = take((size_t)(L + 1) * 4);
    sl.i_xyz = take((size_t)A * 12);
    sl.i_ty = take((size_t)A);
    sl.i_bo = take((size_t)(L + 1) * 4);
    sl.i_b = take((size_t)Nb * 8);
    sl.i_ro = take((size_t)(L + 1) * 4);
    sl.i_rb = take((size_t)Nr * 8);
    sl.i_rm = take((size_t)Nr * lib->mask_words * 8);
    sl.inputs = off;
    t->L = L; t->K = K; t->R = R; t->A = A; t->trace_len = trace_len;
    size_t so = 0;
    auto stake = [&](size_t b) { size_t r = so; so += align256(b); return r; };
    t->o_best = stake((size_t)L * 4);
    t->o_np = stake((size_t)L * 4);
    t->o_st = stake((size_t)L * 4);
    t->o_ps = stake((size_t)L * K * 4);
    t->o_pr = stake((size_t)L * K * 4);
    t->o_xyz = stake(o->pose_xyz ? (size_t)A * K * 12 : 0);
    t->o_rs = stake(o->restart_score ? (size_t)L * R * 4 : 0);
    t->o_tr = stake((size_t)trace_len * 2);
    t->o_ft = stake(o->final_trace ? (size_t)L * K * 2 : 0);
    t->o_pc = stake(o->pose_contacts ? (size_t)L * K * 4 : 0);
    t->stage_bytes = so;
    sl.results = so;
    return sl;
}

int occupancy(dock_ctx *c, const std::string &key, int v) {
    auto it = c->occ.find(key);
    if (it != c->occ.end()) return it->second;
    c->occ[key] = v;
    return v;
}

constexpr int kOutBlocksPerCu = 4;
constexpr size_t kPinnedPoolMax = (size_t)1 << 30;  // pinned bytes kept for reuse at most

// Pinned staging memory for a dock_submit request: a retired ticket's buffer of
// at least `bytes` (and not far larger) when the pool has one, else a new one
// with a quarter more room.  Pinning fresh pages costs milliseconds per request.
int pinned_get(dock_ctx *c, size_t bytes, void **out, size_t *cap) {
    auto it = c->pinned_pool.lower_bound(bytes);
    if (it != c->pinned_pool.end() && it->first <= 4 * bytes + ((size_t)1 << 20)) {
        *out = it->second;
        *cap = it->first;
        c->pinned_pool_bytes -= it->first;
        c->pinned_pool.erase(it);
        return DOCK_OK;
    }
    const size_t capb = bytes + bytes / 4;
    if (hipHostMalloc(out, capb, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        *out = nullptr;
        return fail(DOCK_ENOMEM, "pinned staging allocation failed");
    }
    *cap = capb;
    return DOCK_OK;
}

// Return a staging buffer whose copies have completed to the pool (or free it
// when the pool is full).
void pinned_put(dock_ctx *c, void *p, size_t cap) {
    if (!p) return;
    if (c->pinned_pool_bytes + cap > kPinnedPoolMax) {
        (void)hipHostFree(p);
        return;
    }
    c->pinned_pool.emplace(cap, p);
    c->pinned_pool_bytes += cap;
}

constexpr int kPlainWaves = 4;
constexpr int kPlainSelectWaves = 16;  // plain form: a ligand's candidates over 16 waves
constexpr int kPlainFalignWaves = 4;   // plain form: a workgroup of 4 waves per kept pose
constexpr int kSubmitStreams = 4;
constexpr int kPlainStreams = 4;

// Plain (latency) form: one launch sequence per ligand (checks, restarts, select
// and final step), ligands round-robin over a few streams so that consecutive
// ligands overlap, as the paper's multi-threaded host does with its streams.
// The host needs each ligand's size to pick the kernel, so the offsets are read
// back first (this form is synchronous with respect to the host anyway).
int enqueue_plain(dock_ctx *c, const dock_library *lib, const GridArgs &g, const SearchArgs &sa,
                  const LibArgs &la, const WorkArgs &wa, const OutArgs &oa, const ContactArgs &ca,
                  const std::array<hipEvent_t, 5> &ev, hipStream_t s) {
    const int L = lib->n_ligands;
    std::vector<int32_t> ao(L + 1);
    HIP_TRY(hipMemcpyAsync(ao.data(), lib->atom_off, sizeof(int32_t) * (L + 1),
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    while ((int)c->plain_streams.size() < kPlainStreams) {
        hipStream_t t;
        HIP_TRY(hipStreamCreateWithFlags(&t, hipStreamNonBlocking));
        c->plain_streams.push_back(t);
        hipEvent_t e;
        HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        c->plain_events.push_back(e);
    }
    if (c->timing) HIP_TRY(hipEventRecord(ev[0], s));
    if (c->timing) HIP_TRY(hipEventRecord(ev[1], s));
    if (c->timing) HIP_TRY(hipEventRecord(ev[2], s));  // no separate alignment phase
    hipEvent_t go;
    HIP_TRY(hipEventCreateWithFlags(&go, hipEventDisableTiming));
    HIP_TRY(hipEventRecord(go, s));
    for (auto t : c->plain_streams) HIP_TRY(hipStreamWaitEvent(t, go, 0));
    for (int l = 0; l < L; ++l) {
        hipStream_t t = c->plain_streams[l % kPlainStreams];
        HIP_TRY(launch_prep_one(g, sa, la, wa, oa, l, t));
        const int n = ao[l + 1] - ao[l];
        if (n < 1 || n > kMaxAtoms) continue;  // flagged by the checks
        const int bin = (n - 1) >> 5;
        HIP_TRY(launch_plain(l, bin, kPlainWaves, g, sa, la, wa, oa, t));
        HIP_TRY(launch_select(bin, bin, 1, kPlainSelectWaves, g, sa, la, wa, oa, l, t));
        HIP_TRY(launch_falign(bin, bin, sa.K, kPlainFalignWaves, g, sa, la, wa, oa, l, 0, t));
        HIP_TRY(launch_out(bin, bin, 1, sa, la, wa, oa, l, t));
        if (oa.pcontacts) HIP_TRY(launch_rescore(ca, sa, la, oa, l, 0, t));
    }
    for (size_t i = 0; i < c->plain_streams.size(); ++i) {
        HIP_TRY(hipEventRecord(c->plain_events[i], c->plain_streams[i]));
        HIP_TRY(hipStreamWaitEvent(s, c->plain_events[i], 0));
    }
    HIP_TRY(hipEventDestroy(go));
    if (c->timing) HIP_TRY(hipEventRecord(ev[3], s));
    if (c->timing) HIP_TRY(hipEventRecord(ev[4], s));
    return DOCK_OK;
}

// Bytes of the scratch array a dock_ligands_batch_noalloc call uses: its tables
// followed by its workspace.
size_t noalloc_bytes(const dock_library *lib, const dock_params *p, bool user_trace) {
    const size_t R = (size_t)p->restarts, A = (size_t)p->align_steps, T = (size_t)p->torsion_steps;
    const size_t nC = (A + kAlignJ - 1) / kAlignJ * kAlignJ;
    const size_t tables = align256(R * 3 * sizeof(float4)) + align256(A * A * 3 * sizeof(float4)) +
                          align256(T * sizeof(float2)) + align256(nC * sizeof(float2));
    return tables + ws_layout(lib, p, user_trace).total;
}

// Kernel arguments of one call.
struct Launch {
    GridArgs g;
    SearchArgs sa;
    LibArgs la;
    WorkArgs wa;
    OutArgs oa;
    ContactArgs ca;
};

// Tables, workspace and kernel arguments of a call on a device-resident library
// and results.  With `scratch` (dock_ligands_batch_noalloc) the tables and the
// workspace are placed in that buffer and nothing is allocated on the device.
int prepare_launch(dock_ctx *c, const Pocket &pk, const dock_library *lib, const dock_params *p,
                   const dock_results *o, hipStream_t s, char *scratch, bool timed, Launch *L) {
    if (o->pose_contacts && !pk.has_atoms)
        return fail(DOCK_EINVAL, "pose_contacts needs the pocket's atoms (dock_pocket_set_atoms)");
    Tables tb;
    const bool user_trace = o->trace != nullptr;
    const WsLayout wl = ws_layout(lib, p, user_trace);
    char *base = nullptr;
    if (scratch) {
        const size_t need = noalloc_bytes(lib, p, user_trace);
        if (need > (size_t)DOCK_NOALLOC_SCRATCH_BYTES)
            return fail(DOCK_EINVAL, "request needs " + std::to_string(need) +
                                         " B of scratch memory, more than the " +
                                         std::to_string((size_t)DOCK_NOALLOC_SCRATCH_BYTES) +
                                         " B of DOCK_NOALLOC_SCRATCH_BYTES");
        const std::string key = tables_key(p);
        auto it = c->noalloc_tables.find(key);
        if (it == c->noalloc_tables.end()) {
            TableBlob b;
            make_tables(p, &b);
            it = c->noalloc_tables.emplace(key, std::move(b)).first;
        }
        const TableBlob &b = it->second;
        HIP_TRY(hipMemcpyAsync(scratch, b.bytes.data(), b.bytes.size(), hipMemcpyHostToDevice, s));
        tb = tables_at(b, scratch);
        base = scratch + align256(b.bytes.size());
    } else {
        int rc = get_tables(c, p, &tb);
        if (rc) return rc;
        void *wb = nullptr;
        rc = get_workspace(c, s, wl.total, &wb);
        if (rc) return rc;
        base = (char *)wb;
    }
    // zeroed first: the graph key is the bytes of *L, padding included
    std::memset((void *)L, 0, sizeof(*L));
    std::memcpy((void *)&L->g, (const void *)&pk.g, sizeof(GridArgs));
    SearchArgs &sa = L->sa;
    sa.R = p->restarts;
    sa.T = p->torsion_steps;
    sa.P = p->sweep_passes;
    sa.A = p->align_steps;
    sa.K = p->top_k;
    sa.final_align = p->final_align;
    sa.bmin = p->bump_min_bonds;
    sa.prune = p->bump_prune;
    sa.groups = p->bin_mode ? kMaxGroups : 1;
    {
        const double bg = (double)p->bump_dist * (double)L->g.inv_h;
        sa.bump2g = (float)(bg * bg);
        sa.dedup2 = (float)((double)p->dedup_rmsd * (double)p->dedup_rmsd);
    }
    sa.smat = tb.smat;
    sa.amat = tb.amat;
    sa.tors = tb.tors;
    sa.acs = tb.acs;

    LibArgs &la = L->la;
    la.L = lib->n_ligands;
    la.mask_words = lib->mask_words;
    la.A_total = lib->n_atoms_total;
    la.Nb_total = lib->n_bonds_total;
    la.Nr_total = lib->n_rot_total;
    la.atom_off = lib->atom_off;
    la.xyz = lib->xyz;
    la.type = lib->type;
    la.bond_off = lib->bond_off;
    la.bond = lib->bond;
    la.rot_off = lib->rot_off;
    la.rot_bond = lib->rot_bond;
    la.rot_mask = (const unsigned long long *)lib->rot_mask;

    WorkArgs &wa = L->wa;
    wa.far = (unsigned long long *)(base + wl.far);
    wa.counters = (int *)(base + wl.counters);
    wa.bin_list = (int *)(base + wl.bin_list);
    wa.rscore = (float *)(base + wl.rscore);
    wa.rtrace = user_trace ? o->trace : (uint16_t *)(base + wl.rtrace);
    wa.acc_pose = (float *)(base + wl.acc);
    wa.sel = (int *)(base + wl.sel);
    wa.nsel = (int *)(base + wl.nsel);
    wa.fscore = (float *)(base + wl.fscore);
    wa.fo = (int *)(base + wl.fo);
    wa.scored = timed ? c->d_scored : nullptr;

    OutArgs &oa = L->oa;
    oa.best = o->best_score;
    oa.npose = o->n_poses;
    oa.status = o->status;
    oa.pscore = o->pose_score;
    oa.prestart = o->pose_restart;
    oa.pxyz = o->pose_xyz;
    oa.rscore_user = o->restart_score;
    oa.ftrace = o->final_trace;
    oa.pcontacts = o->pose_contacts;
    if (pk.has_atoms) std::memcpy((void *)&L->ca, (const void *)&pk.ca, sizeof(ContactArgs));
    return DOCK_OK;
}

// Launch shapes of the batched sequence, per size bin: workgroup counts from the
// occupancy API and the bin's tile choice (tuned, or the defaults).
struct Shapes {
    BinShape tile[kNumBins];
    int align_blocks[kNumBins], dock_blocks[kNumBins], select_blocks[kNumBins],
        falign_blocks[kNumBins];
    int out_blocks, rescore_blocks;
};

std::string tune_key(const SearchArgs &sa) {
    return std::to_string(sa.R) + "/" + std::to_string(sa.T) + "/" + std::to_string(sa.A) + "/" +
           std::to_string(sa.K) + "/" + std::to_string(sa.P);
}

int make_shapes(dock_ctx *c, const Launch &L, const BinShape *tile, Shapes *sh) {
    const SearchArgs &sa = L.sa;
    for (int bin = 0; bin < kNumBins; ++bin) {
        const BinShape &t = tile[bin];
        sh->tile[bin] = t;
        if ((size_t)c->lds_arena < align_lds_min(bin, sa.A, sa.R))
            return fail(DOCK_EDEVICE, "device LDS per workgroup too small for the alignment kernel");
        const std::string a = "a" + std::to_string(bin) + "/" + std::to_string(sa.R) + "/" +
                              std::to_string(sa.A) + "/" + std::to_string(c->lds_arena);
        sh->align_blocks[bin] =
            occupancy(c, a, align_blocks_per_cu(bin, sa.R, sa.A, c->lds_arena)) * c->num_cu;
        const std::string k = "d" + std::to_string(bin) + "/" + std::to_string(t.dock_waves) + "/" +
                              std::to_string((sa.T + 63) / 64);
        sh->dock_blocks[bin] =
            occupancy(c, k, dock_blocks_per_cu(bin, t.dock_waves, sa.T)) * c->num_cu;
        const std::string f = "s" + std::to_string(bin) + "/" + std::to_string(t.select_waves) +
                              "/" + std::to_string(sa.R) + "/" + std::to_string(sa.K);
        const int sb =
            occupancy(c, f, select_blocks_per_cu(bin, t.select_waves, sa.R, sa.K)) * c->num_cu;
        sh->select_blocks[bin] = sb > L.la.L ? L.la.L : sb;
        const std::string fa = "fa" + std::to_string(bin) + "/" + std::to_string(t.falign_waves);
        int per_cu = occupancy(c, fa, falign_blocks_per_cu(bin, t.falign_waves));
        if (t.falign_per_cu > 0 && t.falign_per_cu < per_cu) per_cu = t.falign_per_cu;
        sh->falign_blocks[bin] = per_cu * c->num_cu;
    }
    sh->out_blocks = std::min(L.la.L, kOutBlocksPerCu * c->num_cu);
    // rescoring: 4 waves per workgroup, at most one wave per (ligand, pose) item
    sh->rescore_blocks =
        (int)std::min<long long>(((long long)L.la.L * L.sa.K + 3) / 4, 8LL * c->num_cu);
    return DOCK_OK;
}

// The batched launch sequence: reset, prep, then per stage its launch per bin.
// marks (optional): events recorded at the phase boundaries.
int run_sequence(dock_ctx *c, const Launch &L, const Shapes &sh, hipStream_t s,
                 const std::array<hipEvent_t, 5> *marks) {
    const GridArgs &g = L.g;
    const SearchArgs &sa = L.sa;
    const LibArgs &la = L.la;
    const WorkArgs &wa = L.wa;
    const OutArgs &oa = L.oa;
    const int G = sa.groups;
    HIP_TRY(launch_reset(wa.counters, 0, kNumCounters, s));
    if (marks) HIP_TRY(hipEventRecord((*marks)[0], s));
    HIP_TRY(launch_prep(g, sa, la, wa, oa, s));
    if (marks) HIP_TRY(hipEventRecord((*marks)[1], s));
    // each stage: one launch per work list (atom bin, or atom bin x bond group)
    for (int bin = 0; bin < kNumBins; ++bin)
        for (int q = 0; q < G; ++q)
            HIP_TRY(launch_align(bin, bin * G + q, sh.align_blocks[bin], c->lds_arena, g, sa, la,
                                 wa, s));
    if (marks) HIP_TRY(hipEventRecord((*marks)[2], s));
    for (int bin = 0; bin < kNumBins; ++bin)
        for (int q = 0; q < G; ++q)
            HIP_TRY(launch_dock(bin, bin * G + q, sh.dock_blocks[bin], sh.tile[bin].dock_waves, g,
                                sa, la, wa, s));
    if (marks) HIP_TRY(hipEventRecord((*marks)[3], s));
    for (int bin = 0; bin < kNumBins; ++bin)
        for (int q = 0; q < G; ++q)
            HIP_TRY(launch_select(bin, bin * G + q, sh.select_blocks[bin],
                                  sh.tile[bin].select_waves, g, sa, la, wa, oa, -1, s));
    for (int bin = 0; bin < kNumBins; ++bin)
        for (int q = 0; q < G; ++q)
            HIP_TRY(launch_falign(bin, bin * G + q, sh.falign_blocks[bin],
                                  sh.tile[bin].falign_waves, g, sa, la, wa, oa, -1,
                                  sh.tile[bin].falign_xcd ? kXcds : 0, s));
    for (int bin = 0; bin < kNumBins; ++bin)
        for (int q = 0; q < G; ++q)
            HIP_TRY(launch_out(bin, bin * G + q, sh.out_blocks, sa, la, wa, oa, -1, s));
    if (oa.pcontacts) HIP_TRY(launch_rescore(L.ca, sa, la, oa, -1, sh.rescore_blocks, s));
    if (marks) HIP_TRY(hipEventRecord((*marks)[4], s));
    return DOCK_OK;
}

// The tile choice for these search settings: the autotuner's, else the defaults.
const BinShape *bin_tiles(dock_ctx *c, const SearchArgs &sa) {
    static const BinShape defaults[kNumBins] = {};
    auto it = c->tuned.find(tune_key(sa));
    return it != c->tuned.end() ? it->second.data() : defaults;
}

// Enqueue the whole pipeline for a device-resident library.  With `scratch`
// (dock_ligands_batch_noalloc) the tables and the workspace are placed in that
// buffer, nothing is allocated on the device, no graph is captured and no phase
// timing is recorded.
int enqueue_batch(dock_ctx *c, const Pocket &pk, const dock_library *lib, const dock_params *p,
                  const dock_results *o, hipStream_t s, char *scratch = nullptr) {
    if (lib->n_ligands == 0) return DOCK_OK;
    const bool timed = c->timing && !scratch;
    Launch L;
    int rc = prepare_launch(c, pk, lib, p, o, s, scratch, timed, &L);
    if (rc) return rc;
    std::array<hipEvent_t, 5> ev{};
    if (timed) {
        for (auto &e : ev) HIP_TRY(hipEventCreate(&e));
        c->marks.push_back(ev);
    }
    if (p->mode == DOCK_MODE_PLAIN)
        return enqueue_plain(c, lib, L.g, L.sa, L.la, L.wa, L.oa, L.ca, ev, s);
    // launch shapes (occupancy queries stay outside any graph capture)
    Shapes sh;
    rc = make_shapes(c, L, bin_tiles(c, L.sa), &sh);
    if (rc) return rc;
    if (timed || s == nullptr || scratch) return run_sequence(c, L, sh, s, timed ? &ev : nullptr);
    // graph key: everything the kernels' arguments and launch shapes depend on
    std::string key((const char *)&L, sizeof(L));
    key.append((const char *)&sh, sizeof(sh));
    key.append((const char *)&s, sizeof(s));
    auto gi = c->graphs.find(key);
    if (gi == c->graphs.end()) {
        if (c->seen_keys[key]++ == 0) {
            if (c->seen_keys.size() > 256) c->seen_keys.clear();
            return run_sequence(c, L, sh, s, nullptr);  // first time: eager
        }
        if (c->graphs.size() >= 16) {
            for (auto &kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
            c->graphs.clear();
        }
        hipGraph_t graph = nullptr;
        HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
        const int rc2 = run_sequence(c, L, sh, s, nullptr);
        const hipError_t ec = hipStreamEndCapture(s, &graph);
        if (rc2) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc2;
        }
        if (ec != hipSuccess) return fail(DOCK_EDEVICE, std::string("graph capture: ") + hipGetErrorString(ec));
        hipGraphExec_t exec = nullptr;
        const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) return fail(DOCK_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(ei));
        gi = c->graphs.emplace(key, exec).first;
    }
    HIP_TRY(hipGraphLaunch(gi->second, s));
    return DOCK_OK;
}

// Shell atlas of the alignment kernel: band geometry (pass 1), then the bands
// that fit one workgroup's LDS, for every type (pass 2).  Grids wider than 256
// cells in x keep no atlas (every alignment sample reads global memory).
int build_atlas(dock_ctx *c, Pocket &pk) {
    GridArgs &g = pk.g;
    g.atlas = nullptr;
    g.bands = nullptr;
    g.blob16 = nullptr;
    g.nbands = 0;
    if (g.nx > 256) return DOCK_OK;
    const size_t ib = (size_t)2 * kMaxBands * sizeof(int4);
    if (hipMalloc(&pk.d_bands, ib) != hipSuccess) {
        (void)hipGetLastError();
        pk.d_bands = nullptr;
        return fail(DOCK_ENOMEM, "atlas allocation failed");
    }
    HIP_TRY(launch_atlas_count(g, pk.d_bands, nullptr));
    std::vector<int4> info(2 * kMaxBands);
    HIP_TRY(hipMemcpy(info.data(), pk.d_bands, ib, hipMemcpyDeviceToHost));
    int nb = 0;
    long long off = 0;
    std::vector<int> blob((size_t)g.ntypes * kMaxBands);
    // bands up to twice the LDS arena: the alignment kernel streams a band that
    // does not fit its region in two chunks of whole rows
    for (; nb < kMaxBands; ++nb) {
        const int4 q = info[2 * nb + 1];
        const long long size16 = band_padded(q.z / 16 + q.y);
        if (q.y < 0 || size16 * 16 > 2LL * c->lds_arena) break;
    }
    for (int t = 0; t < g.ntypes; ++t)
        for (int b = 0; b < nb; ++b) {
            blob[(size_t)t * nb + b] = (int)off;
            off += band_padded(info[2 * b + 1].z / 16 + info[2 * b + 1].y);
        }
    if (nb == 0 || off >= (1LL << 31) - 64) return DOCK_OK;
    // 64 float4 of padding after the last band: a chunk copy reads whole 64-float4
    // instructions from its start, which for a second chunk may pass its band's end
    if (hipMalloc(&pk.d_atlas, (size_t)(off + 64) * 16) != hipSuccess ||
        hipMalloc(&pk.d_blob16, (size_t)g.ntypes * nb * sizeof(int)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(DOCK_ENOMEM, "atlas allocation failed");
    }
    HIP_TRY(hipMemcpy(pk.d_blob16, blob.data(), (size_t)g.ntypes * nb * sizeof(int),
                      hipMemcpyHostToDevice));
    HIP_TRY(launch_atlas_fill(g, pk.d_bands, pk.d_blob16, pk.d_atlas, nb, nullptr));
    HIP_TRY(hipDeviceSynchronize());
    g.atlas = pk.d_atlas;
    g.bands = pk.d_bands;
    g.blob16 = pk.d_blob16;
    g.nbands = nb;
    return DOCK_OK;
}

}  // namespace

extern "C" {

const char *dock_last_error(void) { return g_err.c_str(); }

int dock_create(int device, uint64_t hbm_budget_bytes, dock_ctx **out) {
    if (!out) return fail(DOCK_EINVAL, "out is NULL");
    *out = nullptr;
    int n = 0;
    HIP_TRY(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(DOCK_EINVAL, "no such device");
    HIP_TRY(hipSetDevice(device));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(DOCK_EDEVICE, std::string("library is built for gfx950, device is ") + prop.gcnArchName);
    auto *c = new (std::nothrow) dock_ctx();
    if (!c) return fail(DOCK_ENOMEM, "context allocation failed");
    c->device = device;
    c->num_cu = prop.multiProcessorCount;
    c->budget = (size_t)hbm_budget_bytes;
    c->lds_arena = (int)std::min<size_t>(prop.sharedMemPerBlock, (size_t)160 * 1024);
    {
        const int rc = scratch_address(device, &c->scratch);
        if (rc) {
            delete c;
            return rc;
        }
    }
    for (int i = 0; i < kSubmitStreams; ++i) {
        hipStream_t t = nullptr;
        if (hipStreamCreateWithFlags(&t, hipStreamNonBlocking) != hipSuccess) {
            for (auto u : c->submit_streams) (void)hipStreamDestroy(u);
            delete c;
            return fail(DOCK_EDEVICE, "stream creation failed");
        }
        c->submit_streams.push_back(t);
    }
    *out = c;
    g_err.clear();
    return DOCK_OK;
}

int dock_destroy(dock_ctx *c) {
    if (!c) return fail(DOCK_EINVAL, "ctx is NULL");
    hipSetDevice(c->device);
    hipDeviceSynchronize();
    for (auto &kv : c->tickets) {
        if (kv.second.done) hipEventDestroy(kv.second.done);
        if (kv.second.pinned) hipHostFree(kv.second.pinned);
    }
    for (auto &kv : c->pinned_pool) hipHostFree(kv.second);
    for (auto &kv : c->pockets) kv.second.release();
    if (c->d_scored) hipFree(c->d_scored);
    for (auto &kv : c->ws) hipFree(kv.second.base);
    for (auto &kv : c->tables) hipFree(kv.second.d);
    for (auto &m : c->marks)
        for (auto &e : m) hipEventDestroy(e);
    for (auto &kv : c->graphs) hipGraphExecDestroy(kv.second);
    for (auto t : c->submit_streams) hipStreamDestroy(t);
    for (auto t : c->plain_streams) hipStreamDestroy(t);
    for (auto e : c->plain_events) hipEventDestroy(e);
    delete c;
    return DOCK_OK;
}

int dock_pocket_load(dock_ctx *c, const dock_grid_desc *gd, int32_t *pocket_id) {
    if (!c || !gd || !pocket_id) return fail(DOCK_EINVAL, "NULL argument");
    if (gd->ntypes < 1 || gd->ntypes > 255) return fail(DOCK_EINVAL, "ntypes must be in [1,255]");
    if (gd->nx < 2 || gd->ny < 2 || gd->nz < 2) return fail(DOCK_EINVAL, "grid dims must be >= 2");
    const long long cells = (long long)gd->nx * gd->ny * gd->nz;
    if (cells >= (1LL << 24)) return fail(DOCK_EINVAL, "nx*ny*nz must be < 2^24");
    const long long bytes = cells * 4 * gd->ntypes;
    const long long qbytes = cells * 32 * gd->ntypes;
    if (qbytes >= (1LL << 32)) return fail(DOCK_EINVAL, "grid too large (ntypes*nx*ny*nz*32 >= 4 GiB)");
    if (!(gd->spacing > 0.f) || !std::isfinite(gd->spacing)) return fail(DOCK_EINVAL, "spacing must be > 0");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(gd->origin[a])) return fail(DOCK_EINVAL, "origin must be finite");
    if (!gd->values) return fail(DOCK_EINVAL, "values is NULL");
    std::lock_guard<std::mutex> lk(c->mu);
    HIP_TRY(hipSetDevice(c->device));
    Pocket pk;
    float *d_vals = nullptr;
    if (hipMalloc(&d_vals, (size_t)bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(DOCK_ENOMEM, "pocket staging allocation failed");
    }
    if (hipMalloc(&pk.d_cubes, (size_t)qbytes) != hipSuccess) {
        (void)hipGetLastError();
        hipFree(d_vals);
        return fail(DOCK_ENOMEM, "pocket allocation failed");
    }
    hipError_t e = hipMemcpy(d_vals, gd->values, (size_t)bytes, hipMemcpyHostToDevice);
    if (!e) e = launch_build_cubes(d_vals, pk.d_cubes, gd->ntypes, gd->nx, gd->ny, gd->nz, nullptr);
    if (!e) e = hipDeviceSynchronize();
    hipFree(d_vals);
    if (e) {
        hipFree(pk.d_cubes);
        return fail(DOCK_EDEVICE, std::string("pocket upload failed: ") + hipGetErrorString(e));
    }
    GridArgs &g = pk.g;
    g.cubes = pk.d_cubes;
    g.ncells = (uint32_t)(cells * gd->ntypes);
    g.type_bytes = (uint32_t)(cells * 32);
    g.ntypes = gd->ntypes;
    g.nx = gd->nx;
    g.ny = gd->ny;
    g.nz = gd->nz;
    g.inv_h = (float)(1.0 / (double)gd->spacing);
    g.ox = gd->origin[0];
    g.oy = gd->origin[1];
    g.oz = gd->origin[2];
    g.cx = (float)((double)gd->origin[0] + (double)gd->spacing * (gd->nx - 1) / 2.0);
    g.cy = (float)((double)gd->origin[1] + (double)gd->spacing * (gd->ny - 1) / 2.0);
    g.cz = (float)((double)gd->origin[2] + (double)gd->spacing * (gd->nz - 1) / 2.0);
    g.mx = (float)(gd->nx - 1);
    g.my = (float)(gd->ny - 1);
    g.mz = (float)(gd->nz - 1);
    g.m2x = (float)(gd->nx - 2);
    g.m2y = (float)(gd->ny - 2);
    g.m2z = (float)(gd->nz - 2);
    g.fnx = (float)gd->nx;
    g.fslab = (float)((long long)gd->nx * gd->ny);
    g.acx = (g.cx - g.ox) * g.inv_h;
    g.acy = (g.cy - g.oy) * g.inv_h;
    g.acz = (g.cz - g.oz) * g.inv_h;
    const int rc = build_atlas(c, pk);
    if (rc) {
        pk.release();
        return rc;
    }
    const int32_t id = c->next_pocket++;
    c->pockets[id] = pk;
    *pocket_id = id;
    return DOCK_OK;
}

int dock_pocket_unload(dock_ctx *c, int32_t pocket_id) {
    if (!c) return fail(DOCK_EINVAL, "ctx is NULL");
    std::lock_guard<std::mutex> lk(c->mu);
    auto it = c->pockets.find(pocket_id);
    if (it == c->pockets.end()) return fail(DOCK_ENOENT, "unknown pocket");
    if (it->second.busy) return fail(DOCK_EBUSY, "pocket has submitted work in flight");
    HIP_TRY(hipSetDevice(c->device));
    HIP_TRY(hipDeviceSynchronize());
    it->second.release();
    c->pockets.erase(it);
    return DOCK_OK;
}

int dock_pocket_set_atoms(dock_ctx *c, int32_t pocket_id, const dock_pocket_atoms *pa) {
    if (!c || !pa) return fail(DOCK_EINVAL, "NULL argument");
    if (pa->n_atoms < 0 || pa->n_atoms >= (1 << 24)) return fail(DOCK_EINVAL, "n_atoms must be in [0, 2^24)");
    if (pa->ntypes < 1 || pa->ntypes > 255) return fail(DOCK_EINVAL, "ntypes must be in [1,255]");
    if (!(pa->contact_dist > 0.f) || !std::isfinite(pa->contact_dist) || pa->contact_dist > 1e3f)
        return fail(DOCK_EINVAL, "contact_dist must be in (0, 1000] Angstrom");
    if (!pa->weight || (pa->n_atoms > 0 && (!pa->xyz || !pa->type)))
        return fail(DOCK_EINVAL, "xyz/type/weight is NULL");
    std::lock_guard<std::mutex> lk(c->mu);
    auto it = c->pockets.find(pocket_id);
    if (it == c->pockets.end()) return fail(DOCK_ENOENT, "unknown pocket");
    Pocket &pk = it->second;
    if (pk.busy) return fail(DOCK_EBUSY, "pocket has submitted work in flight");
    const int lt = pk.g.ntypes, nw = lt * pa->ntypes;
    if (nw > kMaxContactWeights)
        return fail(DOCK_EINVAL, "grid types x pocket atom types must be <= 1024");
    const int n = pa->n_atoms;
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int i = 0; i < n; ++i) {
        if (pa->type[i] >= pa->ntypes) return fail(DOCK_EINVAL, "pocket atom type >= ntypes");
        for (int a = 0; a < 3; ++a) {
            const double v = pa->xyz[3 * i + a];
            if (!std::isfinite(v)) return fail(DOCK_EINVAL, "pocket atom coordinate not finite");
            lo[a] = i == 0 || v < lo[a] ? v : lo[a];
            hi[a] = i == 0 || v > hi[a] ? v : hi[a];
        }
    }
    // cell edge: the contact distance plus a margin far above FP32 rounding of the
    // coordinates, grown if the grid would exceed 2^22 cells
    double h = (double)pa->contact_dist + 1e-3;
    long long dims[3];
    for (;;) {
        long long cells = 1;
        for (int a = 0; a < 3; ++a) {
            dims[a] = (long long)std::floor((hi[a] - lo[a]) / h) + 1;
            cells *= dims[a];
        }
        if (cells <= (1LL << 22)) break;
        h *= 1.25;
    }
    const long long ncell = dims[0] * dims[1] * dims[2];
    std::vector<int> cell_of(n), start(ncell + 1, 0);
    for (int i = 0; i < n; ++i) {
        long long ci[3];
        for (int a = 0; a < 3; ++a) {
            ci[a] = (long long)std::floor(((double)pa->xyz[3 * i + a] - lo[a]) / h);
            ci[a] = ci[a] < 0 ? 0 : (ci[a] >= dims[a] ? dims[a] - 1 : ci[a]);
        }
        cell_of[i] = (int)((ci[2] * dims[1] + ci[1]) * dims[0] + ci[0]);
        start[cell_of[i] + 1] += 1;
    }
    for (long long cidx = 0; cidx < ncell; ++cidx) start[cidx + 1] += start[cidx];
    std::vector<float4> atoms((size_t)(n > 0 ? n : 1));
    {
        std::vector<int> fill(start.begin(), start.end() - 1);
        for (int i = 0; i < n; ++i) {
            int t = pa->type[i];
            float tw;
            std::memcpy(&tw, &t, sizeof(tw));
            atoms[(size_t)fill[cell_of[i]]++] =
                make_float4(pa->xyz[3 * i], pa->xyz[3 * i + 1], pa->xyz[3 * i + 2], tw);
        }
    }
    const size_t b_atoms = align256(atoms.size() * sizeof(float4)),
                 b_start = align256((size_t)(ncell + 1) * sizeof(int)),
                 b_w = align256((size_t)nw * sizeof(int));
    HIP_TRY(hipSetDevice(c->device));
    HIP_TRY(hipDeviceSynchronize());  // no dock_ligands_batch work reads the old list
    void *d = nullptr;
    if (hipMalloc(&d, b_atoms + b_start + b_w) != hipSuccess) {
        (void)hipGetLastError();
        return fail(DOCK_ENOMEM, "pocket atom allocation failed");
    }
    hipError_t e = hipMemcpy(d, atoms.data(), atoms.size() * sizeof(float4), hipMemcpyHostToDevice);
    if (!e) e = hipMemcpy((char *)d + b_atoms, start.data(), (size_t)(ncell + 1) * sizeof(int),
                          hipMemcpyHostToDevice);
    if (!e) e = hipMemcpy((char *)d + b_atoms + b_start, pa->weight, (size_t)nw * sizeof(int),
                          hipMemcpyHostToDevice);
    if (e) {
        hipFree(d);
        return fail(DOCK_EDEVICE, std::string("pocket atom upload failed: ") + hipGetErrorString(e));
    }
    pk.release_atoms();
    pk.d_contacts = d;
    ContactArgs &ca = pk.ca;
    ca.atoms = (const float4 *)d;
    ca.cell_start = (const int *)((char *)d + b_atoms);
    ca.weight = (const int *)((char *)d + b_atoms + b_start);
    ca.ntypes = pa->ntypes;
    ca.nw = nw;
    ca.cx = (int)dims[0];
    ca.cy = (int)dims[1];
    ca.cz = (int)dims[2];
    ca.lox = (float)lo[0];
    ca.loy = (float)lo[1];
    ca.loz = (float)lo[2];
    ca.inv_cell = (float)(1.0 / h);
    ca.dc2 = (float)((double)pa->contact_dist * (double)pa->contact_dist);
    pk.has_atoms = true;
    return DOCK_OK;
}

int dock_ligands_batch(dock_ctx *c, int32_t pocket, const dock_library *lib,
                       const dock_params *p, dock_results *o, void *stream) {
    if (!c) return fail(DOCK_EINVAL, "ctx is NULL");
    int rc = check_params(p);
    if (rc) return rc;
    rc = check_library_shape(lib);
    if (rc) return rc;
    rc = check_results(o, lib->n_ligands);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(c->mu);
    auto it = c->pockets.find(pocket);
    if (it == c->pockets.end()) return fail(DOCK_ENOENT, "unknown pocket");
    HIP_TRY(hipSetDevice(c->device));
    return enqueue_batch(c, it->second, lib, p, o, (hipStream_t)stream);
}

int dock_ligands_batch_noalloc(dock_ctx *c, int32_t pocket, const dock_library *lib,
                               const dock_params *p, dock_results *o, void *stream) {
    if (!c) return fail(DOCK_EINVAL, "ctx is NULL");
    int rc = check_params(p);
    if (rc) return rc;
    if (p->mode != DOCK_MODE_BATCHED)
        return fail(DOCK_EINVAL, "dock_ligands_batch_noalloc runs the batched form only");
    rc = check_library_shape(lib);
    if (rc) return rc;
    rc = check_results(o, lib->n_ligands);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(c->mu);
    auto it = c->pockets.find(pocket);
    if (it == c->pockets.end()) return fail(DOCK_ENOENT, "unknown pocket");
    HIP_TRY(hipSetDevice(c->device));
    return enqueue_batch(c, it->second, lib, p, o, (hipStream_t)stream, c->scratch);
}

int dock_autotune(dock_ctx *c, int32_t pocket, const dock_library *lib, const dock_params *p,
                  dock_bin_tuning *out, void *stream) {
    if (!c) return fail(DOCK_EINVAL, "ctx is NULL");
    int rc = check_params(p);
    if (rc) return rc;
    if (p->mode != DOCK_MODE_BATCHED) return fail(DOCK_EINVAL, "dock_autotune tunes the batched form");
    rc = check_library_shape(lib);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(c->mu);
    auto it = c->pockets.find(pocket);
    if (it == c->pockets.end()) return fail(DOCK_ENOENT, "unknown pocket");
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    if (out) std::memset(out, 0, sizeof(dock_bin_tuning) * kNumBins);
    if (lib->n_ligands == 0) return DOCK_OK;
    // result buffers of the sample (freed at the end)
    const size_t L = (size_t)lib->n_ligands, K = (size_t)p->top_k, A = (size_t)lib->n_atoms_total;
    size_t off = 0;
    auto take = [&](size_t b) { size_t r = off; off += align256(b); return r; };
    const size_t o_best = take(L * 4), o_np = take(L * 4), o_st = take(L * 4),
                 o_ps = take(L * K * 4), o_pr = take(L * K * 4), o_xyz = take(A * K * 12);
    char *d = nullptr;
    if (hipMalloc((void **)&d, off) != hipSuccess) {
        (void)hipGetLastError();
        return fail(DOCK_ENOMEM, "autotune result allocation failed");
    }
    dock_results r{};
    r.best_score = (float *)(d + o_best);
    r.n_poses = (int32_t *)(d + o_np);
    r.status = (int32_t *)(d + o_st);
    r.pose_score = (float *)(d + o_ps);
    r.pose_restart = (int32_t *)(d + o_pr);
    r.pose_xyz = (float *)(d + o_xyz);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto body = [&]() -> int {
        HIP_TRY(hipEventCreate(&e0));
        HIP_TRY(hipEventCreate(&e1));
        Launch Lc;
        int rc2 = prepare_launch(c, it->second, lib, p, &r, s, nullptr, false, &Lc);
        if (rc2) return rc2;
        const BinShape defaults[kNumBins] = {};
        Shapes sh;
        rc2 = make_shapes(c, Lc, defaults, &sh);
        if (rc2) return rc2;
        // one whole pass fills the workspace the stage kernels read
        rc2 = run_sequence(c, Lc, sh, s, nullptr);
        if (rc2) return rc2;
        int lcount[kMaxLists], counts[kNumBins] = {};
        HIP_TRY(hipMemcpyAsync(lcount, Lc.wa.counters, sizeof(lcount), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        const int G = Lc.sa.groups;
        for (int q = 0; q < kNumBins * G; ++q) counts[q / G] += lcount[q];
        const GridArgs &g = Lc.g;
        const SearchArgs &sa = Lc.sa;
        const LibArgs &la = Lc.la;
        const WorkArgs &wa = Lc.wa;
        const OutArgs &oa = Lc.oa;
        // best of two timed runs of one stage launch (each stage's kernels only
        // read what earlier stages wrote and rewrite the same values)
        auto timeit = [&](auto &&launch, float *ms) -> int {
            float best = 3.4e38f;
            for (int rep = 0; rep < 2; ++rep) {
                HIP_TRY(hipEventRecord(e0, s));
                HIP_TRY(launch());
                HIP_TRY(hipEventRecord(e1, s));
                HIP_TRY(hipEventSynchronize(e1));
                float t = 0.f;
                HIP_TRY(hipEventElapsedTime(&t, e0, e1));
                best = t < best ? t : best;
            }
            *ms = best;
            return DOCK_OK;
        };
        std::array<BinShape, kNumBins> pick;
        for (int bin = 0; bin < kNumBins; ++bin) pick[bin] = defaults[bin];
        for (int bin = 0; bin < kNumBins; ++bin) {
            if (counts[bin] <= 0) continue;
            dock_bin_tuning rep{};
            rep.ligands = counts[bin];
            const BinShape def = defaults[bin];
            BinShape &bs = pick[bin];
            // torsion sweep: restarts (waves) per workgroup
            float best = 3.4e38f;
            for (int w : {2, 4, 8}) {
                if (dock_lds_bytes(32 * (bin + 1), w) > (size_t)c->lds_arena) continue;
                const int blocks = dock_blocks_per_cu(bin, w, sa.T) * c->num_cu;
                float t = 0.f;
                int e = timeit([&]() -> hipError_t {
                    hipError_t q = launch_reset(wa.counters, kMaxLists + bin * G, G, s);
                    for (int k = 0; k < G && !q; ++k)
                        q = launch_dock(bin, bin * G + k, blocks, w, g, sa, la, wa, s);
                    return q;
                }, &t);
                if (e) return e;
                if (w == def.dock_waves) rep.dock_ms_default = t;
                if (t < best) { best = t; bs.dock_waves = w; }
            }
            rep.dock_ms = best;
            // pose selection: waves per workgroup
            best = 3.4e38f;
            for (int w : {4, 8, 16}) {
                int blocks = select_blocks_per_cu(bin, w, sa.R, sa.K) * c->num_cu;
                blocks = blocks > la.L ? la.L : blocks;
                float t = 0.f;
                int e = timeit([&]() -> hipError_t {
                    hipError_t q = launch_reset(wa.counters, 2 * kMaxLists + bin * G, G, s);
                    for (int k = 0; k < G && !q; ++k)
                        q = launch_select(bin, bin * G + k, blocks, w, g, sa, la, wa, oa, -1, s);
                    return q;
                }, &t);
                if (e) return e;
                if (w == def.select_waves) rep.select_ms_default = t;
                if (t < best) { best = t; bs.select_waves = w; }
            }
            rep.select_ms = best;
            // final alignment: waves per workgroup and workgroups per CU
            best = 3.4e38f;
            for (int w : {2, 4, 8}) {
                const int occ = falign_blocks_per_cu(bin, w);
                for (int per : {1, 2, 4, 0}) {
                    if (per >= occ) continue;  // same as 0 (all that fit)
                    const int blocks = (per > 0 ? per : occ) * c->num_cu;
                    for (int xg : {0, 1}) {
                        float t = 0.f;
                        int e = timeit([&]() -> hipError_t {
                            hipError_t q = hipSuccess;
                            for (int k = 0; k < G && !q; ++k)
                                q = launch_falign(bin, bin * G + k, blocks, w, g, sa, la, wa, oa,
                                                  -1, xg ? kXcds : 0, s);
                            return q;
                        }, &t);
                        if (e) return e;
                        if (w == def.falign_waves && per == def.falign_per_cu &&
                            xg == def.falign_xcd)
                            rep.falign_ms_default = t;
                        if (t < best) {
                            best = t;
                            bs.falign_waves = w;
                            bs.falign_per_cu = per;
                            bs.falign_xcd = xg;
                        }
                    }
                }
            }
            rep.falign_ms = best;
            rep.dock_waves = bs.dock_waves;
            rep.select_waves = bs.select_waves;
            rep.falign_waves = bs.falign_waves;
            rep.falign_per_cu = bs.falign_per_cu;
            rep.falign_xcd = bs.falign_xcd;
            if (out) out[bin] = rep;
        }
        c->tuned[tune_key(sa)] = pick;
        return DOCK_OK;
    };
    const int rc3 = body();
    (void)hipStreamSynchronize(s);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(d);
    return rc3;
}

int dock_set_tuning(dock_ctx *c, const dock_params *p, const dock_bin_tuning *table) {
    if (!c) return fail(DOCK_EINVAL, "ctx is NULL");
    const int rc = check_params(p);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(c->mu);
    SearchArgs sa{};
    sa.R = p->restarts;
    sa.T = p->torsion_steps;
    sa.A = p->align_steps;
    sa.K = p->top_k;
    sa.P = p->sweep_passes;
    if (!table) {
        c->tuned.erase(tune_key(sa));
        return DOCK_OK;
    }
    std::array<BinShape, kNumBins> pick;
    for (int bin = 0; bin < kNumBins; ++bin) {
        const dock_bin_tuning &t = table[bin];
        BinShape b;
        if (t.ligands > 0) {
            if (t.dock_waves < 1 || t.dock_waves > 8 ||
                dock_lds_bytes(32 * (bin + 1), t.dock_waves) > (size_t)c->lds_arena)
                return fail(DOCK_EINVAL, "dock_waves must be in [1,8] and fit the LDS");
            if (t.select_waves < 1 || t.select_waves > 16)
                return fail(DOCK_EINVAL, "select_waves must be in [1,16]");
            if (t.falign_waves < 1 || t.falign_waves > 8)
                return fail(DOCK_EINVAL, "falign_waves must be in [1,8]");
            if (t.falign_per_cu < 0) return fail(DOCK_EINVAL, "falign_per_cu must be >= 0");
            if (t.falign_xcd != 0 && t.falign_xcd != 1)
                return fail(DOCK_EINVAL, "falign_xcd must be 0 or 1");
            b.falign_xcd = t.falign_xcd;
            b.dock_waves = t.dock_waves;
            b.select_waves = t.select_waves;
            b.falign_waves = t.falign_waves;
            b.falign_per_cu = t.falign_per_cu;
        }
        pick[bin] = b;
    }
    c->tuned[tune_key(sa)] = pick;
    return DOCK_OK;
}

int dock_submit(dock_ctx *c, int32_t pocket, const dock_library *lib, const dock_params *p,
                dock_results *o, uint64_t *ticket) {
    if (!c || !ticket) return fail(DOCK_EINVAL, "NULL argument");
    int rc = check_params(p);
    if (rc) return rc;
    rc = check_library_shape(lib);
    if (rc) return rc;
    rc = check_results(o, lib->n_ligands);
    if (rc) return rc;
    const int L = lib->n_ligands;
    if (L > 0 && (lib->atom_off[L] != lib->n_atoms_total || lib->bond_off[L] != lib->n_bonds_total ||
                  lib->rot_off[L] != lib->n_rot_total))
        return fail(DOCK_EINVAL, "offset totals differ from the declared totals");
    std::lock_guard<std::mutex> lk(c->mu);
    auto it = c->pockets.find(pocket);
    if (it == c->pockets.end()) return fail(DOCK_ENOENT, "unknown pocket");
    HIP_TRY(hipSetDevice(c->device));
    const long long A = lib->n_atoms_total, Nb = lib->n_bonds_total, Nr = lib->n_rot_total;
    Ticket t;
    const SubmitLayout sl = submit_layout(lib, p, o, &t);
    const size_t off = sl.inputs, so = sl.results;
    const size_t i_ao = sl.i_ao, i_xyz = sl.i_xyz, i_ty = sl.i_ty, i_bo = sl.i_bo, i_b = sl.i_b,
                 i_ro = sl.i_ro, i_rb = sl.i_rb, i_rm = sl.i_rm;
    const size_t dev_bytes = off + so;
    // admission: library + results + workspace growth must fit in the budget next to
    // the admitted work (or, without a budget, in free memory less a reserve)
    hipStream_t s_pick = nullptr;
    {
        const WsLayout wl = ws_layout(lib, p, o->trace != nullptr);
        s_pick = c->submit_streams[c->next_submit % c->submit_streams.size()];
        const size_t have_ws = c->ws.count(s_pick) ? c->ws[s_pick].bytes : 0;
        const size_t growth = wl.total > have_ws ? ws_grown_bytes(wl.total) - have_ws : 0;
        const size_t need = dev_bytes + growth;
        if (c->budget > 0) {
            size_t held = c->inflight;
            for (auto u : c->submit_streams) held += c->ws.count(u) ? c->ws[u].bytes : 0;
            if (held + need > c->budget) {
                // release the workspaces of submit streams with nothing in flight
                for (auto u : c->submit_streams) {
                    if (c->stream_tickets[u] > 0 || !c->ws.count(u) || !c->ws[u].base) continue;
                    HIP_TRY(hipStreamSynchronize(u));
                    HIP_TRY(hipFree(c->ws[u].base));
                    held -= c->ws[u].bytes;
                    c->ws[u].base = nullptr;
                    c->ws[u].bytes = 0;
                }
            }
            const size_t have_now = c->ws.count(s_pick) ? c->ws[s_pick].bytes : 0;
            const size_t need_now = dev_bytes + (wl.total > have_now ? ws_grown_bytes(wl.total) - have_now : 0);
            if (held + need_now > c->budget)
                return fail(DOCK_EAGAIN, "request does not fit in the device-memory budget now (" +
                                             std::to_string(held) + " B held, " +
                                             std::to_string(need_now) + " B needed, budget " +
                                             std::to_string(c->budget) + " B)");
        } else {
            size_t freeb = 0, totalb = 0;
            HIP_TRY(hipMemGetInfo(&freeb, &totalb));
            if (need + c->reserve_bytes > freeb) return fail(DOCK_EAGAIN, "not enough free device memory");
        }
    }
    hipStream_t s = s_pick;
    c->next_submit += 1;
    char *d = nullptr;
    if (hipMallocAsync((void **)&d, dev_bytes > 0 ? dev_bytes : 256, s) != hipSuccess) {
        (void)hipGetLastError();
        return fail(DOCK_EAGAIN, "device allocation failed");
    }
    // one pinned buffer per ticket: the inputs (same layout as on the device, so
    // one copy moves them all) followed by the results
    void *pinned = nullptr;
    size_t pcap = 0;
    if (pinned_get(c, off + (so > 0 ? so : 256), &pinned, &pcap) != DOCK_OK) {
        hipFreeAsync(d, s);
        return DOCK_ENOMEM;
    }
    t.host_stage = (char *)pinned + off;
    t.pinned = pinned;
    t.pinned_cap = pcap;
    // inputs are copied into pinned memory before return: the caller may free its own
    char *h = (char *)pinned;
    auto put = [&](size_t at, const void *src, size_t b) {
        if (b) std::memcpy(h + at, src, b);
    };
    if (L > 0) {
        put(i_ao, lib->atom_off, (size_t)(L + 1) * 4);
        put(i_xyz, lib->xyz, (size_t)A * 12);
        put(i_ty, lib->type, (size_t)A);
        put(i_bo, lib->bond_off, (size_t)(L + 1) * 4);
        put(i_b, lib->bond, (size_t)Nb * 8);
        put(i_ro, lib->rot_off, (size_t)(L + 1) * 4);
        put(i_rb, lib->rot_bond, (size_t)Nr * 8);
        put(i_rm, lib->rot_mask, (size_t)Nr * lib->mask_words * 8);
    }
    hipError_t e = off ? hipMemcpyAsync(d, h, off, hipMemcpyHostToDevice, s) : hipSuccess;
    if (e) {
        hipStreamSynchronize(s);
        hipFreeAsync(d, s);
        pinned_put(c, pinned, pcap);
        return fail(DOCK_EDEVICE, std::string("input copy failed: ") + hipGetErrorString(e));
    }
    dock_library dl = *lib;
    dl.atom_off = (const int32_t *)(d + i_ao);
    dl.xyz = (const float *)(d + i_xyz);
    dl.type = (const uint8_t *)(d + i_ty);
    dl.bond_off = (const int32_t *)(d + i_bo);
    dl.bond = (const int32_t *)(d + i_b);
    dl.rot_off = (const int32_t *)(d + i_ro);
    dl.rot_bond = (const int32_t *)(d + i_rb);
    dl.rot_mask = (const uint64_t *)(d + i_rm);
    char *dr = d + off;
    dock_results dres{};
    dres.best_score = (float *)(dr + t.o_best);
    dres.n_poses = (int32_t *)(dr + t.o_np);
    dres.status = (int32_t *)(dr + t.o_st);
    dres.pose_score = (float *)(dr + t.o_ps);
    dres.pose_restart = (int32_t *)(dr + t.o_pr);
    dres.pose_xyz = o->pose_xyz ? (float *)(dr + t.o_xyz) : nullptr;
    dres.restart_score = o->restart_score ? (float *)(dr + t.o_rs) : nullptr;
    dres.trace = o->trace ? (uint16_t *)(dr + t.o_tr) : nullptr;
    dres.final_trace = o->final_trace ? (uint16_t *)(dr + t.o_ft) : nullptr;
    dres.pose_contacts = o->pose_contacts ? (int32_t *)(dr + t.o_pc) : nullptr;
    int rc2 = enqueue_batch(c, it->second, &dl, p, &dres, s);
    if (rc2) {
        hipStreamSynchronize(s);
        hipFreeAsync(d, s);
        pinned_put(c, pinned, pcap);
        return rc2;
    }
    e = hipMemcpyAsync(t.host_stage, dr, so, hipMemcpyDeviceToHost, s);
    if (!e) e = hipFreeAsync(d, s);
    if (!e) e = hipEventCreateWithFlags(&t.done, hipEventDisableTiming);
    if (!e) e = hipEventRecord(t.done, s);
    if (e) {
        hipStreamSynchronize(s);
        pinned_put(c, pinned, pcap);
        return fail(DOCK_EDEVICE, std::string("enqueue failed: ") + hipGetErrorString(e));
    }
    t.pocket = pocket;
    t.user = *o;
    t.dev_bytes = dev_bytes;
    t.stream = s;
    c->inflight += dev_bytes;
    c->stream_tickets[s] += 1;
    it->second.busy += 1;
    const uint64_t id = c->next_ticket++;
    c->tickets[id] = t;
    *ticket = id;
    return DOCK_OK;
}

int dock_request_bytes(const dock_library *lib, const dock_params *p, const dock_results *o,
                       uint64_t *bytes) {
    if (!bytes) return fail(DOCK_EINVAL, "bytes is NULL");
    int rc = check_params(p);
    if (rc) return rc;
    rc = check_library_shape(lib);
    if (rc) return rc;
    if (!o) return fail(DOCK_EINVAL, "results is NULL");
    Ticket t;
    const SubmitLayout sl = submit_layout(lib, p, o, &t);
    const WsLayout wl = ws_layout(lib, p, o->trace != nullptr);
    *bytes = (uint64_t)(sl.inputs + sl.results + ws_grown_bytes(wl.total));
    return DOCK_OK;
}

static int finish_ticket(dock_ctx *c, std::map<uint64_t, Ticket>::iterator it) {
    Ticket &t = it->second;
    const char *h = (const char *)t.host_stage;
    const dock_results &u = t.user;
    const size_t L = t.L, K = t.K, R = t.R;
    if (L > 0) {
        std::memcpy(u.best_score, h + t.o_best, L * 4);
        std::memcpy(u.n_poses, h + t.o_np, L * 4);
        std::memcpy(u.status, h + t.o_st, L * 4);
        std::memcpy(u.pose_score, h + t.o_ps, L * K * 4);
        std::memcpy(u.pose_restart, h + t.o_pr, L * K * 4);
        if (u.pose_xyz) std::memcpy(u.pose_xyz, h + t.o_xyz, (size_t)t.A * K * 12);
        if (u.restart_score) std::memcpy(u.restart_score, h + t.o_rs, L * R * 4);
        if (u.trace) std::memcpy(u.trace, h + t.o_tr, (size_t)t.trace_len * 2);
        if (u.final_trace) std::memcpy(u.final_trace, h + t.o_ft, L * K * 2);
        if (u.pose_contacts) std::memcpy(u.pose_contacts, h + t.o_pc, L * K * 4);
    }
    hipEventDestroy(t.done);
    pinned_put(c, t.pinned, t.pinned_cap);
    c->inflight -= t.dev_bytes < c->inflight ? t.dev_bytes : c->inflight;
    c->stream_tickets[t.stream] -= 1;
    auto pk = c->pockets.find(t.pocket);
    if (pk != c->pockets.end() && pk->second.busy > 0) pk->second.busy -= 1;
    c->tickets.erase(it);
    return DOCK_OK;
}

int dock_poll(dock_ctx *c, uint64_t ticket, int32_t *done) {
    if (!c || !done) return fail(DOCK_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(c->mu);
    auto it = c->tickets.find(ticket);
    if (it == c->tickets.end()) return fail(DOCK_ENOENT, "unknown ticket");
    const hipError_t q = hipEventQuery(it->second.done);
    if (q == hipErrorNotReady) {
        *done = 0;
        return DOCK_OK;
    }
    if (q != hipSuccess) return fail(DOCK_EDEVICE, std::string("event query: ") + hipGetErrorString(q));
    *done = 1;
    return finish_ticket(c, it);
}

int dock_set_timing(dock_ctx *c, int enable) {
    if (!c) return fail(DOCK_EINVAL, "ctx is NULL");
    std::lock_guard<std::mutex> lk(c->mu);
    HIP_TRY(hipSetDevice(c->device));
    if (enable && !c->d_scored) {
        if (hipMalloc(&c->d_scored, sizeof(unsigned long long)) != hipSuccess) {
            c->d_scored = nullptr;
            (void)hipGetLastError();
            return fail(DOCK_ENOMEM, "timing counter allocation failed");
        }
        HIP_TRY(hipMemset(c->d_scored, 0, sizeof(unsigned long long)));
    }
    c->timing = enable != 0;
    return DOCK_OK;
}

int dock_get_timing(dock_ctx *c, dock_timing *out) {
    if (!c || !out) return fail(DOCK_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(c->mu);
    HIP_TRY(hipSetDevice(c->device));
    dock_timing t{};
    for (auto &m : c->marks) {
        HIP_TRY(hipEventSynchronize(m[4]));
        float a = 0.f, al = 0.f, b = 0.f, d = 0.f;
        HIP_TRY(hipEventElapsedTime(&a, m[0], m[1]));
        HIP_TRY(hipEventElapsedTime(&al, m[1], m[2]));
        HIP_TRY(hipEventElapsedTime(&b, m[1], m[3]));
        HIP_TRY(hipEventElapsedTime(&d, m[3], m[4]));
        t.prep_ms += a;
        t.align_ms += al;
        t.dock_ms += b;
        t.final_ms += d;
        t.calls += 1;
        for (auto &e : m) (void)hipEventDestroy(e);
    }
    c->marks.clear();
    if (c->d_scored) {
        unsigned long long v = 0;
        HIP_TRY(hipDeviceSynchronize());
        HIP_TRY(hipMemcpy(&v, c->d_scored, sizeof(v), hipMemcpyDeviceToHost));
        HIP_TRY(hipMemset(c->d_scored, 0, sizeof(v)));
        t.scored_samples = (int64_t)v;
    }
    *out = t;
    return DOCK_OK;
}

int dock_wait(dock_ctx *c, uint64_t ticket) {
    if (!c) return fail(DOCK_EINVAL, "ctx is NULL");
    // Poll under the lock so a concurrent dock_poll cannot retire the ticket
    // (and destroy its event) while this thread waits on it.
    for (;;) {
        {
            std::lock_guard<std::mutex> lk(c->mu);
            auto it = c->tickets.find(ticket);
            if (it == c->tickets.end()) return fail(DOCK_ENOENT, "unknown ticket");
            const hipError_t q = hipEventQuery(it->second.done);
            if (q == hipSuccess) return finish_ticket(c, it);
            if (q != hipErrorNotReady)
                return fail(DOCK_EDEVICE, std::string("event query: ") + hipGetErrorString(q));
        }
        std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
}

}  // extern "C"
