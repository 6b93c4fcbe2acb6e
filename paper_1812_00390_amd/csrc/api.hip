// C ABI of the library: mesh and solver objects, step sequencing for the
// three integrators, graph replay of step chunks, Step 6 and the FP64
// reductions, checkpoints, and batched multi-instance stepping.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "fvlbm_internal.h"

using namespace fvlbm;

namespace {

thread_local std::string g_err;

fvlbm_status fail(fvlbm_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// bytes of one copy of the distributions (np cells)
size_t state_copy_bytes(int storage, int np) {
    if (storage == FVLBM_STORE_I16_DEV) return (size_t)np * (Q * 2 + 1);   // nine int16 planes + exponent plane
    return (size_t)Q * np * (storage == FVLBM_STORE_FP16_DEV ? 2 : 4);
}
int n_fbufs(int scheme) { return scheme == FVLBM_SCHEME_RK4 ? 3 : 2; }

// RK4 coefficients of Eq. 17, read as f(k+1) = f(0) + beta_(k+1) dt RHS(f(k))
constexpr double BETA[4] = {0.25, 1.0 / 3.0, 0.5, 1.0};

struct Layout {
    size_t fbuf[3], r32, mc, snap[2], partial, scal, flag, out, total;
};

// FP16 storage's moment carry: 3 FP16 planes of np (see the step kernel's ConsF16)
size_t carry_bytes(int storage, int np) { return storage == FVLBM_STORE_FP16_DEV ? (size_t)3 * np * 2 : 0; }

Layout layout(int n, int np, const fvlbm_params &p) {
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t b) { size_t o = off; off = align256(off + b); return o; };
    size_t fb = state_copy_bytes(p.storage, np);
    for (int k = 0; k < 3; k++) L.fbuf[k] = k < n_fbufs(p.scheme) ? take(fb) : 0;
    L.r32 = take((size_t)Q * np * sizeof(float));
    L.mc = take(carry_bytes(p.storage, np));
    L.snap[0] = take((size_t)2 * n * sizeof(double));
    L.snap[1] = take((size_t)2 * n * sizeof(double));
    L.partial = take((size_t)2 * reduce_blocks(n * MAX_NF) * sizeof(double));   // also wall-face sums
    L.scal = take(8 * sizeof(double));
    L.flag = take(sizeof(int) * 4);
    L.out = take((size_t)Q * n * sizeof(double));   // FP64 staging for copy-out (rho,u or f or rhs)
    L.total = off;
    return L;
}

enum Kind { E0 = 0, E1, R1, R2, R3, R4, F0, F1, A0, A1, RH0, RH1, RH2, N_KINDS };
// stage kinds whose update is base + coef RHS (descriptor mode 0)
bool mode0(int k) { return k <= R4; }

}  // namespace

struct fvlbm_mesh {
    MeshDev dev;
    int refs = 0;              // solvers holding the mesh
    bool destroyed = false;    // fvlbm_mesh_destroy was called while solvers held it: freed with the last one
};

struct fvlbm_solver {
    fvlbm_mesh *mesh = nullptr;
    fvlbm_params p{};
    hipStream_t stream = nullptr;
    double dt = 0;
    RefDev ref{};
    char *buf = nullptr;
    Layout L{};
    int cur = 0;               // which distribution buffer holds the state (Euler / AB2)
    int64_t steps = 0;
    int snap_cur = -1;         // buffer of the newest snapshot, -1 none
    int64_t snap_step = -1;
    bool res_valid = false;    // the residual scalar holds the change between the last two snapshots
    bool have_prev = false;    // AB2 history valid
    int lag = 1000;
    bool failed = false;
    int batch_refs = 0;        // batches holding the solver
    bool destroyed = false;    // fvlbm_solver_destroy was called while a batch held it: freed with the last one
    InstDesc *desc_dev = nullptr;   // [N_KINDS]
    InstDesc desc_host[N_KINDS];    // host copies (a single instance's first-load values go as kernel arguments)
    UnitTable ut;
    Schedule sched;
    const TileTables *tiles = nullptr;
    // graph cache: key (start buffer, steps)
    std::map<std::pair<int, int>, hipGraphExec_t> graphs;
    ~fvlbm_solver();
};

// One instantiated batch graph, with what a membership change needs to re-point
// its kernel nodes in place: the template it was instantiated from (whose node
// handles name the exec's nodes), each node's descriptor kind and cell kind, and
// each node's argument storage.
struct BatchGraph {
    struct Node {
        hipGraphNode_t node;
        int k, t;                     // descriptor kind (stage), cell kind (3 + t face slots)
        std::unique_ptr<StageArgs> args;
        void *argv[16];               // argv[0] = args, argv[1..14] = argument pointers
    };
    hipGraphExec_t exec = nullptr;
    hipGraph_t tmpl = nullptr;
    std::vector<std::unique_ptr<Node>> nodes;
    unsigned kinds = 0;               // cell kinds with units when built (bit t)
};

struct fvlbm_batch {
    std::vector<fvlbm_solver *> members;
    InstDesc *desc_dev = nullptr;     // [N_KINDS][n]
    double **res_src = nullptr;       // device: each member's residual scalar, then n gathered values
    int res_cap = 0;                  // members res_src has room for
    UnitTable ut[2];                  // by face-slot count (3, 4)
    int h2max[2] = {0, 0};
    int h1max[2] = {0, 0};
    int scheme = 0, storage = 0;
    hipStream_t stream = nullptr;
    std::map<std::pair<int, int>, BatchGraph> graphs;
    Schedule sched;
    int64_t graph_builds = 0, graph_updates = 0;   // instantiated, and re-pointed on a membership change
};

namespace {

// Callers synchronize the stream first: a graph exec, descriptor array or
// unit table must not be destroyed while queued work may still use it.
void free_graphs(std::map<std::pair<int, int>, hipGraphExec_t> &g) {
    for (auto &kv : g) hipGraphExecDestroy(kv.second);
    g.clear();
}
void free_graphs(std::map<std::pair<int, int>, BatchGraph> &g) {
    for (auto &kv : g) {
        hipGraphExecDestroy(kv.second.exec);
        hipGraphDestroy(kv.second.tmpl);
    }
    g.clear();
}

// Build the unit table (instance, tile) for a list of (instance, n_cells).
fvlbm_status make_units(const std::vector<std::pair<int, int>> &inst, int block, UnitTable &ut) {
    std::vector<int2> units;
    for (auto &pr : inst)
        for (int t = 0; t * block < pr.second; t++) units.push_back(make_int2(pr.first, t));
    if (ut.units) { hipFree(ut.units); ut.units = nullptr; }
    if (!ut.queue) {   // the persistent form's work queue: zero, and left zero by every launch
        const size_t qb = 9 * 128;   // eight per-XCD ticket counters and a leaving count, one line each
        if (hipMalloc(&ut.queue, qb) != hipSuccess) return fail(FVLBM_E_NOMEM, "work queue allocation failed");
        if (hipMemset(ut.queue, 0, qb) != hipSuccess) return fail(FVLBM_E_DEVICE, "work queue clear failed");
    }
    ut.n_units = (int)units.size();
    ut.block = block;
    ut.direct = inst.size() == 1 && inst[0].first == 0;   // unit b is (instance 0, tile b): no table lookup
    if (units.empty() || ut.direct) return FVLBM_OK;
    if (hipMalloc(&ut.units, units.size() * sizeof(int2)) != hipSuccess) return fail(FVLBM_E_NOMEM, "unit table allocation failed");
    if (hipMemcpy(ut.units, units.data(), units.size() * sizeof(int2), hipMemcpyHostToDevice) != hipSuccess)
        return fail(FVLBM_E_DEVICE, "unit table copy failed");
    return FVLBM_OK;
}

void *fptr(fvlbm_solver *s, int k) { return s->buf + s->L.fbuf[k]; }
__half *carry_ptr(fvlbm_solver *s) {
    return s->p.storage == FVLBM_STORE_FP16_DEV ? reinterpret_cast<__half *>(s->buf + s->L.mc) : nullptr;
}

InstDesc base_desc(fvlbm_solver *s, const TileTables *tt) {
    const MeshDev &m = s->mesh->dev;
    InstDesc d{};
    d.vxy = m.vxy; d.dxy = m.dxy;
    d.lnbr = tt->lnbr; d.halo_idx = tt->halo_idx; d.halo_code = tt->halo_code;
    d.h1s = tt->h1max; d.h2s = tt->h2max;
    d.n_cells = m.n_cells; d.np = m.np;
    d.inv_tau = (float)(1.0 / s->p.tau);
    d.ref = s->ref;
    d.n_groups = m.n_groups;
    for (int g = 0; g < m.n_groups; g++) {
        const fvlbm_bc &b = m.groups_host[g];
        d.groups[g].kind = b.kind;
        d.groups[g].internal = b.internal;
        d.groups[g].ux = (float)b.u[0];
        d.groups[g].uy = (float)b.u[1];
        d.groups[g].drho = (float)(b.rho - (double)s->ref.rho0);
        d.groups[g].rho = (float)b.rho;
    }
    d.rhs_prev = reinterpret_cast<float *>(s->buf + s->L.r32);
    d.mcarry = nullptr;
    return d;
}

// Descriptors of every stage kind for one solver, for tile tables tt.
void fill_descs(fvlbm_solver *s, const TileTables *tt, InstDesc out[N_KINDS]) {
    InstDesc b = base_desc(s, tt);
    auto set = [&](int k, int src, int base, int dst, double coef, int mode) {
        out[k] = b;
        out[k].src = fptr(s, src);
        out[k].base = fptr(s, base);
        out[k].dst = dst >= 0 ? fptr(s, dst) : (void *)(s->buf + s->L.r32);
        out[k].coef = (float)coef;
        out[k].mode = mode;
    };
    const double dt = s->dt;
    set(E0, 0, 0, 1, dt, 0);
    set(E1, 1, 1, 0, dt, 0);
    if (s->p.scheme == FVLBM_SCHEME_RK4) {
        set(R1, 0, 0, 1, BETA[0] * dt, 0);
        set(R2, 1, 0, 2, BETA[1] * dt, 0);
        set(R3, 2, 0, 1, BETA[2] * dt, 0);
        set(R4, 1, 0, 0, BETA[3] * dt, 0);   // in place on f(0): each cell reads only its own base value
    } else {
        out[R1] = out[R2] = out[R3] = out[R4] = out[E0];
    }
    set(F0, 0, 0, 1, dt, 1);
    set(F1, 1, 1, 0, dt, 1);
    set(A0, 0, 0, 1, dt, 2);
    set(A1, 1, 1, 0, dt, 2);
    set(RH0, 0, 0, -1, 0, 3);
    set(RH1, 1, 1, -1, 0, 3);
    set(RH2, 2, 2, -1, 0, 3);
    // the stage that ends a step adds the carried moment residual back and rewrites it
    for (int k : {E0, E1, R4, F0, F1, A0, A1}) out[k].mcarry = carry_ptr(s);
}

// The sequence of stage kinds of one step, given the solver's position.
void step_kinds(int scheme, int cur, bool have_prev, std::vector<int> &ks) {
    ks.clear();
    if (scheme == FVLBM_SCHEME_RK4) { ks = {R1, R2, R3, R4}; return; }
    if (scheme == FVLBM_SCHEME_EULER) { ks.push_back(cur == 0 ? E0 : E1); return; }
    if (!have_prev) ks.push_back(cur == 0 ? F0 : F1);
    else ks.push_back(cur == 0 ? A0 : A1);
}

void advance_position(int scheme, int &cur, bool &have_prev) {
    if (scheme != FVLBM_SCHEME_RK4) cur ^= 1;
    if (scheme == FVLBM_SCHEME_AB2) have_prev = true;
}

hipError_t take_snapshot(fvlbm_solver *s) {
    const MeshDev &m = s->mesh->dev;
    int nxt = s->snap_cur < 0 ? 0 : (s->snap_cur ^ 1);
    double *snap_new = reinterpret_cast<double *>(s->buf + s->L.snap[nxt]);
    const double *snap_old = s->snap_cur < 0 ? nullptr : reinterpret_cast<double *>(s->buf + s->L.snap[s->snap_cur]);
    double *partial = reinterpret_cast<double *>(s->buf + s->L.partial);
    double *scal = reinterpret_cast<double *>(s->buf + s->L.scal);
    hipError_t e = launch_snapshot(fptr(s, s->cur), s->p.storage, m.n_cells, m.np, s->ref, carry_ptr(s),
                                   snap_new, snap_old, partial, s->stream);
    if (e == hipSuccess && snap_old) e = launch_finish_sums(partial, reduce_blocks(m.n_cells), scal, 1, s->stream);
    s->snap_cur = nxt;
    s->snap_step = s->steps;
    s->res_valid = snap_old != nullptr;
    return e;
}

// Build (or fetch) a graph replaying `nsteps` steps starting from buffer `cur`.
hipGraphExec_t solver_graph(fvlbm_solver *s, int cur, int nsteps) {
    auto key = std::make_pair(cur, nsteps);
    auto it = s->graphs.find(key);
    if (it != s->graphs.end()) return it->second;
    hipGraph_t g;
    if (hipGraphCreate(&g, 0) != hipSuccess) return nullptr;
    std::vector<int> ks;
    std::vector<std::unique_ptr<void *[]>> argstore;
    hipGraphNode_t prev = nullptr;
    int c = cur;
    bool hp = true;
    bool ok = true;
    for (int it2 = 0; it2 < nsteps && ok; it2++) {
        step_kinds(s->p.scheme, c, hp, ks);
        for (int k : ks) {
            argstore.emplace_back(new void *[16]);
            void **ab = argstore.back().get();
            ab[0] = new char[sizeof(StageArgs)];
            hipGraphNode_t node;
            ok = add_stage_node(g, &node, prev ? &prev : nullptr, prev ? 1 : 0, s->desc_dev + k, s->ut,
                                s->mesh->dev.nf, s->p.storage, s->sched.xcd_remap, s->sched.persistent, s->tiles->h2max,
                                s->tiles->h1max, mode0(k), ab, &s->desc_host[k]) == hipSuccess;
            prev = node;
            if (!ok) break;
        }
        advance_position(s->p.scheme, c, hp);
    }
    hipGraphExec_t ex = nullptr;
    if (ok && hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) ex = nullptr;
    for (auto &a : argstore) delete[] static_cast<char *>(a[0]);
    hipGraphDestroy(g);
    if (ex) s->graphs[key] = ex;
    return ex;
}

constexpr int GRAPH_CHUNK = 32;

// Steps replayed by the next graph for `left` steps to go: `chunk` (a power
// of two) while at least that many remain, then the largest power of two (so
// any count uses a handful of graph sizes, each cached by start buffer and size).
int graph_steps(int64_t left, int chunk = GRAPH_CHUNK) {
    if (left >= chunk) return chunk;
    int c = 1;
    while (2 * c <= left) c *= 2;
    return c;
}
// A batch replays graphs of 8 steps: its membership changes as requests come and
// go (each change instantiates new graphs), and a graph's instantiation time grows
// with its node count (steps x stages x cell kinds).
constexpr int BATCH_GRAPH_CHUNK = 8;

// Enqueue n steps without snapshots.  dry: only instantiate the graphs the
// call would replay (the caller saves and restores the solver's position).
fvlbm_status enqueue_steps(fvlbm_solver *s, int64_t n, bool dry = false) {
    std::vector<int> ks;
    int64_t done = 0;
    const int nf = s->mesh->dev.nf;
    while (done < n) {
        int64_t left = n - done;
        bool graphable = s->p.scheme != FVLBM_SCHEME_AB2 || s->have_prev;   // (the first AB2 step is an Euler step)
        if (graphable) {
            const int g = graph_steps(left);
            hipGraphExec_t ex = solver_graph(s, s->cur, g);
            if (!ex) return fail(FVLBM_E_DEVICE, "graph build failed");
            if (!dry && hipGraphLaunch(ex, s->stream) != hipSuccess) return fail(FVLBM_E_DEVICE, "graph launch failed");
            for (int k = 0; k < g; k++) advance_position(s->p.scheme, s->cur, s->have_prev);
            done += g;
            s->steps += g;
            continue;
        }
        if (dry) {
            advance_position(s->p.scheme, s->cur, s->have_prev);
            done++;
            s->steps++;
            continue;
        }
        step_kinds(s->p.scheme, s->cur, s->have_prev, ks);
        for (int k : ks) {
            hipError_t e = launch_stage(s->desc_dev + k, s->ut, nf, s->p.storage, s->sched.xcd_remap, s->sched.persistent,
                                        s->tiles->h2max, s->tiles->h1max, mode0(k), s->stream, &s->desc_host[k]);
            if (e != hipSuccess) return fail(FVLBM_E_DEVICE, std::string("stage launch failed: ") + hipGetErrorString(e));
        }
        advance_position(s->p.scheme, s->cur, s->have_prev);
        done++;
        s->steps++;
    }
    return FVLBM_OK;
}

fvlbm_status upload_descs(fvlbm_solver *s) {
    InstDesc *d = s->desc_host;
    fill_descs(s, s->tiles, d);
    if (hipMemcpy(s->desc_dev, d, sizeof(InstDesc) * N_KINDS, hipMemcpyHostToDevice) != hipSuccess)
        return fail(FVLBM_E_DEVICE, "descriptor upload failed");
    return FVLBM_OK;
}

}  // namespace

// ------------------------------------------------------------ no allocation
//
// fvlbm_macros_noalloc keeps its partial sums and non-finite flag in this
// file-scope array instead of the solver's workspace: one copy per GPU, held
// until the process ends, shared by every call on that GPU.  Host code never
// passes the array's name to a kernel (on the host it is a stand-in, not a
// device address): its device address is taken once per device with
// hipGetSymbolAddress, the device current, and kept in g_scratch.
constexpr int NOALLOC_MAX_CELLS = 1 << 24;
constexpr size_t NOALLOC_FLAG_BYTES = 256;   // the non-finite flag, then the block partial sums
constexpr size_t SCRATCH_BYTES = NOALLOC_FLAG_BYTES + (size_t)2 * ((NOALLOC_MAX_CELLS + 255) / 256) * sizeof(double);
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
std::map<int, char *> g_scratch;   // device -> address of its copy of scratch

// The current device's copy of scratch (looked up once per device).
fvlbm_status scratch_ptr(char **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(FVLBM_E_DEVICE, "hipGetDevice failed");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch.find(dev);
    if (it == g_scratch.end()) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(FVLBM_E_DEVICE, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
        it = g_scratch.emplace(dev, static_cast<char *>(p)).first;
    }
    *out = it->second;
    return FVLBM_OK;
}
}  // namespace

fvlbm_solver::~fvlbm_solver() {
    hipStreamSynchronize(stream);
    free_graphs(graphs);
    if (desc_dev) hipFree(desc_dev);
    if (ut.units) hipFree(ut.units);
    if (ut.queue) hipFree(ut.queue);
}

extern "C" {

const char *fvlbm_last_error(void) { return g_err.c_str(); }

fvlbm_status fvlbm_create_mesh(int32_t n_nodes, const double *xy, int32_t n_cells,
                               const int32_t *cell_ptr, const int32_t *cell_nodes,
                               int32_t n_bfaces, const int32_t *bface_nodes,
                               const int32_t *bface_group, int32_t n_groups,
                               const fvlbm_bc *groups, int32_t n_periodic,
                               const int32_t *periodic_pairs, const double *periodic_shift,
                               int32_t reorder, void *hip_stream, fvlbm_mesh **out) {
    if (!out) return fail(FVLBM_E_ARG, "out is null");
    *out = nullptr;
    try {
        HostTopology topo;
        std::string err;
        fvlbm_status st = build_topology(n_nodes, xy, n_cells, cell_ptr, cell_nodes, n_bfaces, bface_nodes,
                                         bface_group, n_groups, groups, n_periodic, periodic_pairs,
                                         periodic_shift, reorder, topo, err);
        if (st != FVLBM_OK) return fail(st, err);
        auto *m = new fvlbm_mesh();
        st = build_device_mesh(topo, groups, n_groups, (hipStream_t)hip_stream, m->dev, err);
        if (st != FVLBM_OK) {
            if (m->dev.block) hipFree(m->dev.block);
            delete m;
            return fail(st, err);
        }
        *out = m;
        return FVLBM_OK;
    } catch (const std::bad_alloc &) {
        return fail(FVLBM_E_NOMEM, "host allocation failed");
    } catch (...) {
        return fail(FVLBM_E_ARG, "unexpected exception in fvlbm_create_mesh");
    }
}

fvlbm_status fvlbm_mesh_info(const fvlbm_mesh *mesh, int64_t out[4]) {
    if (!mesh || !out) return fail(FVLBM_E_ARG, "null argument");
    out[0] = mesh->dev.n_cells;
    out[1] = mesh->dev.nf;
    out[2] = (int64_t)mesh->dev.bytes;
    out[3] = mesh->dev.n_boundary_cells;
    return FVLBM_OK;
}

double fvlbm_mesh_cfl_length(const fvlbm_mesh *mesh) { return mesh ? mesh->dev.cfl_length : -1.0; }

namespace {
void mesh_free(fvlbm_mesh *mesh) {
    hipDeviceSynchronize();          // solvers on any stream may still read the mesh arrays
    free_tiles(mesh->dev);
    if (mesh->dev.block) hipFree(mesh->dev.block);
    delete mesh;
}
}  // namespace

void fvlbm_mesh_destroy(fvlbm_mesh *mesh) {
    if (!mesh || mesh->destroyed) return;
    if (mesh->refs > 0) {            // solvers still read it: the last solver destroyed frees it
        mesh->destroyed = true;
        return;
    }
    mesh_free(mesh);
}

size_t fvlbm_state_bytes(const fvlbm_mesh *mesh, const fvlbm_params *p) {
    if (!mesh || !p || p->scheme < 0 || p->scheme > 2 || p->storage < 0 || p->storage > 3) return 0;
    return layout(mesh->dev.n_cells, mesh->dev.np, *p).total;
}

fvlbm_status fvlbm_init(fvlbm_mesh *mesh, const fvlbm_params *params, const double *rho0_cells,
                        const double *u0_cells, void *device_buf, size_t buf_bytes, void *hip_stream,
                        fvlbm_solver **out) {
    if (!mesh || !params || !device_buf || !out) return fail(FVLBM_E_ARG, "null argument");
    *out = nullptr;
    const fvlbm_params &p = *params;
    if (!(p.tau > 0)) return fail(FVLBM_E_PARAM, "tau must be positive");
    if (p.scheme < 0 || p.scheme > 2) return fail(FVLBM_E_PARAM, "unknown scheme");
    if (p.storage < 0 || p.storage > 3) return fail(FVLBM_E_PARAM, "unknown storage");
    if (!(p.rho0 > 0)) return fail(FVLBM_E_PARAM, "rho0 must be positive");
    if (((uintptr_t)device_buf & 255) != 0) return fail(FVLBM_E_ARG, "device buffer must be 256-byte aligned");
    const MeshDev &m = mesh->dev;
    Layout L = layout(m.n_cells, m.np, p);
    if (buf_bytes < L.total) return fail(FVLBM_E_PARAM, "state buffer too small (see fvlbm_state_bytes)");
    double dt = p.dt;
    if (dt < 0) return fail(FVLBM_E_PARAM, "dt must be >= 0");
    if (dt == 0) {
        if (!(p.cfl > 0)) return fail(FVLBM_E_PARAM, "dt == 0 needs cfl > 0");
        // Eq. 14 with |e|max = sqrt(2), |U|max = u_ref; Eq. 15 caps at 2 tau
        dt = p.cfl * m.cfl_length / (std::sqrt(2.0) + std::fabs(p.u_ref));
        dt = std::min(dt, 2.0 * p.tau);
    } else if (dt > 2.0 * p.tau && !(p.flags & FVLBM_FLAG_FORCE_DT)) {
        return fail(FVLBM_E_PARAM, "dt > 2 tau violates the collision limit (Eq. 15)");
    }
    auto s = std::make_unique<fvlbm_solver>();
    s->mesh = mesh;
    s->p = p;
    s->stream = (hipStream_t)hip_stream;
    s->dt = dt;
    double S = p.fp16_scale > 0 ? p.fp16_scale : (p.u_ref != 0 ? 3.0 * std::fabs(p.u_ref) : 0.3);
    s->ref = make_ref(p.rho0, p.u_dev[0], p.u_dev[1], S);
    s->buf = (char *)device_buf;
    s->L = L;
    s->lag = p.residual_lag > 0 ? p.residual_lag : 1000;
    if (hipMalloc(&s->desc_dev, sizeof(InstDesc) * N_KINDS) != hipSuccess) return fail(FVLBM_E_NOMEM, "descriptor allocation failed");
    {
        std::string err;
        fvlbm_status tst = get_tiles(mesh->dev, s->sched.block, &s->tiles, err);
        if (tst != FVLBM_OK) return fail(tst, err);
        if (stage_lds_bytes(s->sched.block, s->tiles->h2max, s->tiles->h1max) > stage_lds_limit()) {
            s->sched.block = 128;
            tst = get_tiles(mesh->dev, s->sched.block, &s->tiles, err);
            if (tst != FVLBM_OK) return fail(tst, err);
        }
    }
    fvlbm_status st = make_units({{0, m.n_cells}}, s->sched.block, s->ut);
    if (st != FVLBM_OK) return st;
    st = upload_descs(s.get());
    if (st != FVLBM_OK) return st;
    // Step 0 from the caller's fields (staged through the copy-out area)
    double *stage = reinterpret_cast<double *>(s->buf + L.out);
    const double *rho_dev = nullptr, *u_dev = nullptr;
    hipError_t e = hipSuccess;
    if (rho0_cells) {
        e = hipMemcpyAsync(stage, rho0_cells, (size_t)m.n_cells * sizeof(double), hipMemcpyHostToDevice, s->stream);
        rho_dev = stage;
    }
    if (e == hipSuccess && u0_cells) {
        e = hipMemcpyAsync(stage + m.n_cells, u0_cells, (size_t)2 * m.n_cells * sizeof(double), hipMemcpyHostToDevice, s->stream);
        u_dev = stage + m.n_cells;
    }
    if (e == hipSuccess)
        e = launch_init_eq(fptr(s.get(), 0), p.storage, m.n_cells, m.np, s->ref, rho_dev, u_dev,
                           m.perm_dev, p.rho0, carry_ptr(s.get()), s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return fail(FVLBM_E_DEVICE, std::string("init failed: ") + hipGetErrorString(e));
    {   // set-up of the no-allocation entry point's scratch on this device (once per device)
        char *sp = nullptr;
        fvlbm_status sst = scratch_ptr(&sp);
        if (sst != FVLBM_OK) return sst;
    }
    mesh->refs++;
    *out = s.release();
    return FVLBM_OK;
}

double fvlbm_solver_dt(const fvlbm_solver *s) { return s ? s->dt : -1.0; }

namespace {
void solver_free(fvlbm_solver *s) {
    fvlbm_mesh *m = s->mesh;
    delete s;                        // (syncs the solver's stream)
    if (m && --m->refs == 0 && m->destroyed) mesh_free(m);
}
}  // namespace

void fvlbm_solver_destroy(fvlbm_solver *s) {
    if (!s || s->destroyed) return;
    if (s->batch_refs > 0) {         // a batch still holds it: the batch frees it when destroyed
        s->destroyed = true;
        return;
    }
    solver_free(s);
}

namespace {
// fvlbm_step's sequence: steps split at residual-lag boundaries, where a
// velocity snapshot is taken.  dry: graphs only (see fvlbm_prepare).
fvlbm_status step_impl(fvlbm_solver *s, int64_t n_steps, bool dry) {
    if (!dry && s->snap_cur < 0 && s->steps % s->lag == 0) {
        if (take_snapshot(s) != hipSuccess) { s->failed = true; return fail(FVLBM_E_DEVICE, "snapshot failed"); }
    }
    int64_t left = n_steps;
    while (left > 0) {
        int64_t to_snap = s->lag - (s->steps % s->lag);
        int64_t chunk = std::min(left, to_snap);
        fvlbm_status st = enqueue_steps(s, chunk, dry);
        if (st != FVLBM_OK) { s->failed = true; return st; }
        left -= chunk;
        if (!dry && s->steps % s->lag == 0) {
            if (take_snapshot(s) != hipSuccess) { s->failed = true; return fail(FVLBM_E_DEVICE, "snapshot failed"); }
        }
    }
    return FVLBM_OK;
}
}  // namespace

fvlbm_status fvlbm_step(fvlbm_solver *s, int64_t n_steps) {
    if (!s || n_steps < 0) return fail(FVLBM_E_ARG, "bad arguments to fvlbm_step");
    if (s->failed || s->destroyed) return fail(FVLBM_E_STATE, "solver is in an error state or destroyed");
    return step_impl(s, n_steps, false);
}

fvlbm_status fvlbm_prepare(fvlbm_solver *s, int64_t n_steps) {
    if (!s || n_steps < 0) return fail(FVLBM_E_ARG, "bad arguments to fvlbm_prepare");
    if (s->failed || s->destroyed) return fail(FVLBM_E_STATE, "solver is in an error state or destroyed");
    const int cur = s->cur;
    const bool hp = s->have_prev;
    const int64_t steps = s->steps;
    fvlbm_status st = step_impl(s, n_steps, true);
    s->cur = cur;
    s->have_prev = hp;
    s->steps = steps;
    if (st != FVLBM_OK) s->failed = false;     // nothing ran: a failed graph build leaves the state intact
    return st;
}

fvlbm_status fvlbm_macros(fvlbm_solver *s, double *rho, double *u, double *stats) {
    if (!s) return fail(FVLBM_E_ARG, "null solver");
    if (s->failed || s->destroyed) return fail(FVLBM_E_STATE, "solver is in an error state or destroyed");
    const MeshDev &m = s->mesh->dev;
    double *out = reinterpret_cast<double *>(s->buf + s->L.out);
    double *scal = reinterpret_cast<double *>(s->buf + s->L.scal);
    int *flag = reinterpret_cast<int *>(s->buf + s->L.flag);
    double *partial = reinterpret_cast<double *>(s->buf + s->L.partial);
    int zero = 0;
    hipError_t e = hipMemcpyAsync(flag, &zero, sizeof(int), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess)
        e = launch_macros(fptr(s, s->cur), s->p.storage, m.n_cells, m.np, s->ref, carry_ptr(s), m.area, m.perm_dev,
                          out, out + m.n_cells, partial, flag, s->stream);
    if (e == hipSuccess) e = launch_finish_sums(partial, reduce_blocks(m.n_cells), scal, 0, s->stream);
    double sc[2] = {0, -1};
    int fl = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(sc, scal, 2 * sizeof(double), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&fl, flag, sizeof(int), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess && rho) e = hipMemcpyAsync(rho, out, (size_t)m.n_cells * sizeof(double), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess && u) e = hipMemcpyAsync(u, out + m.n_cells, (size_t)2 * m.n_cells * sizeof(double), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) { s->failed = true; return fail(FVLBM_E_DEVICE, std::string("macros failed: ") + hipGetErrorString(e)); }
    bool have_res = s->res_valid;
    if (stats) {
        stats[0] = sc[0];
        stats[1] = have_res ? sc[1] : -1.0;
        stats[2] = (double)s->steps * s->dt;
        stats[3] = (double)s->steps;
    }
    if (fl) return fail(FVLBM_E_DIVERGED, "non-finite density or velocity");
    return FVLBM_OK;
}

fvlbm_status fvlbm_macros_noalloc(fvlbm_solver *s, double *rho_dev, double *u_dev, double *stats_dev) {
    if (!s || !stats_dev) return fail(FVLBM_E_ARG, "null solver or stats");
    if (s->failed || s->destroyed) return fail(FVLBM_E_STATE, "solver is in an error state or destroyed");
    const MeshDev &m = s->mesh->dev;
    if (m.n_cells > NOALLOC_MAX_CELLS)
        return fail(FVLBM_E_ARG, "fvlbm_macros_noalloc handles meshes of at most 16777216 cells (its static scratch); "
                                 "use fvlbm_macros");
    char *sp = nullptr;
    fvlbm_status st = scratch_ptr(&sp);
    if (st != FVLBM_OK) return st;
    int *flag = reinterpret_cast<int *>(sp);
    double *partial = reinterpret_cast<double *>(sp + NOALLOC_FLAG_BYTES);
    hipError_t e = launch_zero_int(flag, 1, s->stream);
    if (e == hipSuccess)
        e = launch_macros(fptr(s, s->cur), s->p.storage, m.n_cells, m.np, s->ref, carry_ptr(s), m.area, m.perm_dev,
                          rho_dev, u_dev, partial, flag, s->stream);
    if (e == hipSuccess) e = launch_finish_sums(partial, reduce_blocks(m.n_cells), stats_dev, 0, s->stream);
    if (e == hipSuccess) e = launch_flag_out(flag, stats_dev + 1, s->stream);
    if (e != hipSuccess) return fail(FVLBM_E_DEVICE, std::string("macros (no allocation) failed: ") + hipGetErrorString(e));
    return FVLBM_OK;
}

fvlbm_status fvlbm_wall_force(fvlbm_solver *s, int32_t group, double force[2], int32_t *n_faces, double *face_p) {
    if (!s) return fail(FVLBM_E_ARG, "null solver");
    const MeshDev &m = s->mesh->dev;
    if (group < 0 || group >= m.n_groups) return fail(FVLBM_E_ARG, "group out of range");
    if (m.groups_host[group].kind != FVLBM_BC_WALL) return fail(FVLBM_E_ARG, "the force is defined on wall groups");
    const int n = m.gface_off[group + 1] - m.gface_off[group];
    if (n_faces) *n_faces = n;
    if (!force && !face_p) return FVLBM_OK;
    double *partial = reinterpret_cast<double *>(s->buf + s->L.partial);
    double *scal = reinterpret_cast<double *>(s->buf + s->L.scal);
    double *out = reinterpret_cast<double *>(s->buf + s->L.out);
    double fr[2] = {0, 0};
    hipError_t e = hipSuccess;
    if (n > 0) {
        e = launch_wall_force(fptr(s, s->cur), s->p.storage, m.np, s->ref, m.gfaces_dev + m.gface_off[group], n, m.vxy,
                              m.nf, m.groups_host[group].u[0], m.groups_host[group].u[1], partial, face_p ? out : nullptr,
                              s->stream);
        if (e == hipSuccess) e = launch_finish_sums(partial, reduce_blocks(n), scal + 2, 2, s->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(fr, scal + 2, 2 * sizeof(double), hipMemcpyDeviceToHost, s->stream);
        if (e == hipSuccess && face_p) e = hipMemcpyAsync(face_p, out, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    }
    if (e != hipSuccess) return fail(FVLBM_E_DEVICE, std::string("wall force failed: ") + hipGetErrorString(e));
    if (force) { force[0] = fr[0]; force[1] = fr[1]; }
    return FVLBM_OK;
}

fvlbm_status fvlbm_get_f(fvlbm_solver *s, double *f) {
    if (!s || !f) return fail(FVLBM_E_ARG, "null argument");
    const MeshDev &m = s->mesh->dev;
    double *out = reinterpret_cast<double *>(s->buf + s->L.out);
    hipError_t e = launch_get_f(fptr(s, s->cur), s->p.storage, m.n_cells, m.np, s->ref, m.perm_dev, out, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(f, out, (size_t)Q * m.n_cells * sizeof(double), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return fail(FVLBM_E_DEVICE, hipGetErrorString(e));
    return FVLBM_OK;
}

fvlbm_status fvlbm_set_f(fvlbm_solver *s, const double *f) {
    if (!s || !f) return fail(FVLBM_E_ARG, "null argument");
    const MeshDev &m = s->mesh->dev;
    double *stage = reinterpret_cast<double *>(s->buf + s->L.out);
    hipError_t e = hipMemcpyAsync(stage, f, (size_t)Q * m.n_cells * sizeof(double), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess)
        e = launch_set_f(fptr(s, s->cur), s->p.storage, m.n_cells, m.np, s->ref, m.perm_dev, stage, carry_ptr(s), s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return fail(FVLBM_E_DEVICE, hipGetErrorString(e));
    s->have_prev = false;
    s->snap_cur = -1;
    s->snap_step = -1;
    s->res_valid = false;
    return FVLBM_OK;
}

fvlbm_status fvlbm_rhs(fvlbm_solver *s, double *rhs) {
    if (!s || !rhs) return fail(FVLBM_E_ARG, "null argument");
    if (s->p.scheme == FVLBM_SCHEME_AB2 && s->have_prev)
        return fail(FVLBM_E_STATE, "fvlbm_rhs would overwrite the AB2 history; call it before stepping");
    const MeshDev &m = s->mesh->dev;
    double *out = reinterpret_cast<double *>(s->buf + s->L.out);
    int k = s->cur == 0 ? RH0 : (s->cur == 1 ? RH1 : RH2);
    hipError_t e = launch_stage(s->desc_dev + k, s->ut, m.nf, s->p.storage, s->sched.xcd_remap, s->sched.persistent,
                                s->tiles->h2max, s->tiles->h1max, mode0(k), s->stream, &s->desc_host[k]);
    if (e == hipSuccess) e = launch_rhs_out(reinterpret_cast<float *>(s->buf + s->L.r32), m.n_cells, m.np, m.perm_dev, out, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(rhs, out, (size_t)Q * m.n_cells * sizeof(double), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return fail(FVLBM_E_DEVICE, hipGetErrorString(e));
    return FVLBM_OK;
}

size_t fvlbm_checkpoint_bytes(const fvlbm_solver *s) {
    if (!s) return 0;
    const MeshDev &m = s->mesh->dev;
    size_t fb = state_copy_bytes(s->p.storage, m.np);
    size_t extra = s->p.scheme == FVLBM_SCHEME_AB2 ? (size_t)Q * m.np * sizeof(float) : 0;
    return 64 + fb + extra + carry_bytes(s->p.storage, m.np);
}

fvlbm_status fvlbm_checkpoint(fvlbm_solver *s, void *host_buf, size_t bytes) {
    if (!s || !host_buf || bytes < fvlbm_checkpoint_bytes(s)) return fail(FVLBM_E_ARG, "bad checkpoint buffer");
    const MeshDev &m = s->mesh->dev;
    size_t fb = state_copy_bytes(s->p.storage, m.np);
    int64_t hdr[8] = {0x46564c424d31LL, s->steps, s->p.storage, s->p.scheme, m.n_cells, s->have_prev, 0, 0};
    std::memcpy(host_buf, hdr, 64);
    hipError_t e = hipMemcpyAsync((char *)host_buf + 64, fptr(s, s->cur), fb, hipMemcpyDeviceToHost, s->stream);
    const size_t rb = s->p.scheme == FVLBM_SCHEME_AB2 ? (size_t)Q * m.np * sizeof(float) : 0;
    if (e == hipSuccess && rb)
        e = hipMemcpyAsync((char *)host_buf + 64 + fb, s->buf + s->L.r32, rb, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess && carry_ptr(s))
        e = hipMemcpyAsync((char *)host_buf + 64 + fb + rb, carry_ptr(s), carry_bytes(s->p.storage, m.np),
                           hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return fail(FVLBM_E_DEVICE, hipGetErrorString(e));
    return FVLBM_OK;
}

fvlbm_status fvlbm_restore(fvlbm_solver *s, const void *host_buf, size_t bytes) {
    if (!s || !host_buf || bytes < fvlbm_checkpoint_bytes(s)) return fail(FVLBM_E_ARG, "bad checkpoint buffer");
    const MeshDev &m = s->mesh->dev;
    int64_t hdr[8];
    std::memcpy(hdr, host_buf, 64);
    if (hdr[0] != 0x46564c424d31LL || hdr[2] != s->p.storage || hdr[3] != s->p.scheme || hdr[4] != m.n_cells)
        return fail(FVLBM_E_ARG, "checkpoint does not match this solver");
    size_t fb = state_copy_bytes(s->p.storage, m.np);
    s->cur = 0;
    hipError_t e = hipMemcpyAsync(fptr(s, 0), (const char *)host_buf + 64, fb, hipMemcpyHostToDevice, s->stream);
    const size_t rb = s->p.scheme == FVLBM_SCHEME_AB2 ? (size_t)Q * m.np * sizeof(float) : 0;
    if (e == hipSuccess && rb)
        e = hipMemcpyAsync(s->buf + s->L.r32, (const char *)host_buf + 64 + fb, rb, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess && carry_ptr(s))
        e = hipMemcpyAsync(carry_ptr(s), (const char *)host_buf + 64 + fb + rb, carry_bytes(s->p.storage, m.np),
                           hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return fail(FVLBM_E_DEVICE, hipGetErrorString(e));
    s->steps = hdr[1];
    s->have_prev = hdr[5] != 0;
    s->snap_cur = -1;
    s->snap_step = -1;
    s->res_valid = false;
    s->failed = false;
    return FVLBM_OK;
}

namespace {
bool valid_block(int b) { return b >= 64 && b <= 512 && b % 64 == 0; }
}  // namespace

fvlbm_status fvlbm_set_schedule(fvlbm_solver *s, int32_t block, int32_t xcd_remap, int32_t persistent) {
    if (!s || !valid_block(block)) return fail(FVLBM_E_ARG, "unsupported block size (a multiple of 64 from 64 to 512)");
    const TileTables *tt = nullptr;
    std::string err;
    fvlbm_status st = get_tiles(s->mesh->dev, block, &tt, err);
    if (st != FVLBM_OK) return fail(st, err);
    if (stage_lds_bytes(block, tt->h2max, tt->h1max) > stage_lds_limit()) return fail(FVLBM_E_ARG, "tile and halo do not fit the LDS at this block size");
    if (hipStreamSynchronize(s->stream) != hipSuccess) return fail(FVLBM_E_DEVICE, "stream synchronize failed");
    s->sched.block = block;
    s->sched.xcd_remap = xcd_remap ? 1 : 0;
    s->sched.persistent = persistent == 2 ? 2 : (persistent ? 1 : 0);
    s->tiles = tt;
    free_graphs(s->graphs);
    st = make_units({{0, s->mesh->dev.n_cells}}, block, s->ut);
    if (st != FVLBM_OK) return st;
    return upload_descs(s);
}

fvlbm_status fvlbm_set_stream(fvlbm_solver *s, void *hip_stream) {
    if (!s) return fail(FVLBM_E_ARG, "null solver");
    if (s->batch_refs > 0) return fail(FVLBM_E_STATE, "a batch holds the solver; its members keep the batch's stream");
    if (hipStreamSynchronize(s->stream) != hipSuccess) return fail(FVLBM_E_DEVICE, "stream synchronize failed");
    s->stream = (hipStream_t)hip_stream;
    return FVLBM_OK;
}

fvlbm_status fvlbm_get_schedule(const fvlbm_solver *s, int32_t *block, int32_t *xcd_remap, int32_t *persistent) {
    if (!s || !block || !xcd_remap || !persistent) return fail(FVLBM_E_ARG, "null argument");
    *block = s->sched.block;
    *xcd_remap = s->sched.xcd_remap;
    *persistent = s->sched.persistent;
    return FVLBM_OK;
}

// ------------------------------------------------------------------ batch

namespace {
unsigned batch_kinds(const fvlbm_batch *b) {
    return (b->ut[0].n_units ? 1u : 0u) | (b->ut[1].n_units ? 2u : 0u);
}

// (Re)build a batch's descriptors, unit tables and residual table for its
// members and schedule.  Nothing changes when the members' tiles do not fit the
// LDS at the schedule's tile size.  keep_graphs: leave the instantiated graphs
// (the caller re-points or drops them); else they are dropped.
fvlbm_status batch_build(fvlbm_batch *b, bool keep_graphs = false) {
    const int n = (int)b->members.size();
    std::vector<InstDesc> all((size_t)N_KINDS * n);
    int h2max[2] = {0, 0}, h1max[2] = {0, 0};
    for (int i = 0; i < n; i++) {
        fvlbm_solver *s = b->members[i];
        const TileTables *tt = nullptr;
        std::string err;
        fvlbm_status st = get_tiles(s->mesh->dev, b->sched.block, &tt, err);
        if (st != FVLBM_OK) return fail(st, err);
        int t = s->mesh->dev.nf - 3;
        h2max[t] = std::max(h2max[t], tt->h2max);
        h1max[t] = std::max(h1max[t], tt->h1max);
        InstDesc d[N_KINDS];
        fill_descs(s, tt, d);
        for (int k = 0; k < N_KINDS; k++) all[(size_t)k * n + i] = d[k];
    }
    for (int t = 0; t < 2; t++)
        if (stage_lds_bytes(b->sched.block, h2max[t], h1max[t]) > stage_lds_limit())
            return fail(FVLBM_E_ARG, "batch tiles do not fit the LDS at this block size");
    if (hipStreamSynchronize(b->stream) != hipSuccess) return fail(FVLBM_E_DEVICE, "stream synchronize failed");
    if (!keep_graphs) free_graphs(b->graphs);
    if (b->desc_dev) { hipFree(b->desc_dev); b->desc_dev = nullptr; }
    if (hipMalloc(&b->desc_dev, all.size() * sizeof(InstDesc)) != hipSuccess) return fail(FVLBM_E_NOMEM, "batch descriptor allocation failed");
    if (hipMemcpy(b->desc_dev, all.data(), all.size() * sizeof(InstDesc), hipMemcpyHostToDevice) != hipSuccess)
        return fail(FVLBM_E_DEVICE, "batch descriptor upload failed");
    // members' residual scalars (fvlbm_batch_residuals), then room for the gathered values
    if (b->res_cap < n) {
        if (b->res_src) { hipFree(b->res_src); b->res_src = nullptr; }
        b->res_cap = 0;
        if (hipMalloc(&b->res_src, (size_t)n * (sizeof(double *) + sizeof(double))) != hipSuccess)
            return fail(FVLBM_E_NOMEM, "batch residual table allocation failed");
        b->res_cap = n;
    }
    std::vector<double *> src(n);
    for (int i = 0; i < n; i++) src[i] = reinterpret_cast<double *>(b->members[i]->buf + b->members[i]->L.scal) + 1;
    if (hipMemcpy(b->res_src, src.data(), (size_t)n * sizeof(double *), hipMemcpyHostToDevice) != hipSuccess)
        return fail(FVLBM_E_DEVICE, "batch residual table upload failed");
    for (int t = 0; t < 2; t++) {
        b->h2max[t] = h2max[t];
        b->h1max[t] = h1max[t];
        std::vector<std::pair<int, int>> inst;
        for (int i = 0; i < n; i++)
            if (b->members[i]->mesh->dev.nf == 3 + t) inst.push_back({i, b->members[i]->mesh->dev.n_cells});
        fvlbm_status st = make_units(inst, b->sched.block, b->ut[t]);
        if (st != FVLBM_OK) return st;
    }
    return FVLBM_OK;
}

// Members for a batch of this scheme, storage and stream: usable, not repeated,
// at one buffer parity (Euler, AB2), past their first AB2 step.
fvlbm_status check_members(fvlbm_solver *const *solvers, int n, int scheme, int storage, hipStream_t stream) {
    for (int i = 0; i < n; i++) {
        fvlbm_solver *s = solvers[i];
        if (!s || s->failed || s->destroyed) return fail(FVLBM_E_ARG, "null, failed or destroyed solver in batch");
        if (s->p.scheme != scheme || s->p.storage != storage) return fail(FVLBM_E_PARAM, "batch members must share scheme and storage");
        if (s->stream != stream) return fail(FVLBM_E_PARAM, "batch members must share a stream");
        if (s->p.scheme != FVLBM_SCHEME_RK4 && s->cur != solvers[0]->cur) return fail(FVLBM_E_PARAM, "batch members must be at the same buffer parity");
        if (s->p.scheme == FVLBM_SCHEME_AB2 && !s->have_prev) return fail(FVLBM_E_PARAM, "AB2 members must have taken their first step");
        for (int j = 0; j < i; j++)
            if (solvers[j] == s) return fail(FVLBM_E_PARAM, "a solver appears twice in the batch");
    }
    return FVLBM_OK;
}
}  // namespace

fvlbm_status fvlbm_batch_create(fvlbm_solver *const *solvers, int32_t n, fvlbm_batch **out) {
    if (!solvers || n <= 0 || !out) return fail(FVLBM_E_ARG, "bad arguments to fvlbm_batch_create");
    *out = nullptr;
    auto b = std::make_unique<fvlbm_batch>();
    b->scheme = solvers[0]->p.scheme;
    b->storage = solvers[0]->p.storage;
    b->stream = solvers[0]->stream;
    b->sched = solvers[0]->sched;
    fvlbm_status cst = check_members(solvers, n, b->scheme, b->storage, b->stream);
    if (cst != FVLBM_OK) return cst;
    b->members.assign(solvers, solvers + n);
    // the first member's tile size, or the largest smaller one whose tiles fit the LDS
    fvlbm_status st = FVLBM_E_ARG;
    for (int T : {b->sched.block, 256, 128, 64}) {
        if (T > b->sched.block) continue;
        b->sched.block = T;
        st = batch_build(b.get());
        if (st != FVLBM_E_ARG) break;
    }
    if (st != FVLBM_OK) return st;
    for (fvlbm_solver *s : b->members) s->batch_refs++;
    *out = b.release();
    return FVLBM_OK;
}

fvlbm_status fvlbm_batch_get_schedule(const fvlbm_batch *b, int32_t *block, int32_t *xcd_remap, int32_t *persistent) {
    if (!b || !block || !xcd_remap || !persistent) return fail(FVLBM_E_ARG, "null argument");
    *block = b->sched.block;
    *xcd_remap = b->sched.xcd_remap;
    *persistent = b->sched.persistent;
    return FVLBM_OK;
}

namespace {
void repoint_graphs(fvlbm_batch *b);
}  // namespace

fvlbm_status fvlbm_batch_set_members(fvlbm_batch *b, fvlbm_solver *const *solvers, int32_t n) {
    if (!b || !solvers || n <= 0) return fail(FVLBM_E_ARG, "bad arguments to fvlbm_batch_set_members");
    fvlbm_status st = check_members(solvers, n, b->scheme, b->storage, b->stream);
    if (st != FVLBM_OK) return st;
    std::vector<fvlbm_solver *> old = b->members;
    b->members.assign(solvers, solvers + n);
    st = batch_build(b, true);
    if (st != FVLBM_OK) {
        b->members = old;
        if (batch_build(b, true) != FVLBM_OK) free_graphs(b->graphs);
        else repoint_graphs(b);
        return st;
    }
    repoint_graphs(b);
    for (fvlbm_solver *s : b->members) s->batch_refs++;
    // members that left and were destroyed while the batch held them are freed now
    for (fvlbm_solver *s : old)
        if (--s->batch_refs == 0 && s->destroyed) solver_free(s);
    return FVLBM_OK;
}

fvlbm_status fvlbm_batch_remove(fvlbm_batch *b, fvlbm_solver *s) {
    if (!b || !s) return fail(FVLBM_E_ARG, "bad arguments to fvlbm_batch_remove");
    std::vector<fvlbm_solver *> keep;
    keep.reserve(b->members.size());
    for (fvlbm_solver *m : b->members)
        if (m != s) keep.push_back(m);
    if (keep.size() == b->members.size()) return fail(FVLBM_E_ARG, "the solver is not a member of the batch");
    if (keep.empty()) return fail(FVLBM_E_STATE, "cannot remove the last member of a batch (destroy the batch)");
    return fvlbm_batch_set_members(b, keep.data(), (int32_t)keep.size());
}

fvlbm_status fvlbm_batch_graph_counts(const fvlbm_batch *b, int64_t *built, int64_t *repointed) {
    if (!b || !built || !repointed) return fail(FVLBM_E_ARG, "null argument");
    *built = b->graph_builds;
    *repointed = b->graph_updates;
    return FVLBM_OK;
}

fvlbm_status fvlbm_batch_set_schedule(fvlbm_batch *b, int32_t block, int32_t xcd_remap, int32_t persistent) {
    if (!b || !valid_block(block)) return fail(FVLBM_E_ARG, "unsupported block size (a multiple of 64 from 64 to 512)");
    Schedule old = b->sched;
    b->sched.block = block;
    b->sched.xcd_remap = xcd_remap ? 1 : 0;
    b->sched.persistent = (persistent && persistent != 2) ? 1 : 0;   // (the ring form is for single solvers)
    fvlbm_status st = batch_build(b);
    if (st != FVLBM_OK) {
        b->sched = old;
        batch_build(b);
    }
    return st;
}

namespace {
hipGraphExec_t batch_graph(fvlbm_batch *b, int cur, int nsteps) {
    auto key = std::make_pair(cur, nsteps);
    auto it = b->graphs.find(key);
    if (it != b->graphs.end()) return it->second.exec;
    BatchGraph bg;
    if (hipGraphCreate(&bg.tmpl, 0) != hipSuccess) return nullptr;
    bg.kinds = batch_kinds(b);
    std::vector<int> ks;
    std::vector<hipGraphNode_t> prev;
    const int n = (int)b->members.size();
    int c = cur;
    bool hp = true, ok = true;
    for (int st = 0; st < nsteps && ok; st++) {
        step_kinds(b->scheme, c, hp, ks);
        for (int k : ks) {
            std::vector<hipGraphNode_t> now;
            for (int t = 0; t < 2 && ok; t++) {
                if (b->ut[t].n_units == 0) continue;
                auto nd = std::make_unique<BatchGraph::Node>();
                nd->k = k;
                nd->t = t;
                nd->args = std::make_unique<StageArgs>();
                nd->argv[0] = nd->args.get();
                ok = add_stage_node(bg.tmpl, &nd->node, prev.empty() ? nullptr : prev.data(), (int)prev.size(),
                                    b->desc_dev + (size_t)k * n, b->ut[t], 3 + t, b->storage,
                                    b->sched.xcd_remap, b->sched.persistent, b->h2max[t], b->h1max[t], mode0(k),
                                    nd->argv) == hipSuccess;
                now.push_back(nd->node);
                bg.nodes.push_back(std::move(nd));
            }
            prev = now;
        }
        advance_position(b->scheme, c, hp);
    }
    if (ok && hipGraphInstantiate(&bg.exec, bg.tmpl, nullptr, nullptr, 0) != hipSuccess) bg.exec = nullptr;
    if (!bg.exec) {
        hipGraphDestroy(bg.tmpl);
        return nullptr;
    }
    b->graph_builds++;
    hipGraphExec_t ex = bg.exec;
    b->graphs.emplace(key, std::move(bg));
    return ex;
}

// After a membership change: re-point every instantiated graph's kernel nodes at
// the new descriptors and unit tables (grid and LDS size follow).  A graph built
// for another set of cell kinds, or whose update fails, is dropped and rebuilt
// when next needed.  The stream has been synchronized (batch_build).
void repoint_graphs(fvlbm_batch *b) {
    const int n = (int)b->members.size();
    const unsigned kinds = batch_kinds(b);
    for (auto it = b->graphs.begin(); it != b->graphs.end();) {
        BatchGraph &bg = it->second;
        bool ok = bg.kinds == kinds;
        for (size_t i = 0; ok && i < bg.nodes.size(); i++) {
            BatchGraph::Node &nd = *bg.nodes[i];
            ok = set_stage_node(bg.exec, nd.node, b->desc_dev + (size_t)nd.k * n, b->ut[nd.t], 3 + nd.t, b->storage,
                                b->sched.xcd_remap, b->sched.persistent, b->h2max[nd.t], b->h1max[nd.t], mode0(nd.k),
                                nd.argv) == hipSuccess;
        }
        if (ok) {
            b->graph_updates++;
            ++it;
        } else {
            hipGraphExecDestroy(bg.exec);
            hipGraphDestroy(bg.tmpl);
            it = b->graphs.erase(it);
        }
    }
}
}  // namespace

}  // extern "C"

namespace {
// Advance every member n_steps with shared launches: graphs of 32 steps, then
// of the largest power of two that fits (as a single solver).  dry: only
// instantiate those graphs (no launch, no snapshot, positions untouched).
fvlbm_status batch_enqueue(fvlbm_batch *b, int64_t n_steps, bool snapshots, bool dry = false) {
    int64_t left = n_steps;
    // as fvlbm_step(): a member on a lag boundary without a snapshot takes one first
    if (!dry && snapshots && n_steps > 0)
        for (fvlbm_solver *s : b->members)
            if (s->snap_cur < 0 && s->steps % s->lag == 0 && take_snapshot(s) != hipSuccess)
                return fail(FVLBM_E_DEVICE, "snapshot failed");
    int cur = b->members[0]->cur;
    bool hp = true;
    while (left > 0) {
        const int chunk = graph_steps(left, BATCH_GRAPH_CHUNK);
        hipGraphExec_t ex = batch_graph(b, cur, chunk);
        if (!ex) return fail(FVLBM_E_DEVICE, "batch graph build failed");
        for (int k = 0; k < chunk; k++) advance_position(b->scheme, cur, hp);
        left -= chunk;
        if (dry) continue;
        if (hipGraphLaunch(ex, b->stream) != hipSuccess) return fail(FVLBM_E_DEVICE, "batch graph launch failed");
        for (fvlbm_solver *s : b->members) {
            int64_t before = s->steps;
            for (int64_t k = 0; k < chunk; k++) advance_position(s->p.scheme, s->cur, s->have_prev);
            s->steps += chunk;
            // snapshot when a lag boundary is crossed exactly at the chunk end
            if (snapshots && s->steps / s->lag != before / s->lag && s->steps % s->lag == 0) {
                if (take_snapshot(s) != hipSuccess) return fail(FVLBM_E_DEVICE, "snapshot failed");
            }
        }
    }
    return FVLBM_OK;
}

// Device copy of what a step reads and writes (the current distributions and
// the AB2 history) plus the host-side position, for the autotuner.
struct Saved {
    fvlbm_solver *s = nullptr;
    char *dev = nullptr;
    size_t fb = 0, rb = 0, cb = 0;
    int cur = 0;
    int64_t steps = 0;
    bool have_prev = false;
};

fvlbm_status save_state(fvlbm_solver *s, Saved &sv) {
    const MeshDev &m = s->mesh->dev;
    sv.s = s;
    sv.fb = state_copy_bytes(s->p.storage, m.np);
    sv.rb = s->p.scheme == FVLBM_SCHEME_AB2 ? (size_t)Q * m.np * sizeof(float) : 0;
    sv.cb = carry_bytes(s->p.storage, m.np);
    if (hipMalloc(&sv.dev, sv.fb + sv.rb + sv.cb) != hipSuccess) return fail(FVLBM_E_NOMEM, "autotune state copy allocation failed");
    hipError_t e = hipMemcpyAsync(sv.dev, fptr(s, s->cur), sv.fb, hipMemcpyDeviceToDevice, s->stream);
    if (e == hipSuccess && sv.rb) e = hipMemcpyAsync(sv.dev + sv.fb, s->buf + s->L.r32, sv.rb, hipMemcpyDeviceToDevice, s->stream);
    if (e == hipSuccess && sv.cb) e = hipMemcpyAsync(sv.dev + sv.fb + sv.rb, carry_ptr(s), sv.cb, hipMemcpyDeviceToDevice, s->stream);
    if (e != hipSuccess) return fail(FVLBM_E_DEVICE, "autotune state copy failed");
    sv.cur = s->cur;
    sv.steps = s->steps;
    sv.have_prev = s->have_prev;
    return FVLBM_OK;
}

fvlbm_status restore_state(Saved &sv) {
    fvlbm_solver *s = sv.s;
    hipError_t e = hipMemcpyAsync(fptr(s, sv.cur), sv.dev, sv.fb, hipMemcpyDeviceToDevice, s->stream);
    if (e == hipSuccess && sv.rb) e = hipMemcpyAsync(s->buf + s->L.r32, sv.dev + sv.fb, sv.rb, hipMemcpyDeviceToDevice, s->stream);
    if (e == hipSuccess && sv.cb) e = hipMemcpyAsync(carry_ptr(s), sv.dev + sv.fb + sv.rb, sv.cb, hipMemcpyDeviceToDevice, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    hipFree(sv.dev);
    sv.dev = nullptr;
    s->cur = sv.cur;
    s->steps = sv.steps;
    s->have_prev = sv.have_prev;
    if (e != hipSuccess) return fail(FVLBM_E_DEVICE, "autotune state restore failed");
    return FVLBM_OK;
}

// Times `steps` steps of `run` on `stream` with HIP events, after `prep`
// (which instantiates the graphs of that call) and a warm-up of the same
// number of steps; returns ms per step or -1.
template <class Prep, class Run>
double time_steps(hipStream_t stream, int steps, Prep prep, Run run) {
    if (run(steps) != FVLBM_OK || prep(steps) != FVLBM_OK) return -1;
    hipEvent_t a, b;
    hipEventCreate(&a);
    hipEventCreate(&b);
    float best = -1;
    fvlbm_status st = FVLBM_OK;
    for (int rep = 0; rep < 2 && st == FVLBM_OK; rep++) {   // the faster of two runs
        hipEventRecord(a, stream);
        st = run(steps);
        hipEventRecord(b, stream);
        hipEventSynchronize(b);
        float ms = 0;
        hipEventElapsedTime(&ms, a, b);
        if (best < 0 || ms < best) best = ms;
    }
    hipEventDestroy(a);
    hipEventDestroy(b);
    return st == FVLBM_OK ? best / steps : -1;
}

// Tile sizes the autotuners try: the four powers of two, and the sizes that
// split n cells into about 256 k tiles (one, two ... workgroups per CU of a
// 256-CU GPU), rounded up to a multiple of 64.
std::vector<int> tune_blocks(int64_t n) {
    std::vector<int> out = {64, 128, 256, 512};
    int cus = 256, dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    for (int k = 1; k <= 4; k++) {
        const int64_t per = (n + (int64_t)cus * k - 1) / ((int64_t)cus * k);
        const int t = (int)((per + 63) / 64 * 64);
        if (t >= 64 && t <= 512 && std::find(out.begin(), out.end(), t) == out.end()) out.push_back(t);
    }
    return out;
}
}  // namespace

extern "C" {

namespace {
fvlbm_status batch_usable(const fvlbm_batch *b) {
    for (const fvlbm_solver *s : b->members) {
        if (s->destroyed) return fail(FVLBM_E_STATE, "a batch member was destroyed; destroy the batch");
        if (s->failed) return fail(FVLBM_E_STATE, "a batch member is in an error state");
    }
    return FVLBM_OK;
}
}  // namespace

fvlbm_status fvlbm_batch_step(fvlbm_batch *b, int64_t n_steps) {
    if (!b || n_steps < 0) return fail(FVLBM_E_ARG, "bad arguments to fvlbm_batch_step");
    fvlbm_status st = batch_usable(b);
    if (st != FVLBM_OK) return st;
    return batch_enqueue(b, n_steps, true);
}

fvlbm_status fvlbm_batch_residuals(fvlbm_batch *b, double *out) {
    if (!b || !out) return fail(FVLBM_E_ARG, "null argument");
    fvlbm_status st = batch_usable(b);
    if (st != FVLBM_OK) return st;
    const int n = (int)b->members.size();
    double *gathered = reinterpret_cast<double *>(b->res_src + n);
    std::vector<double> r(n);
    hipError_t e = launch_gather(b->res_src, gathered, n, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(r.data(), gathered, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return fail(FVLBM_E_DEVICE, std::string("batch residuals failed: ") + hipGetErrorString(e));
    for (int i = 0; i < n; i++) {
        out[2 * i] = b->members[i]->res_valid ? r[i] : -1.0;
        out[2 * i + 1] = (double)b->members[i]->steps;
    }
    return FVLBM_OK;
}

fvlbm_status fvlbm_autotune(fvlbm_solver *s, int32_t trial_steps, double *best_ms) {
    if (!s || trial_steps <= 0) return fail(FVLBM_E_ARG, "bad arguments to fvlbm_autotune");
    if (s->failed) return fail(FVLBM_E_STATE, "solver is in an error state");
    if (s->p.scheme == FVLBM_SCHEME_AB2 && !s->have_prev) return fail(FVLBM_E_STATE, "take the first AB2 step before tuning");
    Saved sv;
    fvlbm_status st = save_state(s, sv);
    if (st != FVLBM_OK) return st;
    Schedule best = s->sched;
    double best_t = 1e300;
    for (int T : tune_blocks(s->mesh->dev.n_cells))
        for (int x = 0; x < 2; x++)
            for (int ps = 0; ps < (T <= 128 ? 3 : 2); ps++) {
                if (fvlbm_set_schedule(s, T, x, ps) != FVLBM_OK) continue;
                double t = time_steps(
                    s->stream, trial_steps,
                    [&](int n) {
                        const int c = s->cur;
                        const bool hp = s->have_prev;
                        const int64_t st0 = s->steps;
                        fvlbm_status r = enqueue_steps(s, n, true);
                        s->cur = c; s->have_prev = hp; s->steps = st0;
                        return r;
                    },
                    [&](int n) { return enqueue_steps(s, n); });
                if (t > 0 && t < best_t) { best_t = t; best = s->sched; }
            }
    fvlbm_set_schedule(s, best.block, best.xcd_remap, best.persistent);
    st = restore_state(sv);
    if (best_ms) *best_ms = best_t;
    return st;
}

fvlbm_status fvlbm_batch_autotune(fvlbm_batch *b, int32_t trial_steps, double *best_ms) {
    if (!b || trial_steps <= 0) return fail(FVLBM_E_ARG, "bad arguments to fvlbm_batch_autotune");
    fvlbm_status ust = batch_usable(b);
    if (ust != FVLBM_OK) return ust;
    std::vector<Saved> saved(b->members.size());
    for (size_t i = 0; i < b->members.size(); i++) {
        fvlbm_status st = save_state(b->members[i], saved[i]);
        if (st != FVLBM_OK) return st;
    }
    Schedule best = b->sched;
    double best_t = 1e300;
    int64_t cells = 0;
    for (fvlbm_solver *m : b->members) cells += m->mesh->dev.n_cells;
    for (int T : tune_blocks(cells))
        for (int x = 0; x < 2; x++)
            for (int ps = 0; ps < 2; ps++) {
                if (fvlbm_batch_set_schedule(b, T, x, ps) != FVLBM_OK) continue;
                double t = time_steps(b->stream, trial_steps, [&](int n) { return batch_enqueue(b, n, false, true); },
                                      [&](int n) { return batch_enqueue(b, n, false); });
                if (t > 0 && t < best_t) { best_t = t; best = b->sched; }
            }
    fvlbm_batch_set_schedule(b, best.block, best.xcd_remap, best.persistent);
    fvlbm_status res = FVLBM_OK;
    for (auto &sv : saved) {
        fvlbm_status st = restore_state(sv);
        if (st != FVLBM_OK) res = st;
    }
    if (best_ms) *best_ms = best_t;
    return res;
}

void fvlbm_batch_destroy(fvlbm_batch *b) {
    if (!b) return;
    hipStreamSynchronize(b->stream);
    free_graphs(b->graphs);
    if (b->desc_dev) hipFree(b->desc_dev);
    if (b->res_src) hipFree(b->res_src);
    for (auto &u : b->ut) {
        if (u.units) hipFree(u.units);
        if (u.queue) hipFree(u.queue);
    }
    std::vector<fvlbm_solver *> members = std::move(b->members);
    delete b;
    // members destroyed while the batch held them are freed now
    for (fvlbm_solver *s : members)
        if (--s->batch_refs == 0 && s->destroyed) solver_free(s);
}

}  // extern "C"
