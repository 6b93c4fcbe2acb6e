// Internal declarations of the gfx950 FVLBM library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "fvlbm.h"

namespace fvlbm {

constexpr int Q = 9;
constexpr int MAX_GROUPS = 16;
constexpr int MAX_NF = 4;
// neighbour-slot codes: >= 0 neighbour cell, -1-g boundary group g, NB_PAD no face
constexpr int NB_PAD = -1000000;

// ---------------------------------------------------------------- host mesh

struct HostTopology {
    int n_cells = 0;
    int nf = 0;                        // face slots per cell (3 all-triangle, else 4)
    std::vector<int> perm;             // perm[new] = input index
    std::vector<int> iperm;            // iperm[input] = new index
    std::vector<int> ncorner;          // [n] corners of the cell (new order)
    std::vector<double> corner_xy;     // [n][nf][2] corner coordinates (new order)
    std::vector<int> nbr;              // [n][nf] slot code (new order)
    std::vector<int> back;             // [n][nf] slot of the same face in the neighbour (or -1)
    std::vector<double> shift;         // [n][nf][2] added to the neighbour centre (periodic image)
    int n_boundary_cells = 0;
    // the caller's boundary faces, in the caller's order: cell (new order), slot, group (-1 periodic)
    std::vector<int> bface_cell, bface_slot, bface_group;
};

// Builds topology from the raw mesh, validates it and reorders cells.
// Returns FVLBM_OK or FVLBM_E_ARG / FVLBM_E_MESH with a message in err.
fvlbm_status build_topology(int32_t n_nodes, const double *xy, int32_t n_cells,
                            const int32_t *cell_ptr, const int32_t *cell_nodes, int32_t n_bfaces,
                            const int32_t *bface_nodes, const int32_t *bface_group, int32_t n_groups,
                            const fvlbm_bc *groups, int32_t n_periodic,
                            const int32_t *periodic_pairs, const double *periodic_shift,
                            int32_t reorder, HostTopology &topo, std::string &err);

// ---------------------------------------------------------------- device mesh

struct GroupDev {
    int kind;
    int internal;
    float ux, uy;        // u_w or u_inf
    float drho;          // rho_inf - rho0 (deviation form)
    float rho;           // rho_inf
};

// Per tile size T: cells [t*T, t*T+T) form tile t; ring 1 is the set of face
// neighbours outside the tile, ring 2 the face neighbours of ring 1 outside
// tile and ring 1.  Every tile has h1max ring-1 slots and h2max ring-2 slots
// (the largest counts over tiles; unused slots hold -1), so a thread finds its
// halo cell at a fixed position without a per-tile header.  Local indices:
// tile cell i -> i - t*T, ring-1 slot k -> T + k, ring-2 slot k -> T + h1max + k.
struct TileTables {
    int T = 0;
    int n_tiles = 0;
    int h1max = 0;               // ring-1 slots per tile (largest n1)
    int h2max = 0;               // ring-2 slots per tile (largest n2)
    uint2 *lnbr = nullptr;       // [np] four int16 slot codes per tile cell: local index, -1-g, or LN_PAD
    int *halo_idx = nullptr;     // [n_tiles][h1max + h2max] cells of the ring-1 then ring-2 slots, -1 if unused
    uint2 *halo_code = nullptr;  // [n_tiles][h1max] four int16 slot codes per ring-1 slot (as lnbr)
    size_t bytes = 0;
    void *block = nullptr;
};
constexpr int LN_PAD = -32768;

struct MeshDev {
    int n_cells = 0;
    int np = 0;          // plane stride (cells padded to a multiple of 512)
    int nf = 0;
    int n_groups = 0;
    fvlbm_bc groups_host[MAX_GROUPS];
    // FP32 per-cell description, planes [slot][np] (see the geometry pass)
    float2 *vxy = nullptr;       // corner k - centroid
    float2 *dxy = nullptr;       // stencil offset of slot k
    std::vector<int> nbr_host;   // [n][nf] slot codes (new order), for the tile tables
    std::map<int, struct TileTables> tiles;   // by tile size
    // FP64 per cell
    double *area = nullptr;
    double cfl_length = 0;       // min A/(Lx+Ly)
    int n_boundary_cells = 0;
    std::vector<int> perm;       // perm[new] = input index
    int *perm_dev = nullptr;     // same, on the device
    // boundary faces grouped by boundary group (caller's order within a group): (cell, slot)
    int2 *gfaces_dev = nullptr;
    int gface_off[MAX_GROUPS + 1] = {0};
    size_t bytes = 0;
    void *block = nullptr;       // one allocation holding everything above
};

// FP64 geometry + FP32 coefficient pass on the device.
fvlbm_status build_device_mesh(const HostTopology &topo, const fvlbm_bc *groups, int n_groups,
                               hipStream_t stream, MeshDev &mesh, std::string &err);

// Reference state of the deviation storage: h = f - f_eq(rho0, u_dev).
struct RefDev {
    float rho0;          // rho0
    float jx0, jy0;      // rho0 u_dev
    float scale;         // S of FP16 deviation storage (stored value h/(w S))
    float fref[9];       // f_eq(rho0, u_dev) rounded to FP32 (the FP32-storage offset)
    float c0[9];         // (4.5 (e.j0)^2 - 1.5 |j0|^2) / rho0
    float inv_unit[9];   // 1 / (w S), FP16 storage unit
};

RefDev make_ref(double rho0, double ux, double uy, double scale);

// ---------------------------------------------------------------- stage launch

// Host form of the tile tables (see TileTables).
struct HostTiles {
    int T = 0, n_tiles = 0, h1max = 0, h2max = 0;
    std::vector<uint16_t> lnbr;        // [np][4]
    std::vector<int> halo_idx;         // [n_tiles][h1max + h2max]
    std::vector<uint16_t> halo_code;   // [n_tiles][h1max][4]
};
void build_tile_tables_host(const std::vector<int> &nbr, int n, int nf, int np, int T, HostTiles &out);

// Tile tables for tile size T (built on first use, kept with the mesh).
fvlbm_status get_tiles(MeshDev &mesh, int T, const TileTables **out, std::string &err);
void free_tiles(MeshDev &mesh);

// One instance's view for a stage launch (device memory, read through scalar loads).
struct InstDesc {
    const float2 *vxy, *dxy;
    const uint2 *lnbr;
    const int *halo_idx;
    const uint2 *halo_code;
    int h1s, h2s;         // ring-1 / ring-2 slots per tile of this instance's tables
    const void *src;      // state the RHS is evaluated at
    const void *base;     // f(0) of the update (== src for Euler / AB2)
    void *dst;
    float *rhs_prev;      // AB2 history (FP32 planes), or null
    __half *mcarry;       // FP16 storage, the last stage of a step: the rounding residual of each cell's
                          // mass and momentum (3 FP16 planes of 2^12 x the residual in units of S), added
                          // back to the update's base and rewritten by the store; null elsewhere
    int n_cells, np;
    float coef;           // dst = base + coef * RHS   (AB2: dt)
    float inv_tau;
    RefDev ref;
    int mode;             // 0 base+coef*RHS, 1 AB2 first step (Euler, store RHS), 2 AB2, 3 RHS only (FP32 out to dst)
    int n_groups;
    GroupDev groups[MAX_GROUPS];
};

struct Schedule {
    int block = 256;
    int xcd_remap = 1;
    int persistent = 0;
};

// Work units: (instance, tile index) per block; built for a schedule.
struct UnitTable {
    int2 *units = nullptr;   // device; null when direct
    unsigned *queue = nullptr;   // device, zeroed: the persistent form's work queue (ticket, workgroups done)
    int n_units = 0;
    int block = 0;
    bool direct = false;     // one instance: unit b is (0, b), the kernel needs no table
};

// Launch one RHS-evaluation stage over all units (one unit = one tile of
// ut.block cells).  nf: 3 or 4; storage FVLBM_STORE_*; h2max, h1max: the
// largest ring-2 and ring-1 slot counts over the launch's instances (LDS size).
// persistent: 0 one workgroup per tile, 1 a resident-sized grid taking the
// units from a work queue, 2 one workgroup per tile with one more wave for the halo slots (used by
// a single instance's mode-0 stages with tiles of 64 or 128 cells, else as 0).
// mode0: the stage is a base + coef RHS update (descriptor mode 0: Euler, RK
// stages), which runs a kernel compiled for it; other modes run one block per
// unit whatever `persistent` says.
// host_desc: the host copy of the launch's descriptor when it is a single instance
// (its first-load values then go as kernel arguments), or null.
hipError_t launch_stage(const InstDesc *descs_dev, const UnitTable &ut, int nf, int storage,
                        int xcd_remap, int persistent, int h2max, int h1max, bool mode0, hipStream_t stream,
                        const InstDesc *host_desc = nullptr);
size_t stage_lds_bytes(int T, int h2max, int h1max);
// Dynamic LDS a stage workgroup may use on the current device: the device's
// per-workgroup LDS (160 KiB on gfx950) less the kernels' static LDS (the group
// table, and the boundary stash, phase-3 geometry and collision terms of the
// 64-cell halo-wave form).
size_t stage_lds_limit();
// Same as a kernel node for a graph.
// argbuf: argbuf[0] holds a StageArgs, argbuf[1..15] receive the argument pointers.
// (Kernel argument order: the first fourteen dwords, hidx .. ux, are preloaded.)
struct StageArgs {
    const int *hidx;
    const void *src;
    const uint2 *lnbr;
    const float2 *dxy, *vxy;
    int h12, np, nc, ux;      // h1s + 2^16 h2s; 2 n_units + XCD remap
    const uint2 *hcode;
    const void *base;
    const InstDesc *d;
    int nA;
    const int2 *u;
    unsigned *queue;
    bool direct;
};
StageArgs stage_args(const InstDesc *descs_dev, const UnitTable &ut, int xcd_remap, int persistent, int h1max,
                     const InstDesc *host_desc);
hipError_t add_stage_node(hipGraph_t g, hipGraphNode_t *node, const hipGraphNode_t *deps, int ndeps,
                          const InstDesc *descs_dev, const UnitTable &ut, int nf, int storage,
                          int xcd_remap, int persistent, int h2max, int h1max, bool mode0, void **argbuf,
                          const InstDesc *host_desc = nullptr);
// Re-point a kernel node of an instantiated graph, added by add_stage_node() with the
// same nf, storage, tile size, XCD remap, persistent and mode0 (so the same kernel) and
// no host descriptor, at other descriptors and units (grid and LDS size follow).
hipError_t set_stage_node(hipGraphExec_t ex, hipGraphNode_t node, const InstDesc *descs_dev, const UnitTable &ut,
                          int nf, int storage, int xcd_remap, int persistent, int h2max, int h1max, bool mode0,
                          void **argbuf);

// Step 0 and conversions (FP64 host data in input order <-> device storage).
// carry: FP16 storage's moment carry (3 planes of np), written with the rounding residual of
// each cell's mass and momentum (null for the other storages).
hipError_t launch_init_eq(void *dst, int storage, int n, int np, const RefDev &ref,
                          const double *rho_dev, const double *u_dev, const int *perm_dev,
                          double rho_u, __half *carry, hipStream_t stream);
hipError_t launch_get_f(const void *src, int storage, int n, int np, const RefDev &ref,
                        const int *perm_dev, double *f_dev, hipStream_t stream);
hipError_t launch_set_f(void *dst, int storage, int n, int np, const RefDev &ref,
                        const int *perm_dev, const double *f_dev, __half *carry, hipStream_t stream);
hipError_t launch_rhs_out(const float *rhs32, int n, int np, const int *perm_dev, double *out_dev,
                          hipStream_t stream);

// Step 6 + FP64 reductions.  Writes rho/u (input order, FP64) and partial sums.
// carry: FP16 storage's moment carry (the state is the stored values less the carried
// residual of each cell's mass and momentum), or null.
hipError_t launch_macros(const void *src, int storage, int n, int np, const RefDev &ref, const __half *carry,
                         const double *area, const int *perm_dev, double *rho_out, double *u_out,
                         double *partial, int *flag, hipStream_t stream);
hipError_t launch_snapshot(const void *src, int storage, int n, int np, const RefDev &ref, const __half *carry,
                           double *snap_new, const double *snap_old, double *partial,
                           hipStream_t stream);
// partial: [nblk][2] -> out[0] = sum col0, out[1] = sum col1 (fixed order)
hipError_t launch_finish_sums(const double *partial, int nblk, double *out, int mode, hipStream_t stream);
// clear n ints with a kernel; out[0] = (flag[0] != 0) as a double
hipError_t launch_zero_int(int *p, int n, hipStream_t stream);
// dst[i] = *src[i] for n device pointers (src itself a device array)
hipError_t launch_gather(const double *const *src, double *dst, int n, hipStream_t stream);
hipError_t launch_flag_out(const int *flag, double *out, hipStream_t stream);
// Momentum flux through n wall faces (cell, slot) with wall velocity (uwx, uwy): partial sums of
// (Fx, Fy) per block, and p = rho/3 of each face's border cell.
hipError_t launch_wall_force(const void *src, int storage, int np, const RefDev &ref, const int2 *faces, int n,
                             const float2 *vxy, int nf, double uwx, double uwy, double *partial, double *face_p,
                             hipStream_t stream);
int reduce_blocks(int n);

}  // namespace fvlbm
