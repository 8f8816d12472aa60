// Internal declarations shared by the host code and the kernels of the library.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace oedg {

constexpr int kBlock = 256;            // threads per workgroup of the set-up kernels
// The residual and filter passes take the cells in tiles of kTileCells consecutive
// cells, one lane per cell; a pass workgroup stages a tile and its halo (at most
// kHaloCap out-of-tile neighbours) in LDS before it computes the tile.
constexpr int kTileCells = 256;
constexpr int kPassThreads = kTileCells;
constexpr int kHaloCap = 80;
constexpr int n_tiles_of(int n_cell) { return (n_cell + kTileCells - 1) / kTileCells; }
constexpr int kMaxBlocks = 4096;       // upper bound of a single-instance pass grid (= partials)
constexpr int kGroupCells = 256;       // cells per reduction group of the batched passes
constexpr int kNumPartial = 12;        // partials of the residual pass per group
constexpr int kFilterCols = 12;        // partials of the filter pass per group
constexpr int kPartCols = kNumPartial + 1 + kFilterCols + 1;   // + momentum norm, filter, bad averages
constexpr int kColBad = kPartCols - 1;   // residual pass: cells whose average left the admissible set

// Reduction groups of an instance in the batched passes: cells [g * kGroupCells,
// (g + 1) * kGroupCells).  Every group writes its own partial record, so an
// instance's reductions depend only on its own cells, whatever the schedule or
// the other instances of the launch.
constexpr int n_groups(int n_cell) { return (n_cell + kGroupCells - 1) / kGroupCells; }
// a batched pass walks a member's groups as its tiles (halo map, tile-image slots and
// edge ownership of the mesh precompute are per tile)
static_assert(kGroupCells == kTileCells, "groups are the tiles");

// Host-side mesh tables built once per mesh (see mesh_host.cpp).  Per-cell arrays
// that go to the device are structure-of-arrays: component-major, cell fastest.
struct HostMesh {
    int32_t n_cell = 0;
    int k = 0;
    std::vector<int32_t> tri, nbr, nbe, perm;   // [cell][3]
    std::vector<int32_t> link;                  // [3][cell]: (nbr << 2) | nbe, or kLinkOpen / kLinkWall
    // the tiles' halo map for the stage kernels (see kLinkGlobal)
    std::vector<int32_t> llink;                 // [3][cell]
    std::vector<int32_t> halo_ptr;              // [n_tiles + 1]: tile t's halo is halo_cell[halo_ptr[t]..)
    std::vector<int32_t> halo_cell;             // the halo cells of every tile, at most kHaloCap per tile
    std::vector<double> jinv;                   // [4][cell]: xi_x, xi_y, eta_x, eta_y
    std::vector<double> area;                   // [cell]
    std::vector<double> len;                    // [3][cell]
    std::vector<double> node_ref;               // [4][cell]: xi_1, eta_1, xi_2, eta_2
    std::vector<double> ck;                     // [cell] C^DCW_{K,k} |K|
    std::vector<double> ck_zxs;                 // [cell] C^ZXS_{K,k} |K|
    std::vector<double> vx;                     // [6][cell] oriented vertex coordinates
    double minck = 0.0;       // min_K C^DCW_{K,k} |K|
    double minck_zxs = 0.0;   // min_K C^ZXS_{K,k} |K|
    double area_sum = 0.0;
};

// link of a boundary edge: transmissive or reflective (interior links are >= 0)
constexpr int32_t kLinkOpen = -1;
constexpr int32_t kLinkWall = -2;
// llink of an interior edge: (slot << 3) | (low << 2) | nbe, slot the neighbour's LDS
// slot in the tile image (its offset in the tile, or kTileCells + its halo index),
// low = 1 when this cell's index is below the neighbour's; an edge inside the tile
// also carries kLinkRecv on the side that does not own it (the filter's edge work is
// done once, by the owner).  A neighbour beyond the halo cap is read from global
// memory: kLinkGlobal | (nbr << 3) | (low << 2) | nbe.  Boundary edges carry
// kLinkOpen / kLinkWall.
constexpr int32_t kLinkGlobal = 1 << 30;
constexpr int32_t kLinkRecv = 1 << 12;
constexpr int32_t kLinkSlotMask = 0x1FF;   // (llink >> 3) & mask: the slot of a link without kLinkGlobal
static_assert(kTileCells + kHaloCap <= kLinkSlotMask + 1, "slots fit below kLinkRecv");

int build_mesh(int k, int32_t n_vert, const double* xy, int32_t n_cell, const int32_t* tri,
               const double* cell_xy, const int32_t* edge_bc, HostMesh& m, std::string& err);

// Device-resident scalars of one instance.  Written only by the finalize kernels
// (one workgroup per instance, after the pass has published its partials) or by
// the host between steps.
struct Glob {
    double alpha;        // LF viscosity of the current stage input (eq. 1250)
    double alpha_step;   // alpha of u^n, which sets the step's Delta t
    double dt;           // Delta t of the current step
    double t;            // time of u^n
    double t_end;        // stop time (infinity when unset)
    double minck;        // min_K C^DCW_{K,k} |K|
    double area_sum;     // |Omega|
    double c_ssp;
    double ubar[4];      // domain averages of the pre-filter state
    double nrm[4];       // ||u - ubar||_inf per variable
    double nrm_m;        // ||| m - mbar |||_inf
    double inv_nrm[4];   // 1/nrm or 0 where the zero branch of eq. OEScalar:Coef2 applies
    double inv_nrm_m;
    long long step;
    long long n_limited;
    long long n_bad;
    long long n_cfl_exc;
    long long n_flat;    // mixed precision: cells reset to their average by the rounding check
    long long n_restarts;   // steps retried with half the time step
    double min_rho_node;    // min over the limiter nodes of the last stage output: density
    double min_p_node;      // and pressure
    // Momentum bookkeeping that gives the residual pass the domain average of the
    // state it is about to write (see the residual kernel): sum_K |K| mbar_K of a
    // limited state, and the momentum flux through the boundary edges that the
    // residual of that state will see, as A + alpha B (B: the reflective edges'
    // viscosity term).  _c: the last filter output; _n: u^n.
    double mom_c[2], bfa_c[2], bfb_c[2];
    double mom_n[2], bfa_n[2], bfb_n[2];
    int skip;            // a stage of this step left the admissible set: the rest of the step is skipped
    int restarts;        // retries of the current step so far
    int max_restarts;
    int active;          // 0: t reached t_end, or an error stopped the run
    int err;             // sticky: 1 once a cell average left the admissible set
};

struct DevMesh {
    int32_t n_cell;
    const double* jinv;
    const double* area;
    const double* len;
    const double* node_ref;
    const int32_t* link;
    const int32_t* llink;
    const int32_t* halo_ptr;
    const int32_t* halo_cell;
};

// One state buffer.  Cell averages (mode 0) are FP64 in every precision; modes
// l >= 1 are stored in the bulk type (double for DG_PREC_FP64, float for
// DG_PREC_MIXED).  Entry (var v, mode l, cell c) is avg[v * avs + c] for l = 0
// and hi[v * hvs + (l - 1) * n_cell + c] for l >= 1, with the strides of
// StageArgs.  The FP64 view of a [var][mode][cell] array is avg = base,
// hi = base + n_cell, avs = hvs = n_modes * n_cell.
struct StateView {
    double* avg;
    void* hi;
};

struct StageArgs {
    DevMesh m;
    StateView uin;        // stage input (own + neighbours)
    StateView u0;         // u^n for the SSP combination
    StateView w;          // pre-filter state (written by the residual pass)
    StateView uout;       // limited stage output
    size_t avs, hvs;      // variable strides of the averages and of the higher modes
    double* part;         // partial records, column-major; columns 0-12 residual (12:
                          // momentum norm), 13-22 filter.  Single-instance passes:
                          // column j of workgroup b at part[j * kMaxBlocks + b].
                          // Batched passes: column j of group g of this instance at
                          // part[j * gstride + gbase + g].
    size_t gstride;       // batched: groups of all instances sharing `part`
    int gbase;            // batched: first group of this instance in `part`
    Glob* g;
    double gamma;
    int k;                // degree
    int stage;            // 0, 1, 2; -1 = limiter and alpha only (initial data)
    int oe_enable, oe_mode, bp_enable;
    int mixed;            // 0: FP64 bulk, 1: FP32 bulk (averages and limiter stay FP64)
    int zxs;              // 1: classical decomposition's limiter node set (else the optimal one)
    int ustar;            // 1: optimal decomposition, P2 limiter in the u* form (the nodes' mean)
};

// A run of groups [g0, g1) of instance `inst`: the unit a pass workgroup takes.
struct Chunk {
    int inst, g0, g1;
};
// Chunk ranges per XCD: XCD x takes chunks [b[x], b[x+1]).
struct ChunkSplit {
    int b[9];
};

// the passes of a stage
constexpr int kPassResidual = 0, kPassFilter = 1, kNumPasses = 2;

// ---- single instance: persistent passes over the instance's tiles
// Grid of pass `which` (kPassResidual, kPassFilter) at degree k and
// precision `mixed`: a multiple of 8 (one share per XCD), at most kMaxBlocks and
// at most what is resident at once; workgroups stride over their XCD's tiles.
int grid_for_pass(int which, int k, int mixed, int n_cell);
// Kernel launchers; the precision comes from a.mixed.  Return a hipError_t as
// int.  Each pass kernel writes per-workgroup partials; the matching finalize
// kernel (one workgroup) reduces them in a fixed order into Glob.
int launch_residual(int k, const StageArgs& a, void* stream);
int launch_filter(int k, const StageArgs& a, void* stream);
int launch_finalize(int which, int k, const StageArgs& a, void* stream);   // which: kPassResidual, kPassFilter

// ---- no-allocation stage (dg_stage_noalloc): partial records in a device array of
// the library, kScratchDoubles doubles per GPU (the records of kMaxBlocks workgroups)
constexpr size_t kScratchDoubles = (size_t)kPartCols * kMaxBlocks;
// Address of that array on `device`, which must be the current device.  Looked up
// once per device (later calls return the cached address).  Returns a hipError_t
// as int; *out is null on failure.
int scratch_address(int device, double** out);

// ---- batch: passes over a chunk table of several instances (a batch that holds
// both degrees launches each pass once per degree)
// Workgroups of batched pass `which` resident at once for degree kmask (1: P1,
// 2: P2) and precision `mixed`; a multiple of 8.
int resident_grid_batch(int which, int kmask, int mixed);
// Launches batched pass `which`: desc[i] are the device stage arguments of
// instance i, chunks the device chunk table split by XCD as in cs; grid a
// multiple of 8.  Returns a hipError_t as int.
int launch_pass_batch(int which, int kmask, int mixed, const StageArgs* desc, const Chunk* chunks,
                      const ChunkSplit& cs, int grid, void* stream);
// The matching finalize kernel, one workgroup per instance (desc[0..n_inst)):
// reduces the instance's group records in a fixed order into its Glob.
int launch_finalize_batch(int which, const StageArgs* desc, int n_inst, void* stream);
int launch_project(int k, const StageArgs& a, int kind, const double* dparams, int n_params, const double* vx,
                   void* stream);
int launch_set_end(Glob* g, double t_end, void* stream);
// Copies the status of every instance of desc[0..n) into out[kStatusCols n]; per
// member: active, err, t, step, Delta t, t_end
constexpr int kStatusCols = 6;
int launch_gather_status(const StageArgs* desc, int n, double* out, void* stream);

// schedule.cpp: chunks of chunk_groups groups over the instances in order (only
// those of degree only_k unless it is 0), and their split into 8 contiguous
// ranges of equal estimated cost (one per XCD).  Returns 0, or -1 for invalid
// sizes or degrees.
int plan_chunks(int n_inst, const int32_t* n_cell, const int* k, int chunk_groups, std::vector<Chunk>& chunks,
                ChunkSplit& split, int only_k = 0);
// Grid of a pass over a split: 8 times the widest XCD range, at most `resident`.
int grid_for_split(const ChunkSplit& split, int resident);

}  // namespace oedg
