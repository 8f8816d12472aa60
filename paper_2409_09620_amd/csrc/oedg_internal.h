// Internal declarations shared by the host code and the kernels of the library.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace oedg {

constexpr int kBlock = 256;            // threads per workgroup of the stage kernels
constexpr int kCellsPerTile = 64;      // a quad of 4 lanes per cell in the residual/filter passes
constexpr int kCellsPerTileScalar = 256;   // one lane per cell in the momentum-norm pass
constexpr int kMaxBlocks = 4096;       // upper bound of a pass's grid (= number of partials)
constexpr int kNumPartial = 12;        // per-block partials of the residual pass
constexpr int kPartCols = kNumPartial + 1 + 4;   // + momentum norm + 4 filter partials

// Host-side mesh tables built once per mesh (see mesh_host.cpp).  Per-cell arrays
// that go to the device are structure-of-arrays: component-major, cell fastest.
struct HostMesh {
    int32_t n_cell = 0;
    int k = 0;
    std::vector<int32_t> tri, nbr, nbe, perm;   // [cell][3]
    std::vector<int32_t> link;                  // [3][cell]: (nbr << 2) | nbe, or -1
    std::vector<double> jinv;                   // [4][cell]: xi_x, xi_y, eta_x, eta_y
    std::vector<double> area;                   // [cell]
    std::vector<double> len;                    // [3][cell]
    std::vector<double> node_ref;               // [4][cell]: xi_1, eta_1, xi_2, eta_2
    std::vector<double> ck;                     // [cell] C^DCW_{K,k} |K|
    std::vector<double> vx;                     // [6][cell] oriented vertex coordinates
    double minck = 0.0;
    double area_sum = 0.0;
};

int build_mesh(int k, int32_t n_vert, const double* xy, int32_t n_cell, const int32_t* tri,
               const double* cell_xy, const int32_t* edge_bc, HostMesh& m, std::string& err);

// Device-resident scalars of one context.  Written only by the last workgroup of a
// kernel (after all others have published their partials) or by the host between
// steps.
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
    double* part;         // per-block partials: [12][kMaxBlocks] residual, [kMaxBlocks] momentum
                          // norm, [4][kMaxBlocks] filter
    Glob* g;
    double gamma;
    int stage;            // 0, 1, 2; -1 = limiter and alpha only (initial data)
    int oe_enable, oe_mode, bp_enable;
    int mixed;            // 0: FP64 bulk, 1: FP32 bulk (averages and limiter stay FP64)
};

// Grid of pass `which` (0 residual, 1 momentum norm, 2 filter) at degree k and
// precision `mixed`: a multiple of 8 (one share per XCD), at most kMaxBlocks and
// at most what is resident at once; workgroups stride over their XCD's tiles.
int grid_for_pass(int which, int k, int mixed, int n_cell);

// kernel launchers (kernels.hip); the precision comes from a.mixed.  Return a
// hipError_t as int.  Each pass kernel writes per-workgroup partials; the
// matching finalize kernel (one workgroup) reduces them in a fixed order into Glob.
int launch_residual(int k, const StageArgs& a, void* stream);
int launch_mnorm(int k, const StageArgs& a, void* stream);
int launch_filter(int k, const StageArgs& a, void* stream);
int launch_finalize(int which, int k, const StageArgs& a, void* stream);   // 0 residual, 1 mnorm, 2 filter
// L2 projection of a named problem into a.uout; vx holds the oriented vertex
// coordinates [6][cell] (and, for the blast, the origin flags in row 6)
int launch_project(int k, const StageArgs& a, int kind, const double* dparams, int n_params, const double* vx,
                   void* stream);
int launch_set_end(Glob* g, double t_end, void* stream);

}  // namespace oedg
