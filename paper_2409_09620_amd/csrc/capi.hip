// C ABI of the BP RI-OEDG stage library: context, device memory, stage
// sequencing and polling.  All per-cell arithmetic of a stage runs in the
// kernels of kernels.hip; this file only moves data and orders launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "capi_internal.h"

using oedg::Glob;

namespace capi {

dg_status fail(dg_ctx* c, dg_status s, const std::string& msg) {
    if (c && c->status == DG_OK) {
        c->status = s;
        c->err = msg;
    }
    return s;
}

}  // namespace capi

namespace {

using capi::fail;

// The kernels address a state buffer (4 variables x the modes of degree k x n_cell
// doubles) with 32-bit byte offsets, so it must stay below 4 GiB: at most
// 44,739,242 cells at P1 and 22,369,621 at P2.
bool too_many_cells(int32_t n_cell, int k) {
    return (uint64_t)n_cell * 4u * (uint64_t)((k + 1) * (k + 2) / 2) * sizeof(double) > 0xffffffffull;
}

#define HIP_TRY(ctx, call)                                                                       \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess) return fail(ctx, DG_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define LAUNCH_TRY(ctx, expr)                                                                    \
    do {                                                                                         \
        int e_ = (expr);                                                                         \
        if (e_ != 0) return fail(ctx, DG_E_HIP, std::string(#expr) + ": " + hipGetErrorString((hipError_t)e_)); \
    } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Mixed-precision state: FP64 averages [4][cell], then (at a 256-byte boundary)
// the float higher modes [4][mode-1][cell].
size_t mixed_hi_offset(size_t nc) { return align256(4 * nc * sizeof(double)); }
size_t mixed_state_bytes(size_t nc, size_t nm) { return mixed_hi_offset(nc) + 4 * (nm - 1) * nc * sizeof(float); }
size_t fp64_state_bytes(size_t nc, size_t nm) { return 4 * nm * nc * sizeof(double); }

struct Layout {
    size_t jinv, area, len, node, link, llink, hptr, hcell, u0, u, w, part, glob, total;
};

// One layout for both precisions: each state buffer holds either form.
Layout layout(size_t nc, int k) {
    const size_t nm = (size_t)(k + 1) * (k + 2) / 2;
    const size_t state = std::max(fp64_state_bytes(nc, nm), mixed_state_bytes(nc, nm));
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes); return o; };
    L.jinv = take(4 * nc * sizeof(double));
    L.area = take(nc * sizeof(double));
    L.len = take(3 * nc * sizeof(double));
    L.node = take(4 * nc * sizeof(double));
    L.link = take(3 * nc * sizeof(int32_t));
    L.llink = take(3 * nc * sizeof(int32_t));
    const size_t n_tiles = (nc + oedg::kTileCells - 1) / oedg::kTileCells;
    L.hptr = take((n_tiles + 1) * sizeof(int32_t));
    L.hcell = take(n_tiles * oedg::kHaloCap * sizeof(int32_t));
    L.u0 = take(state);
    L.u = take(state);
    L.w = take(std::max(state, 7 * nc * sizeof(double)));   // also carries the coordinates at set-up
    L.part = take((size_t)oedg::kPartCols * oedg::kMaxBlocks * sizeof(double));
    L.glob = take(sizeof(Glob));
    L.total = off;
    return L;
}

bool check_ctx(dg_ctx* c) { return c != nullptr; }

dg_status ready(dg_ctx* c, bool need_init) {
    if (!c) return DG_E_ARG;
    if (c->status != DG_OK) return c->status;
    if (c->host_only) return fail(c, DG_E_STATE, "host-only context");
    if (!c->have_mesh) return fail(c, DG_E_STATE, "no mesh uploaded");
    if (need_init && !c->initialised) return fail(c, DG_E_STATE, "state not initialised");
    HIP_TRY(c, hipSetDevice(c->device));
    return DG_OK;
}

bool is_mixed(const dg_ctx* c) { return c->cfg.precision == DG_PREC_MIXED; }

size_t state_bytes(const dg_ctx* c) {
    const size_t nc = (size_t)c->mesh.n_cell;
    return is_mixed(c) ? mixed_state_bytes(nc, (size_t)c->nm) : fp64_state_bytes(nc, (size_t)c->nm);
}

// the kernels' view of a state buffer in the configured precision
oedg::StateView view_of(const dg_ctx* c, const double* base) {
    double* b = const_cast<double*>(base);
    const size_t nc = (size_t)c->mesh.n_cell;
    if (is_mixed(c)) return {b, (char*)b + mixed_hi_offset(nc)};
    return {b, b + nc};
}

// host [4][nm][nc] FP64 <-> mixed storage (higher modes rounded to nearest float)
void pack_mixed(const double* u, size_t nc, size_t nm, std::vector<char>& out) {
    out.assign(mixed_state_bytes(nc, nm), 0);
    double* avg = (double*)out.data();
    float* hi = (float*)(out.data() + mixed_hi_offset(nc));
    for (size_t v = 0; v < 4; ++v) {
        for (size_t cc = 0; cc < nc; ++cc) avg[v * nc + cc] = u[v * nm * nc + cc];
        for (size_t l = 1; l < nm; ++l)
            for (size_t cc = 0; cc < nc; ++cc) hi[(v * (nm - 1) + l - 1) * nc + cc] = (float)u[(v * nm + l) * nc + cc];
    }
}
void unpack_mixed(const std::vector<char>& in, size_t nc, size_t nm, double* u) {
    const double* avg = (const double*)in.data();
    const float* hi = (const float*)(in.data() + mixed_hi_offset(nc));
    for (size_t v = 0; v < 4; ++v) {
        for (size_t cc = 0; cc < nc; ++cc) u[v * nm * nc + cc] = avg[v * nc + cc];
        for (size_t l = 1; l < nm; ++l)
            for (size_t cc = 0; cc < nc; ++cc) u[(v * nm + l) * nc + cc] = (double)hi[(v * (nm - 1) + l - 1) * nc + cc];
    }
}

// copies a device state buffer to host [4][nm][nc] FP64 (synchronises)
dg_status download_state(dg_ctx* c, const double* src, double* u_modal);

}  // namespace

oedg::StageArgs capi::stage_args(dg_ctx* c, int s) {
    oedg::StageArgs a{};
    a.m.n_cell = c->mesh.n_cell;
    a.m.jinv = c->jinv;
    a.m.area = c->area;
    a.m.len = c->len;
    a.m.node_ref = c->node;
    a.m.link = c->link;
    a.m.llink = c->llink;
    a.m.halo_ptr = c->halo_ptr;
    a.m.halo_cell = c->halo_cell;
    a.uin = view_of(c, s <= 0 ? c->u0 : c->u);
    a.u0 = view_of(c, c->u0);
    a.w = view_of(c, c->w);
    a.uout = view_of(c, s == 2 ? c->u0 : c->u);
    const size_t nc = (size_t)c->mesh.n_cell, nm = (size_t)c->nm;
    a.mixed = is_mixed(c) ? 1 : 0;
    a.avs = a.mixed ? nc : nm * nc;
    a.hvs = a.mixed ? (nm - 1) * nc : nm * nc;
    a.part = c->part;
    a.g = c->g;
    a.gamma = c->cfg.gamma;
    a.stage = s;
    a.oe_enable = c->cfg.oe_enable;
    a.oe_mode = c->cfg.oe_mode;
    a.bp_enable = c->cfg.bp_enable;
    a.k = c->cfg.k;
    a.zxs = c->cfg.decomposition == DG_DECOMP_ZXS;
    a.ustar = !a.zxs && c->cfg.limiter_form == DG_LIMITER_USTAR;
    return a;
}

namespace {

using capi::stage_args;

dg_status check_cfg(dg_ctx* c, const dg_config* cfg) {
    if (!cfg) return fail(c, DG_E_ARG, "null config");
    if (cfg->k != c->mesh.k) return fail(c, DG_E_ARG, "config degree differs from the mesh upload");
    if (cfg->precision != DG_PREC_FP64 && cfg->precision != DG_PREC_MIXED)
        return fail(c, DG_E_ARG, "unsupported precision");
    if (cfg->oe_mode != DG_OE_RI && cfg->oe_mode != DG_OE_CW) return fail(c, DG_E_ARG, "bad oe_mode");
    if (!(cfg->gamma > 1.0) || !(cfg->c_ssp > 0.0)) return fail(c, DG_E_ARG, "bad gamma or c_ssp");
    if (cfg->max_restarts < 0 || cfg->max_restarts > 60) return fail(c, DG_E_ARG, "bad max_restarts");
    if (cfg->decomposition != DG_DECOMP_DCW && cfg->decomposition != DG_DECOMP_ZXS)
        return fail(c, DG_E_ARG, "bad decomposition");
    if (cfg->limiter_form != DG_LIMITER_NODES && cfg->limiter_form != DG_LIMITER_USTAR)
        return fail(c, DG_E_ARG, "bad limiter_form");
    return DG_OK;
}

// fresh device scalars for t = 0; alpha and dt follow from the limiter pass
dg_status reset_glob(dg_ctx* c) {
    Glob h{};
    h.t_end = INFINITY;
    h.minck = c->cfg.decomposition == DG_DECOMP_ZXS ? c->mesh.minck_zxs : c->mesh.minck;
    h.area_sum = c->mesh.area_sum;
    h.c_ssp = c->cfg.c_ssp;
    h.alpha = h.alpha_step = 0.0;
    h.active = 1;
    h.max_restarts = c->cfg.max_restarts;
    HIP_TRY(c, hipMemcpyAsync(c->g, &h, sizeof(Glob), hipMemcpyHostToDevice, c->stream));
    return DG_OK;
}

// limiter (no OE) + alpha^0 + Delta t^0 on u^0, in place
dg_status start(dg_ctx* c) {
    oedg::StageArgs a = stage_args(c, -1);
    a.w = view_of(c, c->u0);
    a.uout = a.w;
    a.oe_enable = 0;
    LAUNCH_TRY(c, oedg::launch_filter(c->cfg.k, a, c->stream));
    LAUNCH_TRY(c, oedg::launch_finalize(oedg::kPassFilter, c->cfg.k, a, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->u, c->u0, state_bytes(c), hipMemcpyDeviceToDevice, c->stream));
    c->last_out = c->u0;
    c->initialised = true;
    c->generation++;
    Glob h{};
    HIP_TRY(c, hipMemcpyAsync(&h, c->g, sizeof(Glob), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (h.err) return fail(c, DG_E_BOUNDS, "initial data has an inadmissible cell average");
    return DG_OK;
}

dg_status read_glob(dg_ctx* c, Glob* h) {
    HIP_TRY(c, hipMemcpyAsync(h, c->g, sizeof(Glob), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return DG_OK;
}

// records the start event of a timed launch; returns the pair index or -1
dg_status prof_begin(dg_ctx* c, int kind, long* pair) {
    *pair = -1;
    if (!c->prof_on) return DG_OK;
    if (c->prof_used == c->prof_kind.size()) {
        hipEvent_t a, b;
        HIP_TRY(c, hipEventCreate(&a));
        HIP_TRY(c, hipEventCreate(&b));
        c->prof_ev.push_back(a);
        c->prof_ev.push_back(b);
        c->prof_kind.push_back(kind);
    }
    c->prof_kind[c->prof_used] = kind;
    HIP_TRY(c, hipEventRecord(c->prof_ev[2 * c->prof_used], c->stream));
    *pair = (long)c->prof_used++;
    return DG_OK;
}

dg_status prof_end(dg_ctx* c, long pair) {
    if (pair >= 0) HIP_TRY(c, hipEventRecord(c->prof_ev[2 * pair + 1], c->stream));
    return DG_OK;
}

#define TIMED_LAUNCH(ctx, kind, expr)                 \
    do {                                              \
        long pair_;                                   \
        dg_status ps_ = prof_begin(ctx, kind, &pair_); \
        if (ps_ != DG_OK) return ps_;                 \
        LAUNCH_TRY(ctx, expr);                        \
        if ((ps_ = prof_end(ctx, pair_)) != DG_OK) return ps_; \
    } while (0)

dg_status run_stage(dg_ctx* c, int s) {
    const oedg::StageArgs a = stage_args(c, s);
    TIMED_LAUNCH(c, oedg::kPassResidual, oedg::launch_residual(c->cfg.k, a, c->stream));
    LAUNCH_TRY(c, oedg::launch_finalize(oedg::kPassResidual, c->cfg.k, a, c->stream));
    TIMED_LAUNCH(c, oedg::kPassFilter, oedg::launch_filter(c->cfg.k, a, c->stream));
    LAUNCH_TRY(c, oedg::launch_finalize(oedg::kPassFilter, c->cfg.k, a, c->stream));
    c->last_out = s == 2 ? c->u0 : c->u;
    return DG_OK;
}

void drop_graph(dg_ctx* c) {
    if (c->step_exec) (void)hipGraphExecDestroy(c->step_exec);
    if (c->step_graph) (void)hipGraphDestroy(c->step_graph);
    c->step_exec = nullptr;
    c->step_graph = nullptr;
}

// Runs one step.  Without kernel timing the three stages are captured once into a
// HIP graph (on a library-owned stream, since the null stream cannot be captured)
// and replayed on the context's stream; every kernel reads its scalars (alpha,
// Delta t, t) from device memory, so a replay is the same as launching them anew.
dg_status run_step(dg_ctx* c) {
    dg_status st;
    if (c->prof_on || c->graph_failed) {
        for (int s = 0; s < 3; ++s)
            if ((st = run_stage(c, s)) != DG_OK) return st;
        return DG_OK;
    }
    if (!c->step_exec) {
        if (!c->cap_stream) HIP_TRY(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        hipStream_t user = c->stream;
        c->stream = c->cap_stream;
        hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
        st = DG_OK;
        if (e == hipSuccess) {
            for (int s = 0; s < 3 && st == DG_OK; ++s) st = run_stage(c, s);
            hipGraph_t g = nullptr;
            const hipError_t e2 = hipStreamEndCapture(c->cap_stream, &g);
            if (st == DG_OK && e2 == hipSuccess && g) {
                c->step_graph = g;
                if (hipGraphInstantiate(&c->step_exec, g, nullptr, nullptr, 0) != hipSuccess) {
                    drop_graph(c);
                    c->graph_failed = true;
                }
            } else {
                if (g) (void)hipGraphDestroy(g);
                c->graph_failed = true;
            }
        } else {
            c->graph_failed = true;
        }
        c->stream = user;
        if (st != DG_OK) return st;
        (void)hipGetLastError();
        if (c->graph_failed) return run_step(c);
    }
    HIP_TRY(c, hipGraphLaunch(c->step_exec, c->stream));
    c->last_out = c->u0;
    return DG_OK;
}

dg_status download_state(dg_ctx* c, const double* src, double* u_modal) {
    if (is_mixed(c)) {
        std::vector<char> packed(state_bytes(c));
        HIP_TRY(c, hipMemcpyAsync(packed.data(), src, packed.size(), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        unpack_mixed(packed, (size_t)c->mesh.n_cell, (size_t)c->nm, u_modal);
        return DG_OK;
    }
    HIP_TRY(c, hipMemcpyAsync(u_modal, src, state_bytes(c), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return DG_OK;
}

}  // namespace

extern "C" {

void dg_config_default(dg_config* cfg) {
    if (!cfg) return;
    cfg->k = 2;
    cfg->gamma = 1.4;
    cfg->c_ssp = 1.0;
    cfg->oe_enable = 1;
    cfg->oe_mode = DG_OE_RI;
    cfg->bp_enable = 1;
    cfg->precision = DG_PREC_FP64;
    cfg->max_restarts = 8;
    cfg->decomposition = DG_DECOMP_DCW;
    cfg->limiter_form = DG_LIMITER_NODES;
}

dg_status dg_create(dg_ctx** out, int hip_device, void* hip_stream) {
    if (!out) return DG_E_ARG;
    *out = nullptr;
    if (hip_device == DG_HOST_ONLY) {
        dg_ctx* c = new (std::nothrow) dg_ctx();
        if (!c) return DG_E_NOMEM;
        c->host_only = true;
        dg_config_default(&c->cfg);
        *out = c;
        return DG_OK;
    }
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || hip_device < 0 || hip_device >= n) return DG_E_HIP;
    if (hipSetDevice(hip_device) != hipSuccess) return DG_E_HIP;
    dg_ctx* c = new (std::nothrow) dg_ctx();
    if (!c) return DG_E_NOMEM;
    c->device = hip_device;
    c->stream = (hipStream_t)hip_stream;
    dg_config_default(&c->cfg);
    // the device's partial-record array of dg_stage_noalloc, looked up once per
    // device with the device current (a failure surfaces there, not here)
    (void)oedg::scratch_address(hip_device, &c->scratch);
    *out = c;
    return DG_OK;
}

dg_status dg_workspace_bytes(int32_t n_cell, int k, size_t* bytes) {
    if (!bytes || n_cell <= 0 || (k != 1 && k != 2) || too_many_cells(n_cell, k)) return DG_E_ARG;
    *bytes = layout((size_t)n_cell, k).total;
    return DG_OK;
}

dg_status dg_bind_workspace(dg_ctx* c, void* dev_ptr, size_t bytes) {
    if (!c) return DG_E_ARG;
    if (c->status != DG_OK) return c->status;
    if (!dev_ptr || bytes == 0) return fail(c, DG_E_ARG, "null workspace");
    if (((uintptr_t)dev_ptr & 255) != 0) return fail(c, DG_E_ARG, "workspace must be 256-byte aligned");
    c->bound = dev_ptr;
    c->bound_bytes = bytes;
    return DG_OK;
}

dg_status dg_mesh_upload(dg_ctx* c, int k, int32_t n_vert, const double* xy, int32_t n_cell, const int32_t* tri,
                         const double* cell_xy, const int32_t* edge_bc) {
    if (!c) return DG_E_ARG;
    if (c->status != DG_OK) return c->status;
    if (k != 1 && k != 2) return fail(c, DG_E_ARG, "degree must be 1 or 2");
    if (n_cell <= 0 || n_vert <= 0) return fail(c, DG_E_MESH, "mesh has no cells or no vertices");
    if (!tri || (!xy && !cell_xy)) return fail(c, DG_E_ARG, "null mesh array");
    if (too_many_cells(n_cell, k)) return fail(c, DG_E_ARG, "mesh too large: a state buffer must stay below 4 GiB");
    oedg::HostMesh m;
    std::string err;
    const int r = oedg::build_mesh(k, n_vert, xy, n_cell, tri, cell_xy, edge_bc, m, err);
    if (r != 0) return fail(c, r == -1 ? DG_E_ARG : DG_E_MESH, err);
    if (c->host_only) {
        c->mesh = std::move(m);
        c->nm = (k + 1) * (k + 2) / 2;
        c->cfg.k = k;
        c->have_mesh = true;
        return DG_OK;
    }
    HIP_TRY(c, hipSetDevice(c->device));

    const size_t nc = (size_t)n_cell;
    const Layout L = layout(nc, k);
    char* base = nullptr;
    if (c->bound) {
        if (c->bound_bytes < L.total) return fail(c, DG_E_NOMEM, "bound workspace too small");
        if (c->owned) {
            HIP_TRY(c, hipFree(c->owned));
            c->owned = nullptr;
        }
        base = (char*)c->bound;
    } else {
        if (c->owned && c->used_bytes < L.total) {
            HIP_TRY(c, hipFree(c->owned));
            c->owned = nullptr;
        }
        if (!c->owned) {
            void* p = nullptr;
            if (hipMalloc(&p, L.total) != hipSuccess) return fail(c, DG_E_NOMEM, "hipMalloc of the workspace failed");
            c->owned = p;
            c->used_bytes = L.total;
        }
        base = (char*)c->owned;
    }
    c->jinv = (double*)(base + L.jinv);
    c->area = (double*)(base + L.area);
    c->len = (double*)(base + L.len);
    c->node = (double*)(base + L.node);
    c->link = (int32_t*)(base + L.link);
    c->u0 = (double*)(base + L.u0);
    c->u = (double*)(base + L.u);
    c->w = (double*)(base + L.w);
    c->part = (double*)(base + L.part);
    c->llink = (int32_t*)(base + L.llink);
    c->halo_ptr = (int32_t*)(base + L.hptr);
    c->halo_cell = (int32_t*)(base + L.hcell);
    c->g = (Glob*)(base + L.glob);
    c->mesh = std::move(m);
    c->nm = (k + 1) * (k + 2) / 2;
    c->cfg.k = k;
    const oedg::HostMesh& hm = c->mesh;
    HIP_TRY(c, hipMemcpyAsync(c->jinv, hm.jinv.data(), 4 * nc * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->area, hm.area.data(), nc * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->len, hm.len.data(), 3 * nc * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->node, hm.node_ref.data(), 4 * nc * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->link, hm.link.data(), 3 * nc * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->llink, hm.llink.data(), 3 * nc * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->halo_ptr, hm.halo_ptr.data(), hm.halo_ptr.size() * sizeof(int32_t),
                              hipMemcpyHostToDevice, c->stream));
    if (!hm.halo_cell.empty())
        HIP_TRY(c, hipMemcpyAsync(c->halo_cell, hm.halo_cell.data(), hm.halo_cell.size() * sizeof(int32_t),
                                  hipMemcpyHostToDevice, c->stream));
    static const Glob zero{};
    HIP_TRY(c, hipMemcpyAsync(c->g, &zero, sizeof(Glob), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->have_mesh = true;
    c->initialised = false;
    c->generation++;
    drop_graph(c);
    return DG_OK;
}

dg_status dg_mesh_tables(dg_ctx* c, int32_t* tri, int32_t* nbr, int32_t* nbe, int32_t* perm, double* node_ref,
                         double* ck, double* minck) {
    if (!c) return DG_E_ARG;
    if (!c->have_mesh) return fail(c, DG_E_STATE, "no mesh uploaded");
    const oedg::HostMesh& m = c->mesh;
    const size_t nc = (size_t)m.n_cell;
    if (tri) std::memcpy(tri, m.tri.data(), 3 * nc * sizeof(int32_t));
    if (nbr) std::memcpy(nbr, m.nbr.data(), 3 * nc * sizeof(int32_t));
    if (nbe) std::memcpy(nbe, m.nbe.data(), 3 * nc * sizeof(int32_t));
    if (perm) std::memcpy(perm, m.perm.data(), 3 * nc * sizeof(int32_t));
    if (node_ref) std::memcpy(node_ref, m.node_ref.data(), 4 * nc * sizeof(double));
    if (ck) std::memcpy(ck, m.ck.data(), nc * sizeof(double));
    if (minck) *minck = m.minck;
    return DG_OK;
}

dg_status dg_init(dg_ctx* c, const dg_config* cfg, const double* u0_modal) {
    dg_status s = ready(c, false);
    if (s != DG_OK) return s;
    if ((s = check_cfg(c, cfg)) != DG_OK) return s;
    if (!u0_modal) return fail(c, DG_E_ARG, "null initial state");
    c->cfg = *cfg;
    drop_graph(c);
    std::vector<char> packed;   // must outlive the copy: start() synchronises
    if (is_mixed(c)) {
        pack_mixed(u0_modal, (size_t)c->mesh.n_cell, (size_t)c->nm, packed);
        HIP_TRY(c, hipMemcpyAsync(c->u0, packed.data(), packed.size(), hipMemcpyHostToDevice, c->stream));
    } else {
        HIP_TRY(c, hipMemcpyAsync(c->u0, u0_modal, state_bytes(c), hipMemcpyHostToDevice, c->stream));
    }
    if ((s = reset_glob(c)) != DG_OK) return s;
    return start(c);
}

dg_status dg_init_problem(dg_ctx* c, const dg_config* cfg, int kind, const double* params, int n_params) {
    dg_status s = ready(c, false);
    if (s != DG_OK) return s;
    if ((s = check_cfg(c, cfg)) != DG_OK) return s;
    static const int need[4] = {7, 18, 4, 12};
    if (kind < 0 || kind > 3 || !params || n_params < need[kind] || n_params > 19)
        return fail(c, DG_E_ARG, "bad problem kind or parameter count");
    c->cfg = *cfg;
    drop_graph(c);
    const oedg::HostMesh& m = c->mesh;
    const size_t nc = (size_t)m.n_cell;
    std::vector<double> P(params, params + n_params);
    // coordinates (and, for the blast, the flags of the cells owning the origin
    // vertex) travel in the pre-filter buffer, which is free until the first stage
    std::vector<double> aux(7 * nc, 0.0);
    std::memcpy(aux.data(), m.vx.data(), 6 * nc * sizeof(double));
    if (kind == 2) {
        const double ov = params[3];
        if (!(ov >= 0) || ov != std::floor(ov)) return fail(c, DG_E_ARG, "bad origin vertex id");
        double hit_area = 0.0;
        for (size_t cc = 0; cc < nc; ++cc) {
            bool hit = false;
            for (int q = 0; q < 3; ++q) hit |= (double)m.tri[3 * cc + q] == ov;
            if (hit) {
                aux[6 * nc + cc] = 1.0;
                hit_area += m.area[cc];
            }
        }
        if (!(hit_area > 0)) return fail(c, DG_E_ARG, "origin vertex is in no cell");
        P.resize(5);
        P[4] = hit_area;
    }
    HIP_TRY(c, hipMemcpyAsync(c->w, aux.data(), 7 * nc * sizeof(double), hipMemcpyHostToDevice, c->stream));
    if ((s = reset_glob(c)) != DG_OK) return s;
    oedg::StageArgs a = stage_args(c, -1);
    a.uout = view_of(c, c->u0);
    LAUNCH_TRY(c, oedg::launch_project(c->cfg.k, a, kind, P.data(), (int)P.size(), c->w, c->stream));
    // the host buffer must outlive the copy
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return start(c);
}

dg_status dg_stage(dg_ctx* c, int s) {
    dg_status st = ready(c, true);
    if (st != DG_OK) return st;
    if (s < 0 || s > 2) return fail(c, DG_E_ARG, "stage must be 0, 1 or 2");
    return run_stage(c, s);
}

dg_status dg_stage_noalloc(dg_ctx* c, int s) {
    dg_status st = ready(c, true);
    if (st != DG_OK) return st;
    if (s < 0 || s > 2) return fail(c, DG_E_ARG, "stage must be 0, 1 or 2");
    if (!c->scratch) {
        const int e = oedg::scratch_address(c->device, &c->scratch);
        if (e != 0 || !c->scratch)
            return fail(c, DG_E_HIP, std::string("hipGetSymbolAddress of the scratch records: ") +
                                         hipGetErrorString((hipError_t)e));
    }
    const int k = c->cfg.k, mixed = is_mixed(c) ? 1 : 0, nc = c->mesh.n_cell;
    for (int which = 0; which < oedg::kNumPasses; ++which) {
        const int grid = oedg::grid_for_pass(which, k, mixed, nc);
        if ((size_t)grid * oedg::kPartCols > oedg::kScratchDoubles)
            return fail(c, DG_E_ARG, "pass grid of " + std::to_string(grid) +
                                         " workgroups exceeds the scratch records (" +
                                         std::to_string(oedg::kMaxBlocks) + ")");
    }
    oedg::StageArgs a = stage_args(c, s);
    a.part = c->scratch;
    LAUNCH_TRY(c, oedg::launch_residual(k, a, c->stream));
    LAUNCH_TRY(c, oedg::launch_finalize(oedg::kPassResidual, k, a, c->stream));
    LAUNCH_TRY(c, oedg::launch_filter(k, a, c->stream));
    LAUNCH_TRY(c, oedg::launch_finalize(oedg::kPassFilter, k, a, c->stream));
    c->last_out = s == 2 ? c->u0 : c->u;
    return DG_OK;
}

dg_status dg_step(dg_ctx* c, double* dt_out) {
    dg_status st = ready(c, true);
    if (st != DG_OK) return st;
    if (dt_out) {
        Glob h{};
        if ((st = read_glob(c, &h)) != DG_OK) return st;
        *dt_out = h.active ? h.dt : 0.0;
    }
    return run_step(c);
}

dg_status dg_step_to(dg_ctx* c, double t_end, int64_t max_steps, int64_t* steps_done) {
    dg_status st = ready(c, true);
    if (st != DG_OK) return st;
    if (max_steps < 0 || std::isnan(t_end)) return fail(c, DG_E_ARG, "bad t_end or max_steps");
    Glob h{};
    if ((st = read_glob(c, &h)) != DG_OK) return st;
    const long long step0 = h.step;
    LAUNCH_TRY(c, oedg::launch_set_end(c->g, t_end, c->stream));
    // a launch either completes a step or retries it (at most max_restarts times
    // per step), so counting completed steps terminates.  Steps go out in chunks
    // between polls (doubling up to 64), each chunk capped by the steps that remain
    // at the current Delta t: a launch past t_end does nothing but still replays the
    // step graph, and Delta t changes from step to step, so an estimate that falls
    // short costs one more poll
    int64_t completed = 0;
    int chunk = 4;
    double t = h.t, dt = h.dt;
    while (completed < max_steps) {
        int64_t want = chunk;
        if (std::isfinite(t_end) && dt > 0.0) {
            const double est = std::ceil((t_end - t) / dt);
            want = std::min<int64_t>(want, est < 1.0 ? 1 : (est > 64.0 ? 64 : (int64_t)est));
        }
        const int64_t n = std::min<int64_t>(want, max_steps - completed);
        for (int64_t i = 0; i < n; ++i)
            if ((st = run_step(c)) != DG_OK) return st;
        if ((st = read_glob(c, &h)) != DG_OK) return st;
        completed = h.step - step0;
        t = h.t;
        dt = h.dt;
        if (!h.active || h.err) break;
        chunk = std::min(chunk * 2, 64);
    }
    if ((st = read_glob(c, &h)) != DG_OK) return st;
    if (steps_done) *steps_done = h.step - step0;
    if (h.err) return fail(c, DG_E_BOUNDS, "a cell average left the admissible set");
    return DG_OK;
}

dg_status dg_readback(dg_ctx* c, double* u_modal, double* t, int64_t* step) {
    dg_status st = ready(c, true);
    if (st != DG_OK && st != DG_E_BOUNDS) return st;
    HIP_TRY(c, hipSetDevice(c->device));
    if (u_modal && (st = download_state(c, c->u0, u_modal)) != DG_OK) return st;
    Glob h{};
    HIP_TRY(c, hipMemcpyAsync(&h, c->g, sizeof(Glob), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (t) *t = h.t;
    if (step) *step = h.step;
    return c->status;
}

dg_status dg_read_state(dg_ctx* c, int which, double* u_modal) {
    if (!c) return DG_E_ARG;
    if (c->host_only) return fail(c, DG_E_STATE, "host-only context");
    if (!c->have_mesh || !c->initialised) return fail(c, DG_E_STATE, "state not initialised");
    if (!u_modal || which < 0 || which > 2) return fail(c, DG_E_ARG, "bad buffer selector");
    HIP_TRY(c, hipSetDevice(c->device));
    const double* src = which == 0 ? c->u0 : (which == 1 ? c->last_out : c->w);
    return download_state(c, src, u_modal);
}

dg_status dg_diag(dg_ctx* c, dg_diag_t* out) {
    if (!c || !out) return DG_E_ARG;
    if (c->host_only) return fail(c, DG_E_STATE, "host-only context");
    if (!c->have_mesh) return fail(c, DG_E_STATE, "no mesh uploaded");
    HIP_TRY(c, hipSetDevice(c->device));
    Glob h{};
    dg_status st = read_glob(c, &h);
    if (st != DG_OK) return st;
    out->t = h.t;
    out->dt = h.dt;
    out->alpha = h.alpha_step;
    out->step = h.step;
    out->n_limited = h.n_limited;
    out->n_bad = h.n_bad;
    out->n_cfl_excursions = h.n_cfl_exc;
    out->n_flat = h.n_flat;
    out->n_restarts = h.n_restarts;
    out->alpha_stage = h.alpha;
    out->min_rho_node = h.min_rho_node;
    out->min_p_node = h.min_p_node;
    for (int v = 0; v < 4; ++v) {
        out->ubar[v] = h.ubar[v];
        out->nrm[v] = h.nrm[v];
    }
    out->nrm_m = h.nrm_m;
    out->active = h.active;
    return DG_OK;
}

dg_status dg_profile_enable(dg_ctx* c, int enable) {
    if (!c) return DG_E_ARG;
    if (c->host_only) return fail(c, DG_E_STATE, "host-only context");
    c->prof_on = enable != 0;
    return DG_OK;
}

dg_status dg_profile_read(dg_ctx* c, double* ms, int64_t* launches) {
    if (!c || !ms || !launches) return DG_E_ARG;
    if (c->host_only) return fail(c, DG_E_STATE, "host-only context");
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (int k = 0; k < DG_PROFILE_KERNELS; ++k) {
        ms[k] = 0.0;
        launches[k] = 0;
    }
    for (size_t i = 0; i < c->prof_used; ++i) {
        float t = 0.0f;
        HIP_TRY(c, hipEventElapsedTime(&t, c->prof_ev[2 * i], c->prof_ev[2 * i + 1]));
        ms[c->prof_kind[i]] += t;
        launches[c->prof_kind[i]] += 1;
    }
    c->prof_used = 0;
    return DG_OK;
}

dg_status dg_sizes(dg_ctx* c, int32_t* n_cell, int* k, int* n_modes) {
    if (!c) return DG_E_ARG;
    if (!c->have_mesh) return fail(c, DG_E_STATE, "no mesh uploaded");
    if (n_cell) *n_cell = c->mesh.n_cell;
    if (k) *k = c->mesh.k;
    if (n_modes) *n_modes = c->nm;
    return DG_OK;
}

const char* dg_last_error(const dg_ctx* c) {
    if (!c) return "null context";
    return c->err.c_str();
}

void dg_destroy(dg_ctx* c) {
    if (!c) return;
    if (!c->host_only) {
        (void)hipSetDevice(c->device);
        (void)hipStreamSynchronize(c->stream);
        for (hipEvent_t e : c->prof_ev) (void)hipEventDestroy(e);
        drop_graph(c);
        if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    }
    if (c->owned && !c->host_only) {
        (void)hipSetDevice(c->device);
        (void)hipStreamSynchronize(c->stream);
        (void)hipFree(c->owned);
    }
    delete c;
}

}  // extern "C"
