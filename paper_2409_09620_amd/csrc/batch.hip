// C ABI of batched stepping: several initialised contexts (instances with their
// own meshes, degrees and states on one device) advanced together, each pass of
// a stage one launch over all of them.  A chunk table cuts every instance into
// runs of 256-cell reduction groups; every group writes its own partial record
// and a per-instance finalize reduces them in a fixed order, so an instance's
// result does not depend on the schedule or on the other members of the batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "capi_internal.h"

struct dg_batch {
    int device = 0;
    hipStream_t stream = nullptr;
    dg_status status = DG_OK;
    std::string err;

    std::vector<dg_ctx*> ctx;
    std::vector<unsigned long long> generation;   // of each member when the batch was built
    int n = 0, mixed = 0, kmask = 0;
    long long total_groups = 0;

    // schedule: one launch per pass, or (both degrees present) one per degree,
    // each over its own part of the chunk table
    int chunk_groups = 1;
    int occupancy_pct = 100;
    std::vector<oedg::Chunk> chunks;
    int n_launch = 1;
    int launch_k[2] = {0, 0};     // degree mask of each launch
    int chunk_off[2] = {0, 0};    // its first chunk
    oedg::ChunkSplit split[2]{};
    int grid[2][oedg::kNumPasses] = {{8, 8}, {8, 8}};
    hipStream_t side = nullptr;   // the second degree's launches, beside the first
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;

    // device memory (one library allocation): stage arguments [3][n], chunk
    // table (one chunk per group at most), partial records, status words
    void* mem = nullptr;
    oedg::StageArgs* d_desc = nullptr;
    oedg::Chunk* d_chunks = nullptr;
    double* d_part = nullptr;
    double* d_status = nullptr;
    std::vector<oedg::StageArgs> h_desc;   // host copy, kept alive for the async upload
    std::vector<double> h_status;

    // one captured step
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool graph_failed = false;
};

namespace {

dg_status bfail(dg_batch* b, dg_status s, const std::string& msg) {
    if (b && b->status == DG_OK) {
        b->status = s;
        b->err = msg;
    }
    return s;
}

#define BHIP_TRY(b, call)                                                                        \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess) return bfail(b, DG_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define BLAUNCH_TRY(b, expr)                                                                     \
    do {                                                                                         \
        int e_ = (expr);                                                                         \
        if (e_ != 0) return bfail(b, DG_E_HIP, std::string(#expr) + ": " + hipGetErrorString((hipError_t)e_)); \
    } while (0)

void drop_graph(dg_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

dg_status ready(dg_batch* b) {
    if (!b) return DG_E_ARG;
    if (b->status != DG_OK) return b->status;
    for (int i = 0; i < b->n; ++i)
        if (b->ctx[i]->generation != b->generation[i] || b->ctx[i]->status != DG_OK)
            return bfail(b, DG_E_STATE, "a member context was re-initialised or failed after the batch was built");
    BHIP_TRY(b, hipSetDevice(b->device));
    return DG_OK;
}

// chunk table, XCD split and grids for the current schedule; uploads the table
dg_status plan(dg_batch* b) {
    std::vector<int32_t> nc(b->n);
    std::vector<int> k(b->n);
    for (int i = 0; i < b->n; ++i) {
        nc[i] = b->ctx[i]->mesh.n_cell;
        k[i] = b->ctx[i]->cfg.k;
    }
    // A batch of both degrees launches the single-degree kernels, one per degree:
    // the kernel that takes both holds the larger register and LDS footprint for
    // every chunk (in the mixed form 255 VGPRs against 119 and 167).
    b->n_launch = b->kmask == 3 ? 2 : 1;
    b->launch_k[0] = b->kmask == 3 ? 1 : b->kmask;
    b->launch_k[1] = 2;
    b->chunks.clear();
    std::vector<oedg::Chunk> part;
    for (int l = 0; l < b->n_launch; ++l) {
        if (oedg::plan_chunks(b->n, nc.data(), k.data(), b->chunk_groups, part, b->split[l],
                              b->n_launch == 2 ? b->launch_k[l] : 0) != 0)
            return bfail(b, DG_E_ARG, "bad schedule");
        b->chunk_off[l] = (int)b->chunks.size();
        b->chunks.insert(b->chunks.end(), part.begin(), part.end());
        for (int w = 0; w < oedg::kNumPasses; ++w) {
            const int resident = oedg::resident_grid_batch(w, b->launch_k[l], b->mixed);
            const int cap = std::max(8, (int)((long long)resident * b->occupancy_pct / 100) / 8 * 8);
            b->grid[l][w] = oedg::grid_for_split(b->split[l], cap);
        }
    }
    BHIP_TRY(b, hipMemcpyAsync(b->d_chunks, b->chunks.data(), b->chunks.size() * sizeof(oedg::Chunk),
                               hipMemcpyHostToDevice, b->stream));
    BHIP_TRY(b, hipStreamSynchronize(b->stream));
    drop_graph(b);
    return DG_OK;
}

dg_status run_stage(dg_batch* b, int s) {
    const oedg::StageArgs* d = b->d_desc + (size_t)s * b->n;
    for (int w = 0; w < oedg::kNumPasses; ++w) {
        if (b->n_launch == 1) {
            BLAUNCH_TRY(b, oedg::launch_pass_batch(w, b->launch_k[0], b->mixed, d, b->d_chunks, b->split[0],
                                                   b->grid[0][w], b->stream));
        } else {
            // the P2 launch on a second stream beside the P1 one (forked from and joined
            // back into the batch's stream: graph capture records two parallel nodes)
            BHIP_TRY(b, hipEventRecord(b->ev_fork, b->stream));
            BHIP_TRY(b, hipStreamWaitEvent(b->side, b->ev_fork, 0));
            BLAUNCH_TRY(b, oedg::launch_pass_batch(w, b->launch_k[0], b->mixed, d, b->d_chunks + b->chunk_off[0],
                                                   b->split[0], b->grid[0][w], b->stream));
            BLAUNCH_TRY(b, oedg::launch_pass_batch(w, b->launch_k[1], b->mixed, d, b->d_chunks + b->chunk_off[1],
                                                   b->split[1], b->grid[1][w], b->side));
            BHIP_TRY(b, hipEventRecord(b->ev_join, b->side));
            BHIP_TRY(b, hipStreamWaitEvent(b->stream, b->ev_join, 0));
        }
        BLAUNCH_TRY(b, oedg::launch_finalize_batch(w, d, b->n, b->stream));
    }
    return DG_OK;
}

// One step of every member.  Replayed from a graph captured on a library stream;
// every kernel reads its scalars from device memory, so a replay equals a fresh
// launch sequence.
dg_status run_step(dg_batch* b) {
    dg_status st;
    if (b->graph_failed) {
        for (int s = 0; s < 3; ++s)
            if ((st = run_stage(b, s)) != DG_OK) return st;
        return DG_OK;
    }
    if (!b->exec) {
        if (!b->cap_stream) BHIP_TRY(b, hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
        hipStream_t user = b->stream;
        b->stream = b->cap_stream;
        st = DG_OK;
        if (hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal) == hipSuccess) {
            for (int s = 0; s < 3 && st == DG_OK; ++s) st = run_stage(b, s);
            hipGraph_t g = nullptr;
            const hipError_t e2 = hipStreamEndCapture(b->cap_stream, &g);
            if (st == DG_OK && e2 == hipSuccess && g) {
                b->graph = g;
                if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
                    drop_graph(b);
                    b->graph_failed = true;
                }
            } else {
                if (g) (void)hipGraphDestroy(g);
                b->graph_failed = true;
            }
        } else {
            b->graph_failed = true;
        }
        b->stream = user;
        if (st != DG_OK) return st;
        (void)hipGetLastError();
        if (b->graph_failed) return run_step(b);
    }
    BHIP_TRY(b, hipGraphLaunch(b->exec, b->stream));
    return DG_OK;
}

dg_status poll(dg_batch* b, int* n_active, int* n_err) {
    BLAUNCH_TRY(b, oedg::launch_gather_status(b->d_desc, b->n, b->d_status, b->stream));
    BHIP_TRY(b, hipMemcpyAsync(b->h_status.data(), b->d_status, oedg::kStatusCols * (size_t)b->n * sizeof(double),
                               hipMemcpyDeviceToHost, b->stream));
    BHIP_TRY(b, hipStreamSynchronize(b->stream));
    int act = 0, err = 0;
    for (int i = 0; i < b->n; ++i) {
        act += b->h_status[oedg::kStatusCols * i] != 0.0;
        err += b->h_status[oedg::kStatusCols * i + 1] != 0.0;
    }
    if (n_active) *n_active = act;
    if (n_err) *n_err = err;
    return DG_OK;
}

}  // namespace

extern "C" {

dg_status dg_plan_chunks(int n_inst, const int32_t* n_cell, const int* k, int chunk_groups, int32_t* chunks,
                         int max_chunks, int* n_chunks, int32_t* split) {
    if (n_inst <= 0 || !n_cell || !k || chunk_groups <= 0 || !n_chunks) return DG_E_ARG;
    std::vector<oedg::Chunk> ch;
    oedg::ChunkSplit sp{};
    if (oedg::plan_chunks(n_inst, n_cell, k, chunk_groups, ch, sp) != 0) return DG_E_ARG;
    *n_chunks = (int)ch.size();
    if (chunks) {
        if (max_chunks < (int)ch.size()) return DG_E_ARG;
        for (size_t i = 0; i < ch.size(); ++i) {
            chunks[3 * i] = ch[i].inst;
            chunks[3 * i + 1] = ch[i].g0;
            chunks[3 * i + 2] = ch[i].g1;
        }
    }
    if (split)
        for (int x = 0; x < 9; ++x) split[x] = sp.b[x];
    return DG_OK;
}

dg_status dg_set_t_end(dg_ctx* c, double t_end) {
    if (!c) return DG_E_ARG;
    if (c->status != DG_OK) return c->status;
    if (c->host_only || !c->initialised) return capi::fail(c, DG_E_STATE, "state not initialised");
    if (std::isnan(t_end)) return capi::fail(c, DG_E_ARG, "t_end is NaN");
    if (hipSetDevice(c->device) != hipSuccess) return capi::fail(c, DG_E_HIP, "hipSetDevice failed");
    const int e = oedg::launch_set_end(c->g, t_end, c->stream);
    if (e != 0) return capi::fail(c, DG_E_HIP, std::string("k_set_end: ") + hipGetErrorString((hipError_t)e));
    return DG_OK;
}

dg_status dg_batch_create(dg_batch** out, dg_ctx* const* ctxs, int n, void* hip_stream) {
    if (!out) return DG_E_ARG;
    *out = nullptr;
    if (!ctxs || n <= 0) return DG_E_ARG;
    const dg_ctx* c0 = ctxs[0];
    for (int i = 0; i < n; ++i) {
        const dg_ctx* c = ctxs[i];
        if (!c || c->host_only || !c->initialised || c->status != DG_OK) return DG_E_STATE;
        if (c->device != c0->device || c->cfg.precision != c0->cfg.precision) return DG_E_ARG;
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == c) return DG_E_ARG;   // an instance appears once
    }
    dg_batch* b = new (std::nothrow) dg_batch();
    if (!b) return DG_E_NOMEM;
    b->device = c0->device;
    b->stream = (hipStream_t)hip_stream;
    b->n = n;
    b->mixed = c0->cfg.precision == DG_PREC_MIXED ? 1 : 0;
    b->ctx.assign(ctxs, ctxs + n);
    std::vector<int> gbase(n);
    for (int i = 0; i < n; ++i) {
        b->generation.push_back(ctxs[i]->generation);
        b->kmask |= ctxs[i]->cfg.k == 1 ? 1 : 2;
        gbase[i] = (int)b->total_groups;
        b->total_groups += oedg::n_groups(ctxs[i]->mesh.n_cell);
    }
    if (b->total_groups > (1LL << 30)) {
        delete b;
        return DG_E_ARG;
    }
    *out = b;
    if (hipSetDevice(b->device) != hipSuccess) return bfail(b, DG_E_HIP, "hipSetDevice failed");
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    const size_t n_desc = 3 * (size_t)n, n_chunk = (size_t)b->total_groups;
    const size_t o_desc = 0, o_chunk = al(n_desc * sizeof(oedg::StageArgs));
    const size_t o_part = o_chunk + al(n_chunk * sizeof(oedg::Chunk));
    const size_t o_stat = o_part + al((size_t)oedg::kPartCols * b->total_groups * sizeof(double));
    const size_t total = o_stat + al(oedg::kStatusCols * (size_t)n * sizeof(double));
    if (hipMalloc(&b->mem, total) != hipSuccess) return bfail(b, DG_E_NOMEM, "hipMalloc of the batch memory failed");
    if (b->kmask == 3) {   // one launch per degree: the second on a stream of its own
        BHIP_TRY(b, hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking));
        BHIP_TRY(b, hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming));
        BHIP_TRY(b, hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming));
    }
    char* base = (char*)b->mem;
    b->d_desc = (oedg::StageArgs*)(base + o_desc);
    b->d_chunks = (oedg::Chunk*)(base + o_chunk);
    b->d_part = (double*)(base + o_part);
    b->d_status = (double*)(base + o_stat);
    b->h_status.assign(oedg::kStatusCols * (size_t)n, 0.0);
    // stage arguments of every member, with the batch's partial records
    b->h_desc.resize(n_desc);
    for (int s = 0; s < 3; ++s)
        for (int i = 0; i < n; ++i) {
            oedg::StageArgs a = capi::stage_args(ctxs[i], s);
            a.part = b->d_part;
            a.gstride = (size_t)b->total_groups;
            a.gbase = gbase[i];
            b->h_desc[(size_t)s * n + i] = a;
        }
    BHIP_TRY(b, hipMemcpyAsync(b->d_desc, b->h_desc.data(), n_desc * sizeof(oedg::StageArgs), hipMemcpyHostToDevice,
                               b->stream));
    return plan(b);
}

dg_status dg_batch_set_schedule(dg_batch* b, int chunk_groups, int occupancy_pct) {
    dg_status st = ready(b);
    if (st != DG_OK) return st;
    if (chunk_groups < 1 || chunk_groups > 4096 || occupancy_pct < 1 || occupancy_pct > 100)
        return bfail(b, DG_E_ARG, "bad schedule parameters");
    b->chunk_groups = chunk_groups;
    b->occupancy_pct = occupancy_pct;
    return plan(b);
}

dg_status dg_batch_get_schedule(const dg_batch* b, int* chunk_groups, int* occupancy_pct, int* n_chunks, int* grid) {
    if (!b) return DG_E_ARG;
    if (chunk_groups) *chunk_groups = b->chunk_groups;
    if (occupancy_pct) *occupancy_pct = b->occupancy_pct;
    if (n_chunks) *n_chunks = (int)b->chunks.size();
    if (grid)
        for (int w = 0; w < oedg::kNumPasses; ++w) grid[w] = b->grid[0][w] + (b->n_launch == 2 ? b->grid[1][w] : 0);
    return DG_OK;
}

dg_status dg_batch_step(dg_batch* b, int64_t n_steps) {
    dg_status st = ready(b);
    if (st != DG_OK) return st;
    if (n_steps < 0) return bfail(b, DG_E_ARG, "negative step count");
    for (int64_t i = 0; i < n_steps; ++i)
        if ((st = run_step(b)) != DG_OK) return st;
    return DG_OK;
}

dg_status dg_batch_run(dg_batch* b, int64_t max_steps, int64_t* steps_done) {
    dg_status st = ready(b);
    if (st != DG_OK) return st;
    if (max_steps < 0) return bfail(b, DG_E_ARG, "negative step count");
    int64_t done = 0;
    int chunk = 4, act = 0, err = 0;
    if ((st = poll(b, &act, &err)) != DG_OK) return st;
    while (done < max_steps && act > 0) {
        // cap the chunk by the most steps any active member still needs at its current
        // Delta t: a launch after every member has finished replays the graph for nothing
        int64_t want = chunk;
        double need = 0.0;
        bool bounded = true;
        for (int i = 0; i < b->n; ++i) {
            const double* s = b->h_status.data() + oedg::kStatusCols * (size_t)i;
            if (s[0] == 0.0) continue;
            if (!std::isfinite(s[5]) || !(s[4] > 0.0)) {
                bounded = false;
                break;
            }
            need = std::max(need, std::ceil((s[5] - s[2]) / s[4]));
        }
        if (bounded) want = std::min<int64_t>(want, need < 1.0 ? 1 : (need > 64.0 ? 64 : (int64_t)need));
        const int64_t m = std::min<int64_t>(want, max_steps - done);
        for (int64_t i = 0; i < m; ++i)
            if ((st = run_step(b)) != DG_OK) return st;
        done += m;
        if ((st = poll(b, &act, &err)) != DG_OK) return st;
        chunk = std::min(chunk * 2, 64);
    }
    if (steps_done) *steps_done = done;
    if (err) return bfail(b, DG_E_BOUNDS, "a cell average of a member left the admissible set");
    return DG_OK;
}

dg_status dg_batch_status(dg_batch* b, int* n_active, double* status) {
    dg_status st = ready(b);
    if (st != DG_OK) return st;
    int act = 0;
    if ((st = poll(b, &act, nullptr)) != DG_OK) return st;
    if (n_active) *n_active = act;
    if (status)
        for (int i = 0; i < b->n; ++i)
            std::memcpy(status + 4 * (size_t)i, b->h_status.data() + oedg::kStatusCols * (size_t)i, 4 * sizeof(double));
    return DG_OK;
}

dg_status dg_batch_autotune(dg_batch* b, int reps, int* chunk_groups, int* occupancy_pct, double* ms_stage) {
    dg_status st = ready(b);
    if (st != DG_OK) return st;
    if (reps < 1) reps = 3;
    // stage 0 reads u^n and writes only the pre-filter and stage-output buffers and
    // the device scalars, which are saved here and restored afterwards
    std::vector<oedg::Glob> saved(b->n);
    for (int i = 0; i < b->n; ++i)
        BHIP_TRY(b, hipMemcpyAsync(&saved[i], b->ctx[i]->g, sizeof(oedg::Glob), hipMemcpyDeviceToHost, b->stream));
    BHIP_TRY(b, hipStreamSynchronize(b->stream));
    hipEvent_t e0, e1;
    BHIP_TRY(b, hipEventCreate(&e0));
    BHIP_TRY(b, hipEventCreate(&e1));
    static const int kChunkGroups[] = {1, 2, 4, 8, 16};
    static const int kOccupancy[] = {100, 50};
    int best_cg = b->chunk_groups, best_occ = b->occupancy_pct;
    double best = INFINITY;
    for (int cg : kChunkGroups) {
        for (int occ : kOccupancy) {
            b->chunk_groups = cg;
            b->occupancy_pct = occ;
            if ((st = plan(b)) != DG_OK) break;
            if ((st = run_stage(b, 0)) != DG_OK) break;   // warm-up
            BHIP_TRY(b, hipEventRecord(e0, b->stream));
            for (int r = 0; r < reps && st == DG_OK; ++r) st = run_stage(b, 0);
            BHIP_TRY(b, hipEventRecord(e1, b->stream));
            BHIP_TRY(b, hipEventSynchronize(e1));
            float ms = 0.0f;
            BHIP_TRY(b, hipEventElapsedTime(&ms, e0, e1));
            if (st == DG_OK && ms / reps < best) {
                best = ms / reps;
                best_cg = cg;
                best_occ = occ;
            }
        }
        if (st != DG_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    for (int i = 0; i < b->n; ++i)
        BHIP_TRY(b, hipMemcpyAsync(b->ctx[i]->g, &saved[i], sizeof(oedg::Glob), hipMemcpyHostToDevice, b->stream));
    BHIP_TRY(b, hipStreamSynchronize(b->stream));
    if (st != DG_OK) return st;
    b->chunk_groups = best_cg;
    b->occupancy_pct = best_occ;
    if ((st = plan(b)) != DG_OK) return st;
    if (chunk_groups) *chunk_groups = best_cg;
    if (occupancy_pct) *occupancy_pct = best_occ;
    if (ms_stage) *ms_stage = best;
    return DG_OK;
}

const char* dg_batch_last_error(const dg_batch* b) {
    if (!b) return "null batch";
    return b->err.c_str();
}

void dg_batch_destroy(dg_batch* b) {
    if (!b) return;
    (void)hipSetDevice(b->device);
    (void)hipStreamSynchronize(b->stream);
    drop_graph(b);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    if (b->side) (void)hipStreamDestroy(b->side);
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    if (b->ev_join) (void)hipEventDestroy(b->ev_join);
    if (b->mem) (void)hipFree(b->mem);
    delete b;
}

}  // extern "C"
