// Library-private declarations shared by the C ABI sources (capi.hip, batch.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "oedg.h"
#include "oedg_internal.h"

struct dg_ctx {
    int device = 0;
    bool host_only = false;
    hipStream_t stream = nullptr;
    dg_status status = DG_OK;
    std::string err;

    void* bound = nullptr;       // caller-owned workspace
    size_t bound_bytes = 0;
    void* owned = nullptr;       // library allocation
    size_t used_bytes = 0;

    oedg::HostMesh mesh;
    bool have_mesh = false;
    bool initialised = false;
    dg_config cfg{};
    int nm = 0;

    double *jinv = nullptr, *area = nullptr, *len = nullptr, *node = nullptr;
    int32_t* link = nullptr;
    double *u0 = nullptr, *u = nullptr, *w = nullptr, *part = nullptr;
    int32_t *llink = nullptr, *halo_ptr = nullptr, *halo_cell = nullptr;
    const double* last_out = nullptr;
    oedg::Glob* g = nullptr;
    double* scratch = nullptr;   // the library's partial records on this device (dg_stage_noalloc)

    // kernel timing (dg_profile_enable)
    bool prof_on = false;
    std::vector<hipEvent_t> prof_ev;    // pairs: start, stop
    std::vector<int> prof_kind;         // kernel id of each pair
    size_t prof_used = 0;               // pairs recorded since the last read

    // one captured SSP-RK3 step, replayed on `stream` (rebuilt after set-up changes)
    hipStream_t cap_stream = nullptr;
    hipGraph_t step_graph = nullptr;
    hipGraphExec_t step_exec = nullptr;
    bool graph_failed = false;

    unsigned long long generation = 0;   // bumped by every mesh upload and (re)initialisation
};

namespace capi {

// records the first error of a context and returns it
dg_status fail(dg_ctx* c, dg_status s, const std::string& msg);
// device stage arguments of stage s (0, 1, 2; -1 initial limiter pass) of a context
oedg::StageArgs stage_args(dg_ctx* c, int s);

}  // namespace capi
