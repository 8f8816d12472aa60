// Host-side work plan of a pass launch over one or more instances: the chunk
// table (runs of reduction groups of one instance) and its split into one
// contiguous range per XCD, balanced by an estimated cost per cell.
#include <algorithm>
#include <vector>

#include "oedg_internal.h"

namespace oedg {

// relative cost of one cell-stage at degree k (P2 carries twice the modes and
// more quadrature points than P1)
static double cell_cost(int k) { return k == 2 ? 2.0 : 1.0; }

int plan_chunks(int n_inst, const int32_t* n_cell, const int* k, int chunk_groups, std::vector<Chunk>& chunks,
                ChunkSplit& split, int only_k) {
    if (n_inst <= 0 || chunk_groups <= 0) return -1;
    chunks.clear();
    std::vector<double> prefix(1, 0.0);
    for (int i = 0; i < n_inst; ++i) {
        if (n_cell[i] <= 0 || (k[i] != 1 && k[i] != 2)) return -1;
        if (only_k != 0 && k[i] != only_k) continue;
        const int ng = n_groups(n_cell[i]);
        for (int g0 = 0; g0 < ng; g0 += chunk_groups) {
            const int g1 = std::min(g0 + chunk_groups, ng);
            const int cells = std::min(g1 * kGroupCells, (int)n_cell[i]) - g0 * kGroupCells;
            chunks.push_back({i, g0, g1});
            prefix.push_back(prefix.back() + cells * cell_cost(k[i]));
        }
    }
    const int n = (int)chunks.size();
    const double total = prefix.back();
    split.b[0] = 0;
    for (int x = 1; x < 8; ++x) {
        // first chunk whose preceding cost reaches x/8 of the total
        const double target = total * x / 8.0;
        const int j = (int)(std::lower_bound(prefix.begin(), prefix.end() - 1, target) - prefix.begin());
        split.b[x] = std::max(split.b[x - 1], std::min(j, n));
    }
    split.b[8] = n;
    return 0;
}

int grid_for_split(const ChunkSplit& split, int resident) {
    int widest = 1;
    for (int x = 0; x < 8; ++x) widest = std::max(widest, split.b[x + 1] - split.b[x]);
    return 8 * std::max(1, std::min(widest, resident / 8));
}

}  // namespace oedg
