// l2c_check.hip -- host-side bounds checks of the index maps the execute kernels use, for
// one plan geometry (a test hook: leg2cheb_debug_check_geometry).  Every map is evaluated
// on the host with the same __host__ __device__ functions the kernels call, and every
// index is compared with the size of the buffer it addresses.  Nothing runs on a device.
#include <vector>

#include "l2c_internal.h"

namespace l2c {

void top_table_unit(int X, int G0, int *rec);   // l2c_fused.hip

// The checks, in order; the return value names the first that fails (0: all pass).
enum GeoCheck {
    kGeoOk = 0,
    kGeoSlots = 1,         // slot_depth: local blocks <-> (depth, index) is not one to one
    kGeoGroups = 2,        // the bottom table's groups do not hold every slot
    kGeoWorkspace = 3,     // a column node of some block lies past the workspace
    kGeoMainLds = 4,       // k_main's LDS exceeds the CU
    kGeoFusedLds = 5,      // k_fused's LDS areas overlap or overrun its allocation (where it applies)
    kGeoTopItems = 6,      // a unit's tree-top items exceed k_fused's register batch or the exchange buffer
    kGeoTopSched = 7,      // a reduction pair or slot of the tree-top table points past the unit's items
    kGeoRegen = 8,         // k_regen's output or factor-table index lies past its buffer
    kGeoUnits = 9          // the subtree count and the finest nodes disagree
};

int check_geometry_indices(int L, int M, int s)
{
    const Geometry G = make_geometry(L, M, s);
    const int kd = G.kd, G0 = G.groot;
    const int64_t P = int64_t(1) << (L + 1);          // finest nodes
    const int64_t U = int64_t(1) << (G0 + 2);         // subtrees of level groot
    if ((U << kd) != P) return kGeoUnits;
    // slot_depth: a bijection from [0, 2^kd - 1) onto {(d, i): 1 <= d <= kd, i < 2^(d-1)}
    const int nown = (1 << kd) - 1;
    std::vector<char> seen(nown > 0 ? nown : 1, 0);
    for (int j = 0; j < nown; ++j) {
        int d, i;
        slot_depth(j, kd, d, i);
        if (d < 1 || d > kd || i < 0 || i >= (1 << (d - 1))) return kGeoSlots;
        const int flat = (1 << (d - 1)) - 1 + i;      // blocks of depths < d come first here
        if (flat < 0 || flat >= nown || seen[flat]) return kGeoSlots;
        seen[flat] = 1;
    }
    if ((int64_t)G.sub_groups * 64 < (int64_t)nown * M) return kGeoGroups;
    // every block's column nodes 2b+2, 2b+3 of level g inside the workspace (NT nodes)
    for (int g = 0; g < L; ++g) {
        const int64_t blocks = (int64_t(1) << (g + 1)) - 1;
        if (node_offset(g) + 2 * (blocks - 1) + 3 >= G.NT) return kGeoWorkspace;
        if (node_offset(g) + (int64_t(1) << (g + 2)) > G.NT) return kGeoWorkspace;
    }
    if (main_lds_doubles(L, M, s, kd) * 8 > kMainLds) return kGeoMainLds;
    // the single launch: applies when fused_max_items' geometry conditions hold
    const int nodes = 1 << kd, R = kFusedRows;
    const bool fused = L >= 2 && kd >= 1 && 2 * M <= 64 && nodes * 2 * ((s + R - 1) / R) <= 64 * kNearWaves &&
                       G0 <= 6 && kd <= 7 && 2 * s <= 64 && 2 * (s * (nodes + 2) + R) <= kFusedStageG * kWorkThreads &&
                       2 * s * M <= kFusedStageT * kWorkThreads && 2 * s + 2 * R <= kWorkThreads &&
                       fused_lds_doubles(L, M, s, kd) * 8 <= kMainLds;
    if (fused) {
        // k_fused's LDS areas in the kernel's order (doubles): B(0), T (later the tree-top
        // items), the near-field area (input of both parities, Q, P; later the output rows),
        // w of every depth and the neighbour nodes, own c, the root c, the top wave's scratch,
        // the dummy node pair, the flag words
        const int64_t NS = 2 * M + 1, GX = fused_gx(s, kd), nQ = fused_nq(s, kd), nP = 2 * s + 2 * R;
        const int64_t Tl = (int64_t)M * M, gp = Tl + fused_t_area(L, M, s, kd);
        const int64_t Ql = gp + 2 * GX, Pl = Ql + nQ, wl = gp + fused_near_area(L, M, s, kd);
        const int64_t cown = wl + fused_wofs(kd + 1) * NS, cR = cown + (2 * (int64_t)nodes - 2) * NS;
        const int64_t w7 = cR + NS, dummy = w7 + fused_w7(M, G0), sync = dummy + 2 * NS;
        if (Pl + nP > wl || sync + 4 > fused_lds_doubles(L, M, s, kd)) return kGeoFusedLds;
        // the output rows (node stride 2s + 1) in the near-field area, dead once the near field is done
        if ((int64_t)nodes * (2 * s + 1) > fused_near_area(L, M, s, kd)) return kGeoFusedLds;
        if (2 * (int64_t)s * M > fused_t_area(L, M, s, kd)) return kGeoFusedLds;  // T
        // the logical input the near field reads per parity, s (nodes + 2) + R values
        if ((int64_t)(s + fused_gpad(s)) * (nodes + 2) > GX) return kGeoFusedLds;
        std::vector<int> rec(kTopSchedInts);
        for (int X = 0; X < (int)U; ++X) {
            top_table_unit(X, G0, rec.data());
            const int nitem = rec[45 + 14];            // entry kSchItems of the table
            if (nitem < 0 || nitem > 36 || 64 + nitem > kTopSchedInts) return kGeoTopItems;
            if ((int64_t)nitem * (2 * M + 1) > fused_t_area(L, M, s, kd)) return kGeoTopItems;   // items in the T area
            for (int it = 0; it < nitem; ++it) {
                const int node = rec[64 + it];
                if (node < 0 || node >= G.NX) return kGeoTopItems;
            }
            for (int r = 1; r <= 3; ++r) {              // reduction rounds: pairs (x, x + 2^(r-1))
                const int np = rec[r - 1];
                if (np < 0 || np > 14) return kGeoTopSched;
                for (int t = 0; t < np; ++t) {
                    const int x = rec[3 + 14 * (r - 1) + t];
                    if (x < 0 || x + (1 << (r - 1)) >= nitem) return kGeoTopSched;
                }
            }
            for (int sl = 0; sl < 14; ++sl) {           // each slot's first item, or -1
                const int f = rec[45 + sl];
                if (f < -1 || f >= nitem) return kGeoTopSched;
            }
        }
    }
    // k_regen: the far-field parts of every own block inside one item's share of cf, and its
    // factor-table rows inside the plan's table
    if (kd >= 1) {
        const int own = 2 * nodes - 2;
        const int64_t per_item = regen_cf_per_item(G), nlm = (int64_t)L * 2 * M * M;
        for (int j = 0; j < nown; ++j) {
            int d, i;
            slot_depth(j, kd, d, i);
            const int64_t last = ((U - 1) * own + (1 << d) - 2 + 2 * i) * 2 * M + 2 * 2 * M;
            if (last > per_item) return kGeoRegen;
            if ((int64_t)(G0 + d) * 2 * M * M + 2 * M * M > nlm) return kGeoRegen;
        }
    }
    return kGeoOk;
}

}  // namespace l2c
