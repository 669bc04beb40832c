// hrlb_plan.h -- work lists of the stage kernel (host only, no HIP dependency).
#pragma once

#include <algorithm>
#include <vector>

namespace hrlb {

constexpr int kPlanTileCells = 64;  // cells per tile of the stage kernel
constexpr int kXcds = 8;            // MI355X: 8 accelerator complex dies, each with its own L2

struct TileRef {   // one block-sized unit of the stage kernel
    int inst;      // -1: padding, skipped
    int ctile;     // cell tile index within the instance
    int group;     // velocity group index within the instance
    int tile_id;   // ctile * ngroups + group (residual partial slot)
};

struct CellRef {   // one block of the per-cell kernel
    int inst;
    int cell0;     // first cell, or kWallLeft / kWallRight for a block that only does that wall
};
constexpr int kWallLeft = -1, kWallRight = -2;
constexpr int kPlanCellThreads = 256;  // threads per block of the per-cell kernel

// The leaving fluxes through a wall are a block-wide reduction over the qx*qy leaving velocities.
// When that takes more than one pass of a block, each wall gets a block of its own, which runs
// beside the cell blocks instead of after the cell work of the edge block; otherwise the edge
// blocks do it (extra blocks for the many small instances of a batch cost more than they save).
// Both give the same bits.
constexpr bool wall_blocks_of_their_own(int qx, int qy) { return qx * qy > kPlanCellThreads; }

// Blocks of the per-cell kernel for a list of instances: the wall blocks first, then the cell
// blocks, cells_per_block[i] cells each.
inline std::vector<CellRef> plan_cell_blocks(const std::vector<int>& ncells, const std::vector<int>& cells_per_block,
                                             const std::vector<char>& own_walls)
{
    std::vector<CellRef> out;
    for (int i = 0; i < (int)ncells.size(); ++i)
        if (own_walls[i]) {
            out.push_back(CellRef{i, kWallLeft});
            out.push_back(CellRef{i, kWallRight});
        }
    for (int i = 0; i < (int)ncells.size(); ++i)
        for (int c0 = 0; c0 < ncells[i]; c0 += cells_per_block[i]) out.push_back(CellRef{i, c0});
    return out;
}
// Order of a batch's cell blocks (positions first, first + 1, ... of the list, after its wall
// blocks).  All blocks of the per-cell kernel are resident at once; they are dealt to the XCDs round
// robin and, within an XCD, to its compute units in turn, so positions p, p + R, p + 2R, ... (R = the
// compute units) share a unit.  The blocks are sorted by the per-cell work of their instance
// (inst_weight), heaviest first, and every other round of R positions is reversed: a unit then pairs
// the heaviest blocks of one round with the lightest of the next, which evens out the units' loads.
// Measured on the 512-instance batch (Q_x from 4 to 32): the per-cell launch from 56 to 47 us, while
// a random order leaves it at 56 us.  Only the order changes, not what any block computes.
inline void balance_cell_blocks(std::vector<CellRef>& blocks, size_t first, const std::vector<double>& inst_weight,
                                int round)
{
    if (round <= 0 || blocks.size() <= first + 1) return;
    std::vector<CellRef> b(blocks.begin() + first, blocks.end());
    std::stable_sort(b.begin(), b.end(),
                     [&](const CellRef& x, const CellRef& y) { return inst_weight[x.inst] > inst_weight[y.inst]; });
    const size_t n = b.size(), R = (size_t)round;
    for (size_t k = 0; k < n; ++k) {
        const size_t r = k / R, i = k % R, len = std::min(R, n - r * R);
        blocks[first + r * R + ((r & 1) ? len - 1 - i : i)] = b[k];
    }
}
inline int cell_block_count(int ncells, int cells_per_block, bool own_walls)
{
    return (own_walls ? 2 : 0) + (ncells + cells_per_block - 1) / cells_per_block;
}

struct PlanShape {  // what the tile list needs to know about one instance
    int nctiles, ngroups, vpt, ncells;
};

// XCD-aware order of a tile list.  Workgroups are dispatched to the 8 XCDs round robin, and the
// persistent stage kernel gives block b the positions b, b + grid, ... (grid a multiple of 8), so
// position p runs on XCD p % 8.  The natural sequence (instance, velocity group, cell tile) keeps
// tiles that share halos and cell tables next to each other; it is cut into 8 contiguous chunks of
// about equal work, chunk x is laid on positions x, x + 8, ..., and short chunks are padded with
// empty tiles (inst = -1) so that every chunk stays on its own XCD's L2.
inline std::vector<TileRef> xcd_order(const std::vector<TileRef>& seq, const std::vector<double>& cost)
{
    double total = 0.0;
    for (double c : cost) total += c;
    std::vector<std::vector<TileRef>> chunk(kXcds);
    double acc = 0.0;
    for (size_t t = 0; t < seq.size(); ++t) {
        const int x = total > 0.0 ? (int)std::min<double>(kXcds - 1, acc / total * kXcds) : 0;
        chunk[x].push_back(seq[t]);
        acc += cost[t];
    }
    size_t mx = 0;
    for (auto& c : chunk) mx = std::max(mx, c.size());
    std::vector<TileRef> out(mx * kXcds, TileRef{-1, 0, 0, 0});
    for (int x = 0; x < kXcds; ++x)
        for (size_t k = 0; k < chunk[x].size(); ++k) out[k * kXcds + x] = chunk[x][k];
    return out;
}

// tile list of one case: natural sequence (velocity group, cell tile), XCD-aware order
inline std::vector<TileRef> case_tiles(int nctiles, int ngroups)
{
    std::vector<TileRef> seq;
    for (int g = 0; g < ngroups; ++g)
        for (int ct = 0; ct < nctiles; ++ct) seq.push_back(TileRef{0, ct, g, ct * ngroups + g});
    return xcd_order(seq, std::vector<double>(seq.size(), 1.0));
}

// tile list of a batch: natural sequence over instances, XCD-aware order weighted by the work of
// each tile (velocities per row x cells)
inline std::vector<TileRef> plan_batch_tiles(const std::vector<PlanShape>& shapes)
{
    std::vector<TileRef> seq;
    std::vector<double> cost;
    for (int i = 0; i < (int)shapes.size(); ++i) {
        const PlanShape& s = shapes[i];
        for (int g = 0; g < s.ngroups; ++g)
            for (int ct = 0; ct < s.nctiles; ++ct) {
                seq.push_back(TileRef{i, ct, g, ct * s.ngroups + g});
                cost.push_back((double)s.vpt * std::min(kPlanTileCells, s.ncells - ct * kPlanTileCells));
            }
    }
    return xcd_order(seq, cost);
}

// every record must name an instance of the list (or be padding) and a cell tile and velocity
// group of that instance; checked on the host before any upload
inline bool tiles_valid(const std::vector<TileRef>& tiles, size_t capacity, int ninst, const int* nctiles,
                        const int* ngroups)
{
    if (tiles.size() > capacity) return false;
    for (const TileRef& t : tiles) {
        if (t.inst == -1) continue;
        if (t.inst < 0 || t.inst >= ninst) return false;
        const int nc = nctiles[t.inst], ng = ngroups[t.inst];
        if (t.ctile < 0 || t.ctile >= nc || t.group < 0 || t.group >= ng || t.tile_id != t.ctile * ng + t.group)
            return false;
    }
    return true;
}

}  // namespace hrlb
