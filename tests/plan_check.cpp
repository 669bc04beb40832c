// CPU check of the stage kernel's work lists (hrlb_plan.h): for many random ragged batches and
// single cases, every natural tile appears exactly once, padding records are the only extras,
// position p of a list belongs to the chunk of XCD p % 8 (chunks contiguous in the natural order),
// and the validator accepts the list at its own length and rejects it one record shorter.  The
// per-cell kernel's block list covers every cell of every instance once and holds two wall blocks
// for each instance that asks for them (none for the others), all of them ahead of the cell blocks;
// the balanced order of a batch's cell blocks is a permutation of them that keeps the wall blocks in
// place and, read round by round in the order it deals them (every other round of R positions
// backwards), lists the blocks by non-increasing weight.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <tuple>
#include <vector>

#include "hrlb_plan.h"

using namespace hrlb;

static int fails = 0;
#define CHECK(c)                                                          \
    do {                                                                  \
        if (!(c)) {                                                       \
            std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            ++fails;                                                      \
        }                                                                 \
    } while (0)

static void check_list(const std::vector<TileRef>& tiles, const std::vector<PlanShape>& shapes)
{
    std::map<std::tuple<int, int, int>, int> seen;
    size_t natural = 0;
    std::vector<int> nct, ngr;
    for (const PlanShape& s : shapes) {
        natural += (size_t)s.nctiles * s.ngroups;
        nct.push_back(s.nctiles);
        ngr.push_back(s.ngroups);
    }
    CHECK(tiles.size() % kXcds == 0);
    CHECK(tiles.size() >= natural);
    size_t real = 0;
    for (const TileRef& t : tiles) {
        if (t.inst < 0) continue;
        ++real;
        seen[std::make_tuple(t.inst, t.ctile, t.group)]++;
    }
    CHECK(real == natural);
    for (auto& kv : seen) CHECK(kv.second == 1);
    CHECK(tiles_valid(tiles, tiles.size(), (int)shapes.size(), nct.data(), ngr.data()));
    if (!tiles.empty()) CHECK(!tiles_valid(tiles, tiles.size() - 1, (int)shapes.size(), nct.data(), ngr.data()));
    // chunks: the records at positions x, x+8, ... are contiguous in the natural order
    for (int x = 0; x < kXcds; ++x) {
        long last = -1;
        for (size_t p = x; p < tiles.size(); p += kXcds) {
            const TileRef& t = tiles[p];
            if (t.inst < 0) continue;
            long key = 0;
            for (int i = 0; i < t.inst; ++i) key += (long)shapes[i].nctiles * shapes[i].ngroups;
            key += (long)t.group * shapes[t.inst].nctiles + t.ctile;
            CHECK(key > last);
            last = key;
        }
    }
}

static void check_cell_cover(const std::vector<CellRef>& b, const std::vector<int>& ncells, const std::vector<int>& cpb,
                             const std::vector<char>& own)
{
    size_t expect = 0;
    for (size_t i = 0; i < ncells.size(); ++i) expect += cell_block_count(ncells[i], cpb[i], own[i]);
    CHECK(b.size() == expect);
    std::vector<int> walls_l(ncells.size(), 0), walls_r(ncells.size(), 0);
    std::vector<std::vector<int>> covered(ncells.size());
    for (size_t i = 0; i < ncells.size(); ++i) covered[i].assign(ncells[i], 0);
    bool seen_cells = false;
    for (const CellRef& r : b) {
        CHECK(r.inst >= 0 && r.inst < (int)ncells.size());
        if (r.cell0 < 0) {
            CHECK(!seen_cells);
            CHECK(r.cell0 == kWallLeft || r.cell0 == kWallRight);
            (r.cell0 == kWallLeft ? walls_l : walls_r)[r.inst]++;
            continue;
        }
        seen_cells = true;
        CHECK(r.cell0 < ncells[r.inst]);
        for (int s = r.cell0; s < r.cell0 + cpb[r.inst] && s < ncells[r.inst]; ++s) covered[r.inst][s]++;
    }
    for (size_t i = 0; i < ncells.size(); ++i) {
        CHECK(walls_l[i] == (own[i] ? 1 : 0) && walls_r[i] == walls_l[i]);
        for (int c : covered[i]) CHECK(c == 1);
    }
}

static void check_cell_blocks(const std::vector<int>& ncells, const std::vector<int>& cpb, const std::vector<char>& own)
{
    const std::vector<CellRef> b = plan_cell_blocks(ncells, cpb, own);
    check_cell_cover(b, ncells, cpb, own);
    // the balanced order, with random instance weights and unit counts
    std::vector<double> w(ncells.size());
    for (double& x : w) x = (double)(std::rand() % 7);
    const int R = 1 + std::rand() % 300;
    size_t first = 0;
    while (first < b.size() && b[first].cell0 < 0) ++first;
    std::vector<CellRef> bb = b;
    balance_cell_blocks(bb, first, w, R);
    check_cell_cover(bb, ncells, cpb, own);
    for (size_t k = 0; k < first; ++k) CHECK(bb[k].inst == b[k].inst && bb[k].cell0 == b[k].cell0);
    const size_t n = bb.size() - first;
    double prev = 1e300;
    for (size_t r = 0; r * R < n; ++r) {
        const size_t len = std::min((size_t)R, n - r * R);
        for (size_t i = 0; i < len; ++i) {
            const size_t pos = first + r * R + ((r & 1) ? len - 1 - i : i);
            CHECK(w[bb[pos].inst] <= prev);
            prev = w[bb[pos].inst];
        }
    }
}

int main()
{
    std::srand(12345);
    for (int trial = 0; trial < 400; ++trial) {
        const int n = 1 + std::rand() % 40;
        std::vector<PlanShape> shapes;
        for (int i = 0; i < n; ++i) {
            const int ncells = 8 + 4 * (std::rand() % 600);
            const int nct = (ncells + kPlanTileCells - 1) / kPlanTileCells;
            shapes.push_back(PlanShape{nct, 1 + std::rand() % 60, 1 + std::rand() % 8, ncells});
        }
        check_list(plan_batch_tiles(shapes), shapes);
        std::vector<int> nc, cpb;
        std::vector<char> own;
        for (const PlanShape& s : shapes) {
            nc.push_back(s.ncells);
            cpb.push_back(256 >> (std::rand() % 5));  // 1 to 16 lanes per cell
            own.push_back((char)(std::rand() % 2));
        }
        check_cell_blocks(nc, cpb, own);
        const PlanShape& s = shapes[0];
        std::vector<PlanShape> one{s};
        check_list(case_tiles(s.nctiles, s.ngroups), one);
    }
    std::printf("plan checks: %d failures\n", fails);
    return fails ? 1 : 0;
}
