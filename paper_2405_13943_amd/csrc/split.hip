// Scene splitting into K blocks (Alg. 1) and the overlap grouping that makes
// shared Gaussians (Sec. 3.2).  Host code: it runs once per scene, before
// training, over the initial point cloud and the camera centres.
//
// Alg. 1: start from the tight box of all points; in rounds, every current
// cell (first in, first out) is removed, cut in two along its longer ground
// axis, and the two halves re-tightened and appended, until there are K
// cells (the last round stops at K); a cell of one point cannot be cut into
// two non-empty halves, so its turn appends it again unchanged.  The cut is
// the median: the floor(n/2) points with the smallest (coordinate, point id)
// form the first half, so blocks hold similar numbers of points.  Grouping:
// a point (or camera centre) belongs to every block whose cell box, grown by
// (s - 1) / 2 of its extent on each side (the box scaled by s about its
// centre), covers it on the tested axes (all three for points, the ground
// axes for cameras).
#include <algorithm>
#include <cstdint>
#include <deque>
#include <utility>
#include <vector>

#include "gs_internal.hpp"

namespace gs {

namespace {

struct Cell {
    double box[6];
    std::vector<int64_t> ids;       // ascending
};

void tight_box(const double* p, const std::vector<int64_t>& ids, double* box) {
    for (int a = 0; a < 3; a++) {
        box[a] = p[3 * ids[0] + a];
        box[3 + a] = p[3 * ids[0] + a];
    }
    for (int64_t i : ids)
        for (int a = 0; a < 3; a++) {
            box[a] = std::min(box[a], p[3 * i + a]);
            box[3 + a] = std::max(box[3 + a], p[3 * i + a]);
        }
}

// the two halves of a cell, cut along `axis`
void cut(const double* p, const Cell& c, int axis, Cell& lo, Cell& hi) {
    const size_t n = c.ids.size(), half = n / 2;
    std::vector<std::pair<double, int64_t>> keys(n);
    for (size_t k = 0; k < n; k++) keys[k] = {p[3 * c.ids[k] + axis], c.ids[k]};
    std::nth_element(keys.begin(), keys.begin() + half, keys.end());
    const std::pair<double, int64_t> pivot = keys[half];     // first key of the second half
    lo.ids.clear();
    hi.ids.clear();
    lo.ids.reserve(half);
    hi.ids.reserve(n - half);
    for (int64_t i : c.ids) {                                  // ascending ids stay ascending
        const std::pair<double, int64_t> k{p[3 * i + axis], i};
        (k < pivot ? lo.ids : hi.ids).push_back(i);
    }
    tight_box(p, lo.ids, lo.box);
    tight_box(p, hi.ids, hi.box);
}

}  // namespace

gs_status split_scene(const double* p, int64_t n, int32_t K, int32_t axes, double* boxes, int64_t* cell_of) {
    std::vector<int> ground;
    for (int a = 0; a < 3; a++)
        if (axes & (1 << a)) ground.push_back(a);
    std::deque<Cell> cells(1);
    cells[0].ids.resize(size_t(n));
    for (int64_t i = 0; i < n; i++) cells[0].ids[size_t(i)] = i;
    tight_box(p, cells[0].ids, cells[0].box);
    while (int32_t(cells.size()) < K) {
        // this round: the current cells, first in first out; each is removed
        // from the front and its halves appended at the back
        size_t round = cells.size();
        while (round > 0 && int32_t(cells.size()) < K) {
            Cell c = std::move(cells.front());
            cells.pop_front();
            round--;
            if (c.ids.size() < 2) {
                cells.push_back(std::move(c));
                continue;
            }
            int axis = ground[0];
            for (int a : ground)
                if (c.box[3 + a] - c.box[a] > c.box[3 + axis] - c.box[axis]) axis = a;
            Cell lo, hi;
            cut(p, c, axis, lo, hi);
            cells.push_back(std::move(lo));
            cells.push_back(std::move(hi));
        }
    }
    for (int32_t k = 0; k < K; k++) {
        for (int a = 0; a < 6; a++) boxes[6 * k + a] = cells[size_t(k)].box[a];
        if (cell_of)
            for (int64_t i : cells[size_t(k)].ids) cell_of[i] = k;
    }
    return GS_OK;
}

void split_group(const double* boxes, int32_t K, double s, int32_t axes, const double* p, int64_t n, int64_t* counts,
                 int64_t* members, int64_t capacity, int64_t* total) {
    std::vector<double> e(size_t(6) * size_t(K));
    for (int32_t k = 0; k < K; k++)
        for (int a = 0; a < 3; a++) {
            const double lo = boxes[6 * k + a], hi = boxes[6 * k + 3 + a];
            const double g = (s - 1.0) / 2.0 * (hi - lo);
            e[6 * size_t(k) + a] = lo - g;
            e[6 * size_t(k) + 3 + a] = hi + g;
        }
    auto covers = [&](int32_t k, int64_t i) {
        for (int a = 0; a < 3; a++) {
            if (!(axes & (1 << a))) continue;
            const double v = p[3 * i + a];
            if (!(e[6 * size_t(k) + a] <= v && v <= e[6 * size_t(k) + 3 + a])) return false;
        }
        return true;
    };
    int64_t sum = 0;
    for (int32_t k = 0; k < K; k++) {
        int64_t c = 0;
        for (int64_t i = 0; i < n; i++) c += covers(k, i) ? 1 : 0;
        counts[k] = c;
        sum += c;
    }
    *total = sum;
    if (!members || capacity < sum) return;
    int64_t o = 0;
    for (int32_t k = 0; k < K; k++)
        for (int64_t i = 0; i < n; i++)
            if (covers(k, i)) members[o++] = i;
}

}  // namespace gs
