// Host planning of the tiled forward projector (FP64, once per geometry).
//
// The rays of a work item (up to W angles x 64 bins) march through the image in
// slabs of H pixel rows (or columns, whichever axis the rays are closer to), (H, W)
// one of the forward's tilings.
// For each slab the planner computes the transverse pixel range every ray of the
// item can touch there, so the kernel stages exactly that window into LDS.
#include <algorithm>
#include <cmath>
#include <vector>

#include "radon_launch.hpp"

namespace radon {

namespace {

struct Span {
    int lo, hi;
};

// Transverse tap range [lo, hi] of one ray over march coordinates [m0, m1], with a
// one-pixel margin on each side for FP32 rounding in the kernel.
Span ray_span(const double4 &r, int axis, double m0, double m1) {
    const double om = axis ? r.x : r.y, ot = axis ? r.y : r.x;
    const double sm = axis ? r.z : r.w, st = axis ? r.w : r.z;
    const double t0 = ot + (m0 - om) * (st / sm);
    const double t1 = ot + (m1 - om) * (st / sm);
    const double lo = std::min(t0, t1), hi = std::max(t0, t1);
    return {(int)std::floor(lo) - 1, (int)std::floor(hi) + 2};
}

bool plan_item(int n, int det_count, const std::vector<double4> &rays, int slab_h, int a0, int na,
               int d0, int nd, std::vector<FwdItem> &items, std::vector<int2> &ranges, int &tile_t) {
    const double4 &mid = rays[(size_t)(a0 + na / 2) * det_count + d0 + nd / 2];
    const int axis = std::fabs(mid.w) >= std::fabs(mid.z) ? 0 : 1;
    // every ray must advance along the march axis by at least half a step per sample
    for (int a = a0; a < a0 + na; ++a)
        for (int d = d0; d < d0 + nd; ++d) {
            const double4 &r = rays[(size_t)a * det_count + d];
            const double sm = axis ? r.z : r.w;
            if (std::fabs(sm) < 0.5 * std::hypot(r.z, r.w)) return false;
        }
    const int nslabs = (n + 1 + slab_h - 1) / slab_h;
    std::vector<int2> local(nslabs);
    int first = -1, last = -1, width = 0;
    for (int s = 0; s < nslabs; ++s) {
        const double m_lo = -1.0 + (double)s * slab_h;
        int lo = 1 << 30, hi = -(1 << 30);
        for (int a = a0; a < a0 + na; ++a)
            for (int d : {d0, d0 + nd - 1}) {
                const Span sp = ray_span(rays[(size_t)a * det_count + d], axis, m_lo, m_lo + slab_h);
                lo = std::min(lo, sp.lo);
                hi = std::max(hi, sp.hi);
            }
        // taps of samples inside the support lie in [-1, N]; one more zero pixel on
        // each side absorbs FP32 rounding of boundary samples
        lo = std::max(lo, -2);
        hi = std::min(hi, n + 1);
        // keep every staged window at least 2 wide and inside [-2, N+1]
        if (lo == hi) {
            if (hi < n + 1)
                ++hi;
            else
                --lo;
        }
        local[s] = make_int2(lo, hi);
        if (lo <= hi) {
            if (first < 0) first = s;
            last = s;
            width = std::max(width, hi - lo + 1);
        }
    }
    if (width > kTileTMax) return false;
    if (first < 0) first = 0, last = -1;   // the rays miss the image: the item writes zeros
    FwdItem it;
    it.a0 = a0;
    it.na = na;
    it.d0 = d0;
    it.nd = nd;
    it.axis = axis;
    it.slab0 = first;
    it.nslab = last - first + 1;
    it.range = (int)ranges.size();
    for (int s = first; s <= last; ++s) ranges.push_back(local[s]);
    items.push_back(it);
    tile_t = std::max(tile_t, width);
    return true;
}

}  // namespace

bool plan_forward_tiles(int n, int n_angles, int det_count, const std::vector<double4> &rays,
                        int slab_h, int angles, std::vector<FwdItem> &items,
                        std::vector<int2> &ranges, int &tile_t) {
    items.clear();
    ranges.clear();
    tile_t = 0;
    for (int a0 = 0; a0 < n_angles; a0 += angles) {
        const int na = std::min(angles, n_angles - a0);
        for (int d0 = 0; d0 < det_count; d0 += kFwdLanes) {
            const int nd = std::min(kFwdLanes, det_count - d0);
            if (plan_item(n, det_count, rays, slab_h, a0, na, d0, nd, items, ranges, tile_t)) continue;
            // split: one angle per item, then fewer bins per item
            for (int a = a0; a < a0 + na; ++a) {
                int step = nd;
                for (int d = d0; d < d0 + nd;) {
                    const int cnt = std::min(step, d0 + nd - d);
                    if (plan_item(n, det_count, rays, slab_h, a, 1, d, cnt, items, ranges, tile_t)) {
                        d += cnt;
                    } else if (step > 8) {
                        step /= 2;
                    } else {
                        return false;
                    }
                }
            }
        }
    }
    return true;
}

BpWork plan_backproject(int beam, int n, const std::vector<double2> &trig, double spacing,
                        double step, double source_distance, double det_distance) {
    BpWork w;
    double hmax = 0.0;
    for (const double2 &cs : trig) hmax = std::max(hmax, std::fabs(cs.x) + std::fabs(cs.y));
    // 3 candidate steps must cover the footprint's extent along a ray (2*(|wx|+|wy|))
    if (2.0 * std::sqrt(2.0) / step > 3.0) return w;
    if (beam == 0) {
        // 3 candidate bins must cover the footprint's extent across the rays
        if (2.0 * hmax / spacing > 3.0) return w;
        const int win = (int)std::floor((kBpTile - 1) * hmax / spacing) + 3 + 3;
        if (((win + 3) & ~3) > kBpWinPar) return w;     // cannot happen (see kBpWinPar)
        w.window = (win + 3) & ~3;
        w.bins = 3;
        return w;
    }
    // fan beam: bound on the gradient of the detector coordinate s(P) over the image:
    // magnification at the image point nearest the source, times the secant of the
    // widest ray angle there
    const double S = source_distance, SE = source_distance + det_distance;
    const double reach = 0.5 * (n + 1) * std::sqrt(2.0) + 1.0;
    if (!(S > reach)) return w;
    const double grad = SE / (S - reach) * std::sqrt(1.0 + (reach / (S - reach)) * (reach / (S - reach)));
    // the kernel bounds s over a pixel footprint to first order with a margin of
    // 1% + 0.05 bins; the second-order term (|d|^2 |s''| / 2 <= 2 grad / (S - reach))
    // must stay inside that margin
    if (2.0 * grad / (S - reach) / spacing > 0.05) return w;
    const double span = 2.0 * std::sqrt(2.0) * grad / spacing * 1.01 + 0.1;
    const int nb = (int)std::floor(span) + 1;
    if (nb > 6) return w;
    w.bins = nb <= 4 ? 4 : 6;
    // window of a 16x16 tile footprint (corner to corner) plus the candidate span
    const double tile_span = (kBpTile + 1) * std::sqrt(2.0) * grad / spacing;
    const int win = (int)std::ceil(tile_span) + w.bins + 4;
    w.window = (win + 3) & ~3;
    return w;
}

}  // namespace radon
