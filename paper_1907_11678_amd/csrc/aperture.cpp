// aperture.cpp -- host-side construction of CRS apertures by radius: the
// gathers whose midpoint lies within a radius of the central gather's (the
// paper's neighbourhood of a central CDP, section 2.2, Fig. 2b), as the CSR
// lists that crs_scan and scan_batch take.  A uniform grid hash with cells of
// the radius's size keeps the search to the 3 x 3 cells around the central.

#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <unordered_map>
#include <vector>

#include "internal.h"

namespace {

struct CellKey {
    int64_t cx, cy;
    bool operator==(const CellKey &o) const { return cx == o.cx && cy == o.cy; }
};

struct CellHash {
    size_t operator()(const CellKey &k) const
    {
        const uint64_t a = (uint64_t)k.cx * 0x9E3779B97F4A7C15ULL, b = (uint64_t)k.cy + 0x632BE59BD9B4E019ULL;
        return std::hash<uint64_t>()(a ^ (b * 0xBF58476D1CE4E5B9ULL));
    }
};

}  // namespace

extern "C" int64_t semb_radius_apertures(const double *x, const double *y, int32_t ngathers,
                                         const int32_t *centrals, int32_t ncentrals, double radius,
                                         int32_t *apert_ptr, int32_t *apert_gather, int32_t *max_apert)
{
    if (!x || ngathers < 0 || ncentrals < 0 || (ncentrals > 0 && !centrals) || !apert_ptr ||
        !(radius >= 0.0) || !isfinite(radius)) {
        semb::set_last_error("semb_radius_apertures: invalid arguments (x, centrals and apert_ptr are "
                             "required, radius finite and >= 0)");
        return -1;
    }
    for (int32_t i = 0; i < ngathers; ++i)
        if (!isfinite(x[i]) || (y && !isfinite(y[i]))) {
            semb::set_last_error("semb_radius_apertures: midpoint coordinates must be finite");
            return -1;
        }
    for (int32_t c = 0; c < ncentrals; ++c)
        if (centrals[c] < 0 || centrals[c] >= ngathers) {
            semb::set_last_error("semb_radius_apertures: central gather out of range");
            return -1;
        }
    // cells of the radius's size (any positive size when the radius is 0:
    // then only coinciding midpoints are neighbours)
    const double cell = radius > 0.0 ? radius : 1.0;
    auto key_of = [&](int32_t i) {
        return CellKey{(int64_t)floor(x[i] / cell), y ? (int64_t)floor(y[i] / cell) : 0};
    };
    std::unordered_map<CellKey, std::vector<int32_t>, CellHash> grid;
    grid.reserve((size_t)ngathers);
    for (int32_t i = 0; i < ngathers; ++i) grid[key_of(i)].push_back(i);

    const double r2 = radius * radius;
    int64_t total = 0;
    int32_t longest = 0;
    std::vector<int32_t> found;
    apert_ptr[0] = 0;
    for (int32_t c = 0; c < ncentrals; ++c) {
        const int32_t g = centrals[c];
        const CellKey k = key_of(g);
        found.clear();
        for (int64_t dx = -1; dx <= 1; ++dx)
            for (int64_t dy = (y ? -1 : 0); dy <= (y ? 1 : 0); ++dy) {
                const auto it = grid.find(CellKey{k.cx + dx, k.cy + dy});
                if (it == grid.end()) continue;
                for (int32_t i : it->second) {
                    const double ex = x[i] - x[g], ey = y ? y[i] - y[g] : 0.0;
                    if (ex * ex + ey * ey <= r2) found.push_back(i);
                }
            }
        std::sort(found.begin(), found.end());
        if (apert_gather)
            std::copy(found.begin(), found.end(), apert_gather + total);
        total += (int64_t)found.size();
        if (total > INT32_MAX) {
            semb::set_last_error("semb_radius_apertures: more than 2^31 - 1 aperture entries");
            return -1;
        }
        apert_ptr[c + 1] = (int32_t)total;
        longest = std::max(longest, (int32_t)found.size());
    }
    if (max_apert) *max_apert = longest;
    return total;
}
