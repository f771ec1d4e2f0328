// Host-only footprint geometry of set_footprint / mppi_check_footprint, in
// plain C++ (no HIP), so that it can also be built on its own, for instance
// with the address and undefined-behaviour sanitizers.
#pragma once
#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <vector>

namespace emppi_host {

// Orientation of c relative to the line ab (twice the signed triangle area).
inline double orient2(const double* a, const double* b, const double* c) {
    return (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0]);
}
inline bool on_segment(const double* a, const double* b, const double* p) {
    return std::min(a[0], b[0]) <= p[0] && p[0] <= std::max(a[0], b[0]) &&
           std::min(a[1], b[1]) <= p[1] && p[1] <= std::max(a[1], b[1]);
}
// Proper intersection or touching of segments ab and cd (double precision).
inline bool segments_meet(const double* a, const double* b, const double* c, const double* d) {
    const double o1 = orient2(a, b, c), o2 = orient2(a, b, d);
    const double o3 = orient2(c, d, a), o4 = orient2(c, d, b);
    if (((o1 > 0 && o2 < 0) || (o1 < 0 && o2 > 0)) && ((o3 > 0 && o4 < 0) || (o3 < 0 && o4 > 0)))
        return true;
    if (o1 == 0 && on_segment(a, b, c)) return true;
    if (o2 == 0 && on_segment(a, b, d)) return true;
    if (o3 == 0 && on_segment(c, d, a)) return true;
    if (o4 == 0 && on_segment(c, d, b)) return true;
    return false;
}

// Simple-polygon check of the B vertices v = (x0, y0, x1, y1, ...): finite,
// no zero-length edge, non-zero area, and no two non-adjacent edges meeting
// (adjacent edges may only share their common vertex: a fold-back onto the
// previous edge is rejected too).  Returns 0 when the polygon passes,
// otherwise 1 with the reason in msg (len bytes).
inline int polygon_defect(const std::vector<double>& v, int B, char* msg, size_t len) {
    if (B < 3 || v.size() < static_cast<size_t>(2 * B)) {
        std::snprintf(msg, len, "need at least 3 vertices");
        return 1;
    }
    for (int k = 0; k < 2 * B; ++k)
        if (!std::isfinite(v[k])) {
            std::snprintf(msg, len, "non-finite vertex coordinate");
            return 1;
        }
    double area2 = 0.0;
    for (int b = 0; b < B; ++b) {
        const double* p = &v[2 * b];
        const double* q = &v[2 * ((b + 1) % B)];
        if (p[0] == q[0] && p[1] == q[1]) {
            std::snprintf(msg, len, "zero-length edge %d", b);
            return 1;
        }
        area2 += p[0] * q[1] - q[0] * p[1];
    }
    if (std::fabs(area2) * 0.5 < 1e-12) {
        std::snprintf(msg, len, "polygon area below 1e-12");
        return 1;
    }
    for (int i = 0; i < B; ++i) {
        const double* a = &v[2 * i];
        const double* b = &v[2 * ((i + 1) % B)];
        for (int j = i + 1; j < B; ++j) {
            const double* c = &v[2 * j];
            const double* d = &v[2 * ((j + 1) % B)];
            const bool next = (j == i + 1), prev = ((j + 1) % B == i);
            if (next || prev) {
                // adjacent: collinear overlap beyond the shared vertex is a fold-back
                const double* far = next ? d : c;          // the non-shared end of edge j
                const double* far_i = next ? a : b;        // the non-shared end of edge i
                const double* shared = next ? b : a;
                if ((orient2(a, b, far) == 0 && on_segment(a, b, far) &&
                     !(far[0] == shared[0] && far[1] == shared[1])) ||
                    (orient2(c, d, far_i) == 0 && on_segment(c, d, far_i))) {
                    std::snprintf(msg, len, "edges %d and %d fold back", i, j);
                    return 1;
                }
                continue;
            }
            if (segments_meet(a, b, c, d)) {
                std::snprintf(msg, len, "edges %d and %d touch or cross (not simple)", i, j);
                return 1;
            }
        }
    }
    return 0;
}

}  // namespace emppi_host
