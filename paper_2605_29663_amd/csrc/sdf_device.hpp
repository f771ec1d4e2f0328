// Device building blocks of the fused rollout-frame transform + exact
// signed distance + min-over-points stage, shared by the single-scene
// kernels and the batched persistent kernel.
//
// Paper: Section "Signed Distance Evaluation" (rollout-frame transform, box
// distance, polygon distance with ray-casting sign) and Section "Batched
// Rollout and Distance Computation" (K x T x N queries, masked min).
//
// Mapping on gfx950 (wave64, VALU-bound): one lane = one pose (rollout r,
// horizon h).  The footprint is rotated into the lane's frame once per work
// item (6 registers per polygon edge); every obstacle point is broadcast to
// all lanes from LDS, so the inner loop is pure per-lane VALU work with no
// cross-lane traffic, and the min over points is a private running minimum.
// Distances are kept squared and signed, s = sign(d) d^2 (monotone in d), so
// one square root per pose replaces one per (point, edge).
#pragma once
#include "kernels.hpp"

namespace emppi {

// Hardware reciprocal square root (v_rsq_f32, within 1 ulp) of the
// per-pose edge set-up: it normalises the edge direction and gives the edge
// length, both of which only scale the along/across coordinates by 1 +
// O(2^-23); a correctly rounded square root and division cost about 40
// instructions per edge and work item, against about 11 per edge and point
// in the loop.
__device__ __forceinline__ float fast_rsq(float x) { return __builtin_amdgcn_rsqf(x); }

// One polygon edge, from (xa, ya) to (xb, yb), taken from its lower end
// p = (px, py) towards its upper end (a horizontal edge keeps its order):
// unit direction e, length l, and the offsets that give the point's
// coordinates along and across the edge in two fused multiply-adds each,
//   u = e . (d - p) = fma(dx, ex, fma(dy, ey, nc)),   nc = -(e . p),
//   v = e x (d - p) = fma(dy, ex, fma(dx, -ey, cv)),  cv = ey px - ex py.
// The clipped projection is clamp(u, 0, l) and the squared point-to-segment
// distance (u - clamp(u, 0, l))^2 + v^2.  Because the edge points upwards, v
// > 0 says the point lies left of its line, i.e. a ray from the point towards
// +x crosses the edge when the edge straddles the point's height: the
// ray-casting test is the sign of v.  A zero-length edge gets e = 0, l = 0
// and cv = 3e18, a squared distance of 9e36 that never wins the minimum (its
// end points are those of the neighbouring edges), and never straddles.
struct EdgeC {
    float ex, ey, nc, cv, len;
};

__device__ __forceinline__ EdgeC edge_setup(float xa, float ya, float xb, float yb) {
    const bool down = yb < ya;
    const float px = down ? xb : xa, py = down ? yb : ya;
    const float qx = down ? xa : xb, qy = down ? ya : yb;
    const float dx = qx - px, dy = qy - py;
    const float l2 = __builtin_fmaf(dx, dx, dy * dy);
    const float r = l2 > 0.0f ? fast_rsq(l2) : 0.0f;
    EdgeC c;
    c.ex = dx * r;
    c.ey = dy * r;
    c.len = l2 * r;
    c.nc = -__builtin_fmaf(c.ex, px, c.ey * py);
    c.cv = l2 > 0.0f ? __builtin_fmaf(c.ey, px, -(c.ex * py)) : 3.0e18f;
    return c;
}

// The edge against the point (dx, dy): the squared distance, "the edge's
// first vertex lies above the point" (y > dy; Y = that vertex's y) and
// "the edge's line passes right of the point" (v > 0).
struct EdgeEval {
    float d2;
    bool above;
    bool right;
};

__device__ __forceinline__ EdgeEval edge_eval(float dx, float dy, float Y, float ex, float ey,
                                              float nc, float cv, float len) {
    const float u = __builtin_fmaf(dx, ex, __builtin_fmaf(dy, ey, nc));
    const float v = __builtin_fmaf(dy, ex, __builtin_fmaf(dx, -ey, cv));
    const float du = u - __builtin_amdgcn_fmed3f(u, 0.0f, len);
    EdgeEval e;
    e.d2 = __builtin_fmaf(du, du, v * v);
    e.above = dy < Y;
    e.right = v > 0.0f;
    return e;
}

// Signed squared distance of one box (centre c, half extents h) to the
// body-frame point (px, py): with a = |p - c| - h, i = max(a_x, a_y) and
// j = max(min(a_x, a_y), 0), sign(d) d^2 = i |i| + j^2, which is
// |max(a,0)|^2 outside and -(max(a_x, a_y))^2 inside (the box formula).
__device__ __forceinline__ float box_s(float px, float py, float4 b) {
    const float ax = fabsf(px - b.x) - b.z;
    const float ay = fabsf(py - b.y) - b.w;
    const float i = fmaxf(ax, ay);
    const float j = fmaxf(fminf(ax, ay), 0.0f);
    return __builtin_fmaf(j, j, i * fabsf(i));
}

__device__ __forceinline__ float pose_tau(const PoseTime& pt, int g) {
    const int h = (g / pt.div) % pt.mod;
    return static_cast<float>(h + pt.off) * pt.dt;
}

__device__ __forceinline__ float signed_sqrt(float s) {
    return s < 0.0f ? -__builtin_sqrtf(-s) : __builtin_sqrtf(s);
}

// A value that is the same in every lane, moved to scalar registers: every
// 32-bit word is taken from the first active lane.  For loads the compiler
// cannot prove uniform and unclobbered (a persistent kernel's descriptors,
// read after atomics of the previous work item), which would otherwise hold
// uniform data in vector registers.
template <typename T>
__device__ __forceinline__ T wave_uniform(const T& v) {
    static_assert(sizeof(T) % 4 == 0, "32-bit words");
    T r;
    const int* src = reinterpret_cast<const int*>(&v);
    int* dst = reinterpret_cast<int*>(&r);
#pragma unroll
    for (unsigned i = 0; i < sizeof(T) / 4; ++i) dst[i] = __builtin_amdgcn_readfirstlane(src[i]);
    return r;
}

// Stage points [t0, t0 + tn) of the compacted set into LDS: (x, y) pairs for
// static sets, (x, y, vx, vy) for moving ones.
template <bool MOVING>
__device__ __forceinline__ void stage_points(float* lds, const PointArgs& pts, int t0, int tn) {
    if (MOVING) {
        float4* l4 = reinterpret_cast<float4*>(lds);
        for (int i = threadIdx.x; i < tn; i += blockDim.x)
            l4[i] = make_float4(pts.x[t0 + i], pts.y[t0 + i], pts.vx[t0 + i], pts.vy[t0 + i]);
    } else {
        float2* l2 = reinterpret_cast<float2*>(lds);
        for (int i = threadIdx.x; i < tn; i += blockDim.x)
            l2[i] = make_float2(pts.x[t0 + i], pts.y[t0 + i]);
    }
}

// Point i of the staged tile at time tau, relative to the pose position.
template <bool MOVING>
__device__ __forceinline__ void point_rel(const float* lds, int i, float tau, float qx, float qy,
                                          float& dx, float& dy) {
    if (MOVING) {
        const float4 o = reinterpret_cast<const float4*>(lds)[i];
        dx = __builtin_fmaf(o.z, tau, o.x) - qx;
        dy = __builtin_fmaf(o.w, tau, o.y) - qy;
    } else {
        const float2 o = reinterpret_cast<const float2*>(lds)[i];
        dx = o.x - qx;
        dy = o.y - qy;
    }
}

// Two consecutive staged points i, i + 1 (i even) as raw LDS words, one
// 16-byte read per point pair (static) or per point (moving), so that the
// next pair's read can be in flight while the current pair is evaluated.
template <bool MOVING>
struct PointPair {
    float4 a, b;  // static: a = (x_i, y_i, x_i+1, y_i+1), b unused
};

template <bool MOVING>
__device__ __forceinline__ PointPair<MOVING> load_pair(const float* lds, int i) {
    const float4* l4 = reinterpret_cast<const float4*>(lds);
    PointPair<MOVING> p;
    if (MOVING) {
        p.a = l4[i];
        p.b = l4[i + 1];
    } else {
        p.a = l4[i >> 1];
        p.b = p.a;
    }
    // keep the read where it is issued (the scheduler would otherwise sink
    // it next to its first use, leaving its latency exposed)
    __builtin_amdgcn_sched_barrier(0);
    return p;
}

template <bool MOVING>
__device__ __forceinline__ void pair_rel(const PointPair<MOVING>& p, float tau, float qx, float qy,
                                         float& dx0, float& dy0, float& dx1, float& dy1) {
    if (MOVING) {
        dx0 = __builtin_fmaf(p.a.z, tau, p.a.x) - qx;
        dy0 = __builtin_fmaf(p.a.w, tau, p.a.y) - qy;
        dx1 = __builtin_fmaf(p.b.z, tau, p.b.x) - qx;
        dy1 = __builtin_fmaf(p.b.w, tau, p.b.y) - qy;
    } else {
        dx0 = p.a.x - qx;
        dy0 = p.a.y - qy;
        dx1 = p.a.z - qx;
        dy1 = p.a.w - qy;
    }
}

// f(pair, i) over the point pairs (i, i + 1) of a staged tile of tn points,
// i = 0, 2, ...: each pair's LDS read is issued one pair ahead, into two
// alternating register sets.  Returns the number of points covered (tn
// rounded down to even).
template <bool MOVING, typename Fn>
__device__ __forceinline__ int for_point_pairs(const float* lds, int tn, Fn&& f) {
    if (tn < 2) return 0;
    int i = 0;
    PointPair<MOVING> pa = load_pair<MOVING>(lds, 0);
    for (; i + 4 <= tn; i += 4) {
        const PointPair<MOVING> pb = load_pair<MOVING>(lds, i + 2);
        f(pa, i);
        pa = load_pair<MOVING>(lds, min(i + 4, tn - 2));
        f(pb, i + 2);
    }
    if (i + 2 <= tn) {
        f(pa, i);
        i += 2;
    }
    return i;
}

// Running min (and lowest-index argmin: points arrive in increasing index).
template <bool ARGMIN>
__device__ __forceinline__ void take(float s, int i, float& best, int& besti) {
    if (ARGMIN) {
        if (s < best) {
            best = s;
            besti = i;
        }
    } else {
        best = fminf(best, s);
    }
}

// Footprint of BP (padded) vertices rotated into the frame of pose q:
// centred at the pose, aligned with the planning frame, 6 registers per
// edge (the first vertex's y and EdgeC).  Padding repeats vertex 0, giving
// zero-length edges that never change the min and never straddle the ray.
template <int BP>
struct PolyFrame {
    float Y[BP], EX[BP], EY[BP], NC[BP], CV[BP], LN[BP];

    __device__ __forceinline__ void init(const float2* __restrict__ verts, float c, float s) {
        float2 v[BP];
#pragma unroll
        for (int b = 0; b < BP; ++b) v[b] = verts[b];
        init_from(v, c, s);
    }

    // The same from vertices already in registers.
    __device__ __forceinline__ void init_from(const float2 (&v)[BP], float c, float s) {
        float X[BP];
#pragma unroll
        for (int b = 0; b < BP; ++b) {
            X[b] = __builtin_fmaf(c, v[b].x, -(s * v[b].y));
            Y[b] = __builtin_fmaf(s, v[b].x, c * v[b].y);
        }
#pragma unroll
        for (int b = 0; b < BP; ++b) {
            const int bn = (b + 1) % BP;
            const EdgeC e = edge_setup(X[b], Y[b], X[bn], Y[bn]);
            EX[b] = e.ex;
            EY[b] = e.ey;
            NC[b] = e.nc;
            CV[b] = e.cv;
            LN[b] = e.len;
        }
    }

    // sign(d) d^2 of the point (dx, dy), given relative to the pose position.
    __device__ __forceinline__ float eval(float dx, float dy) const {
        EdgeEval e = edge_eval(dx, dy, Y[0], EX[0], EY[0], NC[0], CV[0], LN[0]);
        float m = e.d2;
        const bool above0 = e.above;
        bool above = e.above, right = e.right, odd = false;
#pragma unroll
        for (int b = 1; b < BP; ++b) {
            e = edge_eval(dx, dy, Y[b], EX[b], EY[b], NC[b], CV[b], LN[b]);
            m = fminf(m, e.d2);
            odd ^= (above != e.above) & right;
            above = e.above;
            right = e.right;
        }
        odd ^= (above != above0) & right;
        return odd ? -m : m;
    }
};

// Part of a footprint of L HB (padded) vertices for L = 2 or 4 consecutive
// lanes that share one pose: lane j of the group holds edges
// [j HB, (j + 1) HB), rotated exactly as in PolyFrame, and the y of the
// vertex closing its last edge.  Splitting the per-lane registers lets large
// polygons run at the occupancy of small ones; the group's partial minima
// and crossing parities are combined per point (min and parity are exact, so
// the result is the same bits as one lane holding every edge).
template <int HB, int L>
struct PolyPart {
    static_assert(L == 2 || L == 4, "lane groups of 2 or 4");
    float Y[HB], EX[HB], EY[HB], NC[HB], CV[HB], LN[HB];
    float Yend;

    __device__ __forceinline__ void init(const float2* __restrict__ verts, int b0, float c, float s) {
        float X[HB];
#pragma unroll
        for (int b = 0; b < HB; ++b) {
            const float2 v = verts[b0 + b];
            X[b] = __builtin_fmaf(c, v.x, -(s * v.y));
            Y[b] = __builtin_fmaf(s, v.x, c * v.y);
        }
        const float2 vn = verts[(b0 + HB) % (L * HB)];
        const float Xn = __builtin_fmaf(c, vn.x, -(s * vn.y));
        const float Yn = __builtin_fmaf(s, vn.x, c * vn.y);
#pragma unroll
        for (int b = 0; b < HB; ++b) {
            const EdgeC e = edge_setup(X[b], Y[b], b + 1 < HB ? X[b + 1] : Xn,
                                       b + 1 < HB ? Y[b + 1] : Yn);
            EX[b] = e.ex;
            EY[b] = e.ey;
            NC[b] = e.nc;
            CV[b] = e.cv;
            LN[b] = e.len;
        }
        Yend = Yn;
    }

    // Minimum squared distance over this lane's edges, and the crossing
    // parities of the ray from (dx, dy) over each lane's edges as a lane mask
    // of the wave (bit l set: lane l saw an odd number of crossings).  The
    // parity runs on the scalar unit on the compare masks; every lane of the
    // wave must be active.
    __device__ __forceinline__ void eval(float dx, float dy, float& m, unsigned long long& odd) const {
        EdgeEval e = edge_eval(dx, dy, Y[0], EX[0], EY[0], NC[0], CV[0], LN[0]);
        m = e.d2;
        unsigned long long above = __builtin_amdgcn_ballot_w64(e.above);
        unsigned long long right = __builtin_amdgcn_ballot_w64(e.right);
        odd = 0;
#pragma unroll
        for (int b = 1; b < HB; ++b) {
            e = edge_eval(dx, dy, Y[b], EX[b], EY[b], NC[b], CV[b], LN[b]);
            m = fminf(m, e.d2);
            const unsigned long long ab = __builtin_amdgcn_ballot_w64(e.above);
            odd ^= (above ^ ab) & right;
            above = ab;
            right = __builtin_amdgcn_ballot_w64(e.right);
        }
        odd ^= (above ^ __builtin_amdgcn_ballot_w64(dy < Yend)) & right;
    }
};

// Signed squared distance from a lane group's partial results (lanes
// L k .. L k + L - 1), valid in the group's first lane: the smallest
// minimum, negative when the group saw an odd number of crossings in total.
// The parities combine on the scalar unit (the wave's parity mask XOR
// itself shifted down by one lane, and for quads that result XOR itself
// shifted by two, leaves the group's parity in the bit of its first lane);
// the minima are non-negative, so their integer order is their float order
// and the partners' values arrive through DPP quad permutations ([1, 0, 3,
// 2], then [2, 3, 0, 1] for quads) folded into integer mins.  Every lane of
// the wave must be active.
template <int L>
__device__ __forceinline__ float part_combine(float m, unsigned long long odd) {
    unsigned long long par = odd ^ (odd >> 1);
    if (L == 4) par ^= par >> 2;
    const bool neg = __builtin_amdgcn_inverse_ballot_w64(par);
    int mi = __float_as_int(m);
    mi = min(mi, __builtin_amdgcn_mov_dpp(mi, 0xB1, 0xF, 0xF, true));
    if (L == 4) mi = min(mi, __builtin_amdgcn_mov_dpp(mi, 0x4E, 0xF, 0xF, true));
    const float mm = __int_as_float(mi);
    return neg ? -mm : mm;
}

// Min over the valid points [c0, c1) of the signed squared distance to the
// polygon for the pose (q, tau) held by this lane.  All threads of the
// workgroup must call it (LDS staging uses barriers).
template <int BP, bool MOVING, bool ARGMIN>
__device__ __forceinline__ void dmin_poly_range(float4 q, float tau, const PointArgs& pts, int c0,
                                                int c1, const float2* __restrict__ verts,
                                                float* lds, float& best, int& besti) {
    PolyFrame<BP> F;
    F.init(verts, q.z, q.w);
    best = INFINITY;
    besti = -1;
    for (int t0 = c0; t0 < c1; t0 += DMIN_TILE) {
        const int tn = min(DMIN_TILE, c1 - t0);
        __syncthreads();
        stage_points<MOVING>(lds, pts, t0, tn);
        __syncthreads();
        int i = 0;
        // two points per iteration while registers allow (a moving point
        // holds two more registers until its position at tau is formed),
        // the next pair read from LDS during the current one
        if (BP <= (MOVING ? 14 : 20)) {
            i = for_point_pairs<MOVING>(lds, tn, [&](const PointPair<MOVING>& p, int k) {
                float dx0, dy0, dx1, dy1;
                pair_rel<MOVING>(p, tau, q.x, q.y, dx0, dy0, dx1, dy1);
                const float s0 = F.eval(dx0, dy0);
                const float s1 = F.eval(dx1, dy1);
                take<ARGMIN>(s0, t0 + k, best, besti);
                take<ARGMIN>(s1, t0 + k + 1, best, besti);
            });
        }
        for (; i < tn; ++i) {
            float dx, dy;
            point_rel<MOVING>(lds, i, tau, q.x, q.y, dx, dy);
            take<ARGMIN>(F.eval(dx, dy), t0 + i, best, besti);
        }
    }
}

// Same with a group of L lanes per pose (L HB padded vertices, see
// PolyPart); the group's first lane returns the pose's minimum (the other
// lanes' results are not the pose's).  Every lane of the workgroup must call
// it with the same range.
template <int HB, int L, bool MOVING, bool ARGMIN = false>
__device__ __forceinline__ void dmin_poly_part_range(float4 q, float tau, const PointArgs& pts,
                                                     int c0, int c1, const float2* __restrict__ verts,
                                                     float* lds, float& best, int& besti) {
    PolyPart<HB, L> F;
    F.init(verts, (threadIdx.x & (L - 1)) * HB, q.z, q.w);
    best = INFINITY;
    besti = -1;
    for (int t0 = c0; t0 < c1; t0 += DMIN_TILE) {
        const int tn = min(DMIN_TILE, c1 - t0);
        __syncthreads();
        stage_points<MOVING>(lds, pts, t0, tn);
        __syncthreads();
        const int i = for_point_pairs<MOVING>(lds, tn, [&](const PointPair<MOVING>& p, int k) {
            float dx0, dy0, dx1, dy1, m0, m1;
            unsigned long long o0, o1;
            pair_rel<MOVING>(p, tau, q.x, q.y, dx0, dy0, dx1, dy1);
            F.eval(dx0, dy0, m0, o0);
            F.eval(dx1, dy1, m1, o1);
            take<ARGMIN>(part_combine<L>(m0, o0), t0 + k, best, besti);
            take<ARGMIN>(part_combine<L>(m1, o1), t0 + k + 1, best, besti);
        });
        if (i < tn) {
            float dx, dy, m;
            unsigned long long o;
            point_rel<MOVING>(lds, i, tau, q.x, q.y, dx, dy);
            F.eval(dx, dy, m, o);
            take<ARGMIN>(part_combine<L>(m, o), t0 + i, best, besti);
        }
    }
}

// Same for the rectangle cover: points rotated into the body frame,
// p = R(theta)^T (o - t), then the min over the RP (padded) boxes.
template <int RP, bool MOVING, bool ARGMIN>
__device__ __forceinline__ void dmin_rect_range(float4 q, float tau, const PointArgs& pts, int c0,
                                                int c1, const float4* __restrict__ rects,
                                                float* lds, float& best, int& besti) {
    float4 bx[RP];
#pragma unroll
    for (int j = 0; j < RP; ++j) bx[j] = RP <= 12 ? wave_uniform(rects[j]) : rects[j];
    best = INFINITY;
    besti = -1;
    auto eval = [&](float dx, float dy) {
        const float px = __builtin_fmaf(q.z, dx, q.w * dy);
        const float py = __builtin_fmaf(q.z, dy, -(q.w * dx));
        float s = box_s(px, py, bx[0]);
#pragma unroll
        for (int j = 1; j < RP; ++j) s = fminf(s, box_s(px, py, bx[j]));
        return s;
    };
    for (int t0 = c0; t0 < c1; t0 += DMIN_TILE) {
        const int tn = min(DMIN_TILE, c1 - t0);
        __syncthreads();
        stage_points<MOVING>(lds, pts, t0, tn);
        __syncthreads();
        const int i = for_point_pairs<MOVING>(lds, tn, [&](const PointPair<MOVING>& p, int k) {
            float dx0, dy0, dx1, dy1;
            pair_rel<MOVING>(p, tau, q.x, q.y, dx0, dy0, dx1, dy1);
            take<ARGMIN>(eval(dx0, dy0), t0 + k, best, besti);
            take<ARGMIN>(eval(dx1, dy1), t0 + k + 1, best, besti);
        });
        if (i < tn) {
            float dx, dy;
            point_rel<MOVING>(lds, i, tau, q.x, q.y, dx, dy);
            take<ARGMIN>(eval(dx, dy), t0 + i, best, besti);
        }
    }
}

}  // namespace emppi
