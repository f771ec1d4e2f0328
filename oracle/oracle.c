/*
 * CPU oracle for one MPPI control step with exact footprint signed distance.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and
 * the CPU-baseline leg of the benchmark may load this library.  The product
 * path (the HIP library) never links, loads or calls it, and this file shares
 * no code, header or constant table with it.
 *
 * Everything here is plain scalar C in IEEE double precision, written from the
 * paper's text (section and equation names are given at each function), except
 * the "FP32 mirror" block: the paper leaves the sampling distribution and the
 * arithmetic precision of the rollout open, and the method's contract asks for
 * rollouts that are bit-identical to the GPU's for the same counter-based seed.
 * That block therefore spells out one single-precision operation sequence
 * (Philox4x64-10, Box-Muller with series-based log/sin/cos, forward Euler) that
 * any IEEE-754 implementation reproduces exactly.  Its accuracy is pinned
 * against the double-precision rollout and closed forms, not against itself.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC.
 * No fused multiply-add is formed implicitly; the FP32 mirror calls fmaf()
 * exactly where the operation sequence says "fma".
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#include <float.h>

#define EXPORT __attribute__((visibility("default")))

/* ======================================================================== */
/* Geometry (Section "Signed Distance Evaluation")                          */
/* ======================================================================== */

/* Point-to-segment distance, Section "Distance to General Simple Polygonal
 * Footprint": clipped projection parameter alpha_b = clamp(((p-v_b).e_b) /
 * |e_b|^2, 0, 1) and d_seg = |p - (v_b + alpha_b e_b)|.  (The printed d_seg
 * groups alpha_b with v_b; the point on the edge is v_b + alpha_b e_b.)     */
EXPORT double orc_seg_dist(double px, double py, double ax, double ay,
                           double bx, double by) {
    double ex = bx - ax, ey = by - ay;
    double l2 = ex * ex + ey * ey;
    double alpha = ((px - ax) * ex + (py - ay) * ey) / l2;
    if (alpha < 0.0) alpha = 0.0;
    if (alpha > 1.0) alpha = 1.0;
    double qx = ax + alpha * ex, qy = ay + alpha * ey;
    double dx = px - qx, dy = py - qy;
    return sqrt(dx * dx + dy * dy);
}

/* Orientation of p relative to the directed line a->b (twice the signed
 * triangle area): > 0 when p lies to the left.                              */
static double orient(double ax, double ay, double bx, double by, double px, double py) {
    return (bx - ax) * (py - ay) - (px - ax) * (by - ay);
}

/* Winding number of the closed vertex cycle V (B vertices, x0,y0,x1,y1,...)
 * around p.  A simple polygon contains p iff the winding number is non-zero.
 * This is the orientation-based crossing count: an upward edge that has p
 * strictly on its left adds one, a downward edge with p strictly on its
 * right subtracts one.                                                      */
EXPORT int orc_winding(const double* V, int B, double px, double py) {
    int wn = 0;
    for (int b = 0; b < B; ++b) {
        int c = (b + 1) % B;
        double ay = V[2 * b + 1], cy = V[2 * c + 1];
        double o = orient(V[2 * b], ay, V[2 * c], cy, px, py);
        if (ay <= py) {
            if (cy > py && o > 0.0) ++wn;
        } else {
            if (cy <= py && o < 0.0) --wn;
        }
    }
    return wn;
}

/* The paper's own inside test, "implemented via ray casting" (Section
 * "Distance to General Simple Polygonal Footprint"): parity of the crossings
 * of the ray from p towards +x, counting an edge when its end-point y values
 * straddle p_y under the half-open rule and the crossing lies right of p.    */
EXPORT int orc_inside_raycast(const double* V, int B, double px, double py) {
    int odd = 0;
    for (int b = 0; b < B; ++b) {
        int c = (b + 1) % B;
        double ax = V[2 * b], ay = V[2 * b + 1], cx = V[2 * c], cy = V[2 * c + 1];
        if ((ay > py) != (cy > py)) {
            double xc = ax + (py - ay) * (cx - ax) / (cy - ay);
            if (px < xc) odd ^= 1;
        }
    }
    return odd;
}

/* Signed distance to a simple polygon, eq. for d_poly: sigma(p) times the
 * minimum over edges of d_seg.  The sign is -1 inside, +1 outside (Section
 * "Robot--Obstacle Signed Distance"); inside-ness is decided by the winding
 * number, the plain definition of containment for a closed curve.           */
EXPORT double orc_sdf_polygon(const double* V, int B, double px, double py) {
    double dmin = INFINITY;
    for (int b = 0; b < B; ++b) {
        int c = (b + 1) % B;
        double d = orc_seg_dist(px, py, V[2 * b], V[2 * b + 1], V[2 * c], V[2 * c + 1]);
        if (d < dmin) dmin = d;
    }
    return orc_winding(V, B, px, py) != 0 ? -dmin : dmin;
}

/* Point-to-box signed distance, Section "Distance to Orthogonal Footprints":
 * a = |p - c| - s (elementwise), d_box = |max(a,0)|_2 + min(max(a_x,a_y),0).
 * rect = (c_x, c_y, s_x, s_y).                                              */
EXPORT double orc_sdf_box(const double* rect, double px, double py) {
    double ax = fabs(px - rect[0]) - rect[2];
    double ay = fabs(py - rect[1]) - rect[3];
    double mx = ax > 0.0 ? ax : 0.0, my = ay > 0.0 ? ay : 0.0;
    double outside = sqrt(mx * mx + my * my);
    double m = ax > ay ? ax : ay;
    double inside = m < 0.0 ? m : 0.0;
    return outside + inside;
}

/* Rectangle-cover signed distance: minimum over the R boxes (same section). */
EXPORT double orc_sdf_rectcover(const double* rects, int R, double px, double py) {
    double d = INFINITY;
    for (int j = 0; j < R; ++j) {
        double dj = orc_sdf_box(rects + 4 * j, px, py);
        if (dj < d) d = dj;
    }
    return d;
}

EXPORT void orc_sdf_polygon_batch(const double* V, int B, const double* px,
                                  const double* py, long n, double* out) {
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) out[i] = orc_sdf_polygon(V, B, px[i], py[i]);
}

EXPORT void orc_sdf_rectcover_batch(const double* rects, int R, const double* px,
                                    const double* py, long n, double* out) {
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) out[i] = orc_sdf_rectcover(rects, R, px[i], py[i]);
}

/* Rollout-frame transformation, Section "Rollout-Frame Transformation":
 * p = R(theta)^T (o - t).  The pose is given as (x, y, cos theta, sin theta),
 * so R(theta)^T d = (c d_x + s d_y, -s d_x + c d_y).                        */
static void to_body(const double* pose, double ox, double oy, double* bx, double* by) {
    double dx = ox - pose[0], dy = oy - pose[1];
    double c = pose[2], s = pose[3];
    *bx = c * dx + s * dy;
    *by = -s * dx + c * dy;
}

/* Minimum signed-distance matrix, Section "Batched Rollout and Distance
 * Computation" and Algorithm 1 step 2: for every pose, the minimum over the
 * valid obstacle points of d(p_i) in that pose's body frame.  Masked points
 * never contribute; with no valid point the minimum is +inf.  Points may
 * move with constant velocity: at pose k the point is o_i + v_i tau[k].
 * kind 0 = polygon (geom = B vertices), kind 1 = rectangle cover (geom = R
 * boxes).  argmin (may be NULL) receives the lowest index attaining the
 * minimum, or -1.                                                           */
EXPORT void orc_dmin(const double* poses, const double* tau, long npose,
                     const double* ox, const double* oy, const double* ovx,
                     const double* ovy, const unsigned char* valid, long n,
                     int kind, const double* geom, int count, double* dmin,
                     int* argmin) {
#pragma omp parallel for schedule(dynamic, 16)
    for (long k = 0; k < npose; ++k) {
        double best = INFINITY;
        int bi = -1;
        for (long i = 0; i < n; ++i) {
            if (valid && !valid[i]) continue;
            double x = ox[i], y = oy[i];
            if (ovx) x += ovx[i] * tau[k];
            if (ovy) y += ovy[i] * tau[k];
            double bx, by;
            to_body(poses + 4 * k, x, y, &bx, &by);
            double d = kind == 0 ? orc_sdf_polygon(geom, count, bx, by)
                                 : orc_sdf_rectcover(geom, count, bx, by);
            if (d < best) { best = d; bi = (int)i; }
        }
        dmin[k] = best;
        if (argmin) argmin[k] = bi;
    }
}

/* ======================================================================== */
/* Motion models, Section "Robot Kinematic Models" (double precision)       */
/* ======================================================================== */

enum { M_UNICYCLE = 0, M_ACKERMANN = 1, M_OMNI = 2, M_SPIN = 3, M_PARALLEL = 4 };

/* F_m(q, u) for the five models of the paper.  u holds (v, omega) for the
 * unicycle, (v, delta) for Ackermann with wheelbase L, (v_x, v_y, omega) for
 * omni, (omega) for spin-in-place and (v_para) for parallel motion.          */
static void kin_f64(int model, double L, double th, const double* u, double f[3]) {
    double c = cos(th), s = sin(th);
    switch (model) {
    case M_UNICYCLE: f[0] = u[0] * c; f[1] = u[0] * s; f[2] = u[1]; break;
    case M_ACKERMANN: f[0] = u[0] * c; f[1] = u[0] * s; f[2] = u[0] / L * tan(u[1]); break;
    case M_OMNI: f[0] = u[0] * c - u[1] * s; f[1] = u[0] * s + u[1] * c; f[2] = u[2]; break;
    case M_SPIN: f[0] = 0.0; f[1] = 0.0; f[2] = u[0]; break;
    default: f[0] = -u[0] * s; f[1] = u[0] * c; f[2] = 0.0; break;
    }
}

/* Forward-Euler propagation q_{h+1} = q_h + F_m(q_h, u_h) dt (Section
 * "Robot Kinematic Models").  u is T x nu row-major; states receives the
 * (T+1) x 3 states q_0 .. q_T.                                              */
EXPORT void orc_rollout_f64(int model, int T, int nu, double dt, double L,
                            const double* q0, const double* u, double* states) {
    double x = q0[0], y = q0[1], th = q0[2];
    states[0] = x; states[1] = y; states[2] = th;
    for (int h = 0; h < T; ++h) {
        double f[3];
        kin_f64(model, L, th, u + (long)h * nu, f);
        x += f[0] * dt; y += f[1] * dt; th += f[2] * dt;
        states[3 * (h + 1)] = x; states[3 * (h + 1) + 1] = y; states[3 * (h + 1) + 2] = th;
    }
}

/* ======================================================================== */
/* Costs, weights and update (Sections "MPPI Formulation" and "Safety        */
/* Penalties and Trajectory Validation"; Algorithm 1 steps 2-3)              */
/* ======================================================================== */

typedef struct {
    double d_safe, w_coll, w_rep, w_inf, w_goal, goal_x, goal_y, lambda;
    double w_ctrl[3];
    double w_path;
    int n_path;            /* guidance waypoints (0: no path term)          */
    const double* path;    /* x0, y0, x1, y1, ... (planning frame)          */
} orc_cost_params;

/* Obstacle penalty phi_obs(d) = w_coll I(d < 0) + w_rep max(d_safe - d, 0)^2. */
EXPORT double orc_phi_obs(const orc_cost_params* p, double d) {
    double gap = p->d_safe - d;
    if (gap < 0.0) gap = 0.0;
    return (d < 0.0 ? p->w_coll : 0.0) + p->w_rep * gap * gap;
}

/* Distance of (x, y) to the guidance polyline: the smallest distance to one
 * of its segments (one waypoint: the distance to that point).              */
EXPORT double orc_path_dist(const double* path, int n, double x, double y) {
    double best = hypot(x - path[0], y - path[1]);
    for (int k = 1; k < n; ++k) {
        const double* a = path + 2 * k - 2;
        /* a repeated waypoint is a point, not a segment */
        double d = (a[0] == a[2] && a[1] == a[3]) ? hypot(x - a[2], y - a[3])
                                                   : orc_seg_dist(x, y, a[0], a[1], a[2], a[3]);
        if (d < best) best = d;
    }
    return best;
}

/* Task term: distance of the scored position to the goal, weighted by w_goal
 * (the paper names "goal seeking" and "path following"; these are the
 * position-goal reading and the distance to the guidance polyline, weighted
 * by w_path).                                                               */
EXPORT double orc_phi_task(const orc_cost_params* p, double x, double y) {
    double dx = x - p->goal_x, dy = y - p->goal_y;
    double v = p->w_goal * sqrt(dx * dx + dy * dy);
    if (p->n_path > 0) v += p->w_path * orc_path_dist(p->path, p->n_path, x, y);
    return v;
}

/* Control regulariser: sum_c w_ctrl[c] u_c^2 of the sampled control.        */
EXPORT double orc_phi_ctrl(const orc_cost_params* p, const double* u, int nu) {
    double s = 0.0;
    for (int c = 0; c < nu; ++c) s += p->w_ctrl[c] * u[c] * u[c];
    return s;
}

/* Rollout cost J (eq. for J^{(r)}), unsafe flag chi and augmented cost
 * J~ = J + w_inf I(chi) (Algorithm 1 steps 2-3).  Inputs are per rollout r
 * and horizon step h (row-major K x T): the scored positions xy (K x T x 2),
 * the sampled controls u (K x T x nu) and the minimum signed distances dmin. */
EXPORT void orc_costs(const orc_cost_params* p, int K, int T, int nu,
                      const double* xy, const double* u, const double* dmin,
                      double* J, unsigned char* chi, double* Jt) {
    for (int r = 0; r < K; ++r) {
        double acc = 0.0;
        int unsafe = 0;
        for (int h = 0; h < T; ++h) {
            long k = (long)r * T + h;
            double d = dmin[k];
            acc += orc_phi_task(p, xy[2 * k], xy[2 * k + 1]) +
                   orc_phi_ctrl(p, u + k * nu, nu) + orc_phi_obs(p, d);
            if (d < p->d_safe) unsafe = 1;
        }
        J[r] = acc;
        chi[r] = (unsigned char)unsafe;
        Jt[r] = acc + (unsafe ? p->w_inf : 0.0);
    }
}

/* Path-integral weights (eq. for omega^{(r)}): beta = min_r J~, then
 * omega_r = exp(-(J~_r - beta)/lambda) / sum_j exp(-(J~_j - beta)/lambda).  */
EXPORT void orc_weights(int K, const double* Jt, double lambda, double* w) {
    double beta = INFINITY;
    for (int r = 0; r < K; ++r) if (Jt[r] < beta) beta = Jt[r];
    double z = 0.0;
    for (int r = 0; r < K; ++r) { w[r] = exp(-(Jt[r] - beta) / lambda); z += w[r]; }
    for (int r = 0; r < K; ++r) w[r] /= z;
}

/* Nominal update u_h <- u_h + sum_r omega_r eps_h^{(r)} (eq. after the
 * weights; Algorithm 1 step 3).  eps is K x T x nu, U is T x nu (in place). */
EXPORT void orc_update(int K, int T, int nu, const double* w, const double* eps, double* U) {
    for (int h = 0; h < T; ++h)
        for (int c = 0; c < nu; ++c) {
            double s = 0.0;
            for (int r = 0; r < K; ++r) s += w[r] * eps[((long)r * T + h) * nu + c];
            U[h * nu + c] += s;
        }
}

/* Validation and execution (Algorithm 1 step 4): the nominal is valid when
 * every d_h^{min,nom} >= d_safe.  A nominal with a non-finite control has no
 * defined trajectory (its states, hence its distances, are not numbers), so
 * it is never valid.  Valid: u* = U_0 and U is shifted forward (the last
 * entry is repeated).  Invalid: u* = 0 and U is reset to zero.  Returns 1
 * when valid.                                                               */
EXPORT int orc_validate_shift(int T, int nu, const double* dnom, double d_safe,
                              double* U, double* u_star) {
    int ok = 1;
    for (int h = 0; h < T; ++h) if (!(dnom[h] >= d_safe)) ok = 0;
    for (int k = 0; k < T * nu; ++k) if (!isfinite(U[k])) ok = 0;
    if (ok) {
        for (int c = 0; c < nu; ++c) u_star[c] = U[c];
        for (int h = 0; h + 1 < T; ++h)
            for (int c = 0; c < nu; ++c) U[h * nu + c] = U[(h + 1) * nu + c];
    } else {
        for (int c = 0; c < nu; ++c) u_star[c] = 0.0;
        for (int k = 0; k < T * nu; ++k) U[k] = 0.0;
    }
    return ok;
}

/* ======================================================================== */
/* Counter-based random numbers: Philox4x64-10                              */
/* (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2,   */
/* 3", SC'11).  Ten rounds of the 4x64 S-box with the published multipliers  */
/* and Weyl key increments; integer-only, hence bit-exact on any machine.    */
/* ======================================================================== */

#define PHILOX_M0 0xD2E7470EE14C6C93ULL
#define PHILOX_M1 0xCA5A826395121157ULL
#define PHILOX_W0 0x9E3779B97F4A7C15ULL /* golden ratio */
#define PHILOX_W1 0xBB67AE8584CAA73BULL /* sqrt(3) - 1  */

EXPORT void orc_philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4]) {
    uint64_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += PHILOX_W0; k1 += PHILOX_W1; }
        unsigned __int128 p0 = (unsigned __int128)PHILOX_M0 * x0;
        unsigned __int128 p1 = (unsigned __int128)PHILOX_M1 * x2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t y0 = hi1 ^ x1 ^ k0;
        uint64_t y1 = lo1;
        uint64_t y2 = hi0 ^ x3 ^ k1;
        uint64_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* ======================================================================== */
/* FP32 mirror: one fixed single-precision operation sequence for the noise  */
/* and the rollout.  Every + - * / sqrt below is one correctly rounded IEEE  */
/* binary32 operation and every fmaf() one fused multiply-add; no other      */
/* library function is used.                                                 */
/* ======================================================================== */

/* Cody-Waite split of pi/2 into three floats (A = nearest float to pi/2,
 * B = nearest float to pi/2 - A, C = nearest float to pi/2 - A - B).        */
static const float kPio2A = 0x1.921fb6p+0f;
static const float kPio2B = -0x1.777a5cp-25f;
static const float kPio2C = -0x1.ee59dap-50f;
static const float kTwoOverPi = 0x1.45f306p-1f;  /* nearest float to 2/pi */
static const float kTwoPi = 0x1.921fb6p+2f;      /* nearest float to 2 pi */
/* Taylor coefficients (-1)^k / (2k+1)! and (-1)^k / (2k)!, rounded to float. */
static const float kS3 = -0x1.555556p-3f, kS5 = 0x1.111112p-7f, kS7 = -0x1.a01a02p-13f,
                   kS9 = 0x1.71de3ap-19f;
static const float kC2 = -0x1.0p-1f, kC4 = 0x1.555556p-5f, kC6 = -0x1.6c16c2p-10f,
                   kC8 = 0x1.a01a02p-16f, kC10 = -0x1.27e4fcp-22f;
/* ln 2 = kLn2Hi + kLn2Lo, kLn2Hi with 16 significant bits; 1/(2k+1) for the
 * atanh series; sqrt(2) rounded to float.                                   */
static const float kLn2Hi = 0x1.62e4p-1f, kLn2Lo = 0x1.7f7d1cp-20f;
static const float kInv3 = 0x1.555556p-2f, kInv5 = 0x1.99999ap-3f, kInv7 = 0x1.24924ap-3f,
                   kInv9 = 0x1.c71c72p-4f;
static const float kSqrt2 = 0x1.6a09e6p+0f;

static uint32_t f2u(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }
static float u2f(uint32_t u) { float f; memcpy(&f, &u, 4); return f; }

/* sin and cos: quadrant k = rint(x * 2/pi), residual r = x - k pi/2 by three
 * fused steps, Taylor polynomials of degree 9 (sin) and 10 (cos) on
 * |r| <= pi/4 in Horner form, quadrant rotation.                            */
EXPORT void orc_f32_sincos(float x, float* s_out, float* c_out) {
    float k = rintf(x * kTwoOverPi);
    float r = fmaf(-k, kPio2A, x);
    r = fmaf(-k, kPio2B, r);
    r = fmaf(-k, kPio2C, r);
    float r2 = r * r;
    float ps = fmaf(r2, kS9, kS7);
    ps = fmaf(r2, ps, kS5);
    ps = fmaf(r2, ps, kS3);
    float sn = fmaf(r * r2, ps, r);
    float pc = fmaf(r2, kC10, kC8);
    pc = fmaf(r2, pc, kC6);
    pc = fmaf(r2, pc, kC4);
    pc = fmaf(r2, pc, kC2);
    float cs = fmaf(r2, pc, 1.0f);
    int q = ((int)k) & 3;
    float s, c;
    if (q == 0) { s = sn; c = cs; }
    else if (q == 1) { s = cs; c = -sn; }
    else if (q == 2) { s = -sn; c = -cs; }
    else { s = -cs; c = sn; }
    *s_out = s; *c_out = c;
}

/* Natural log of a positive normal float: x = m 2^e with m in [sqrt(2)/2,
 * sqrt(2)), log x = e ln2 + 2 atanh(s), s = (m - 1)/(m + 1), atanh series to
 * s^9.                                                                       */
EXPORT float orc_f32_log(float x) {
    uint32_t b = f2u(x);
    int e = (int)((b >> 23) & 0xffu) - 127;
    float m = u2f((b & 0x7fffffu) | 0x3f800000u);
    if (m > kSqrt2) { m = m * 0.5f; e += 1; }
    float f = m - 1.0f;
    float s = f / (m + 1.0f);
    float z = s * s;
    float p = fmaf(z, kInv9, kInv7);
    p = fmaf(z, p, kInv5);
    p = fmaf(z, p, kInv3);
    float a = fmaf(s * z, p, s);
    float lnm = a + a;
    float fe = (float)e;
    return fmaf(fe, kLn2Hi, fmaf(fe, kLn2Lo, lnm));
}

EXPORT float orc_f32_tan(float x) {
    float s, c;
    orc_f32_sincos(x, &s, &c);
    return s / c;
}

/* Uniform in (0,1) from the top 23 bits of a 64-bit word: (2 j + 1) 2^-24,
 * exact in binary32.                                                        */
static float word_to_uniform(uint64_t w) {
    uint32_t j = (uint32_t)(w >> 41);
    return (float)(2u * j + 1u) * 0x1.0p-24f;
}

/* Four standard normals for (seed, step, rollout r, horizon step h, stream):
 * Philox4x64-10 with counter (h, r, step, stream) and key (seed, 0); words
 * (w0, w1) and (w2, w3) each give one Box-Muller pair
 * z = sqrt(-2 log u1) (cos(2 pi u2), sin(2 pi u2)).                         */
EXPORT void orc_f32_normals(uint64_t seed, uint64_t step, uint32_t r, uint32_t h,
                            uint64_t stream, float z[4]) {
    uint64_t ctr[4] = {h, r, step, stream}, key[2] = {seed, 0}, w[4];
    orc_philox4x64_10(ctr, key, w);
    for (int p = 0; p < 2; ++p) {
        float u1 = word_to_uniform(w[2 * p]), u2 = word_to_uniform(w[2 * p + 1]);
        float rad = sqrtf(-2.0f * orc_f32_log(u1));
        float s, c;
        orc_f32_sincos(kTwoPi * u2, &s, &c);
        z[2 * p] = rad * c;
        z[2 * p + 1] = rad * s;
    }
}

/* One forward-Euler step of the FP32 sequence with (s, c) = sincos(theta_h):
 *   unicycle   x += (v c) dt, y += (v s) dt, theta += w dt
 *   ackermann  same x, y; theta += ((v tan(delta)) / L) dt
 *   omni       x += fma(vx, c, -(vy s)) dt, y += fma(vx, s, vy c) dt, theta += w dt
 *   spin       theta += w dt
 *   parallel   x += (-(v s)) dt, y += (v c) dt
 * each "a += b dt" being fmaf(b, dt, a).                                    */
static void euler_f32(int model, const float* u, float dt, float L, float s, float c,
                      float* x, float* y, float* th) {
    switch (model) {
    case M_UNICYCLE:
        *x = fmaf(u[0] * c, dt, *x); *y = fmaf(u[0] * s, dt, *y); *th = fmaf(u[1], dt, *th);
        break;
    case M_ACKERMANN: {
        float w = (u[0] * orc_f32_tan(u[1])) / L;
        *x = fmaf(u[0] * c, dt, *x); *y = fmaf(u[0] * s, dt, *y); *th = fmaf(w, dt, *th);
        break;
    }
    case M_OMNI: {
        float xd = fmaf(u[0], c, -(u[1] * s));
        float yd = fmaf(u[0], s, u[1] * c);
        *x = fmaf(xd, dt, *x); *y = fmaf(yd, dt, *y); *th = fmaf(u[2], dt, *th);
        break;
    }
    case M_SPIN:
        *th = fmaf(u[0], dt, *th);
        break;
    default:
        *x = fmaf(-(u[0] * s), dt, *x); *y = fmaf(u[0] * c, dt, *y);
        break;
    }
}

static void put_pose(float* dst, float x, float y, float c, float s) {
    dst[0] = x; dst[1] = y; dst[2] = c; dst[3] = s;
}

/* Sampling and rollout in the FP32 sequence (Algorithm 1 step 1):
 *   eps_c = sigma_c z_c; u = min(max(U_h + eps, u_min), u_max) (the sampled
 *   control is kept inside the actuator box); eps_eff = u - U_h; then one
 *   Euler step (euler_f32) and (s, c) = sincos(theta_{h+1}).
 * Scored pose of (r, h): the post-step state q_{h+1} when state_offset == 1,
 * the pre-step state q_h when 0.  Outputs are row-major K x T:
 * poses (x, y, cos, sin), eps_eff and u (each x nu).                       */
EXPORT void orc_rollout_f32(int model, int K, int T, int nu, float dt, float L,
                            const float q0[3], const float* U, const float* sigma,
                            const float* umin, const float* umax, uint64_t seed,
                            uint64_t step, uint64_t stream, int state_offset,
                            float* poses, float* eps_eff, float* usamp) {
    for (int r = 0; r < K; ++r) {
        float x = q0[0], y = q0[1], th = q0[2], s, c;
        orc_f32_sincos(th, &s, &c);
        for (int h = 0; h < T; ++h) {
            long k = (long)r * T + h;
            float z[4], u[3];
            orc_f32_normals(seed, step, (uint32_t)r, (uint32_t)h, stream, z);
            for (int ch = 0; ch < nu; ++ch) {
                float base = U[h * nu + ch];
                float v = base + sigma[ch] * z[ch];
                v = fmaxf(v, umin[ch]);
                v = fminf(v, umax[ch]);
                u[ch] = v;
                eps_eff[k * nu + ch] = v - base;
                usamp[k * nu + ch] = v;
            }
            if (!state_offset) put_pose(poses + 4 * k, x, y, c, s);
            euler_f32(model, u, dt, L, s, c, &x, &y, &th);
            orc_f32_sincos(th, &s, &c);
            if (state_offset) put_pose(poses + 4 * k, x, y, c, s);
        }
    }
}

/* Deterministic rollout of one control sequence in the same FP32 sequence
 * (the nominal trajectory of Algorithm 1 step 4).  poses: T x 4.            */
EXPORT void orc_rollout_nominal_f32(int model, int T, int nu, float dt, float L,
                                    const float q0[3], const float* U, int state_offset,
                                    float* poses) {
    float x = q0[0], y = q0[1], th = q0[2], s, c;
    orc_f32_sincos(th, &s, &c);
    for (int h = 0; h < T; ++h) {
        if (!state_offset) put_pose(poses + 4 * h, x, y, c, s);
        euler_f32(model, U + h * nu, dt, L, s, c, &x, &y, &th);
        orc_f32_sincos(th, &s, &c);
        if (state_offset) put_pose(poses + 4 * h, x, y, c, s);
    }
}

/* Normals for rollouts r = 0..n-1 at one (seed, step, h, stream): 4n floats. */
EXPORT void orc_f32_normals_batch(uint64_t seed, uint64_t step, uint32_t h, uint64_t stream,
                                  long n, float* z) {
    for (long r = 0; r < n; ++r) orc_f32_normals(seed, step, (uint32_t)r, h, stream, z + 4 * r);
}

#ifdef _OPENMP
#include <omp.h>
#endif
/* Number of threads the OpenMP loops above use. */
EXPORT int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Set the number of threads of the OpenMP loops above (n >= 1). */
EXPORT void orc_set_num_threads(int n) {
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}

/* ======================================================================== */
/* Features of the learned proposal in the FP32 sequence (not part of the   */
/* paper's method).  Every operation is one correctly rounded binary32      */
/* operation, so the result is reproducible bit for bit:                    */
/*   robot frame: (s, c) = sincos(theta0); d = o - q0; x = c dx + s dy,     */
/*     y = c dy - s dx;                                                     */
/*   bin: quadrant q and pseudo-angle t in [0, 1] (y/(x+y), -x/(y-x),       */
/*     -y/(-x-y), x/(x-y) for q = 0..3; the origin has t = 0),              */
/*     bin = 16 q + min(15, floor(16 t));                                   */
/*   value: min over the bin of min(sqrt(x x + y y), r_max), / r_max;       */
/*     empty bins are r_max / r_max = 1;                                    */
/*   goal (g - q0) rotated the same way, / r_max;                           */
/*   previous controls (u - mid) / half per channel (0 when half = 0).      */
/* ======================================================================== */
EXPORT void orc_f32_features(const float* px, const float* py, const unsigned char* valid, long n,
                             const float q0[3], const float goal[2], const float* U_prev, int T,
                             int nu, const float* umin, const float* umax, float r_max, float* out) {
    float hist[64];
    for (int b = 0; b < 64; ++b) hist[b] = r_max;
    float s, c;
    orc_f32_sincos(q0[2], &s, &c);
    for (long i = 0; i < n; ++i) {
        if (valid && !valid[i]) continue;
        if (!isfinite(px[i]) || !isfinite(py[i])) continue;
        float dx = px[i] - q0[0], dy = py[i] - q0[1];
        float x = c * dx + s * dy;
        float y = c * dy - s * dx;
        int q;
        float t;
        if (y >= 0.0f) {
            if (x >= 0.0f) { q = 0; t = (x == 0.0f && y == 0.0f) ? 0.0f : y / (x + y); }
            else { q = 1; t = -x / (y - x); }
        } else {
            if (x < 0.0f) { q = 2; t = -y / (-x - y); }
            else { q = 3; t = x / (x - y); }
        }
        int k = (int)(t * 16.0f);
        if (k > 15) k = 15;
        int bin = q * 16 + k;
        float r = sqrtf(x * x + y * y);
        if (r > r_max) r = r_max;
        if (r < hist[bin]) hist[bin] = r;
    }
    for (int b = 0; b < 64; ++b) out[b] = hist[b] / r_max;
    float gx = goal[0] - q0[0], gy = goal[1] - q0[1];
    out[64] = (c * gx + s * gy) / r_max;
    out[65] = (c * gy - s * gx) / r_max;
    for (int k = 0; k < T * nu; ++k) {
        int ch = k % nu;
        float mid = (umax[ch] + umin[ch]) * 0.5f;
        float half = (umax[ch] - umin[ch]) * 0.5f;
        out[66 + k] = half > 0.0f ? (U_prev[k] - mid) / half : 0.0f;
    }
}
