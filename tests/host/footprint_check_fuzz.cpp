// Fuzz of the library's host-side footprint check (polygon_defect) for the
// address and undefined-behaviour sanitizers: random star-shaped polygons
// (simple by construction) must pass, and so must their reversal and cyclic
// shifts; random vertex orders, bow-ties, repeated and non-finite vertices,
// fold-backs and near-zero areas exercise every rejection path.  Prints the
// number of cases and exits non-zero on a violated expectation.
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "../../paper_2605_29663_amd/csrc/host_geom.hpp"

using emppi_host::polygon_defect;

static int check(const std::vector<double>& v, int B) {
    char msg[160];
    return polygon_defect(v, B, msg, sizeof msg);
}

int main() {
    std::mt19937_64 rng(12345);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    long cases = 0;
    int bad = 0;
    for (int it = 0; it < 20000; ++it) {
        const int B = 3 + static_cast<int>(U(rng) * 62);
        // star-shaped: sorted distinct angles, positive radii
        std::vector<double> ang(B);
        for (int k = 0; k < B; ++k) ang[k] = (k + 0.1 + 0.8 * U(rng)) * 2.0 * M_PI / B;
        std::vector<double> v(2 * B);
        for (int k = 0; k < B; ++k) {
            const double r = 0.3 + U(rng);
            v[2 * k] = r * std::cos(ang[k]);
            v[2 * k + 1] = r * std::sin(ang[k]);
        }
        if (check(v, B) != 0) ++bad;
        std::vector<double> rev(2 * B), sh(2 * B);
        const int s = static_cast<int>(U(rng) * B);
        for (int k = 0; k < B; ++k) {
            rev[2 * k] = v[2 * (B - 1 - k)];
            rev[2 * k + 1] = v[2 * (B - 1 - k) + 1];
            sh[2 * k] = v[2 * ((k + s) % B)];
            sh[2 * k + 1] = v[2 * ((k + s) % B) + 1];
        }
        if (check(rev, B) != 0 || check(sh, B) != 0) ++bad;
        // a random vertex order (usually self-intersecting): any answer, no fault
        std::vector<double> w(2 * B);
        for (int k = 0; k < 2 * B; ++k) w[k] = U(rng) * 2.0 - 1.0;
        (void)check(w, B);
        // a repeated vertex, a non-finite one, a fold-back
        std::vector<double> d = v;
        const int k = static_cast<int>(U(rng) * B);
        d[2 * ((k + 1) % B)] = d[2 * k];
        d[2 * ((k + 1) % B) + 1] = d[2 * k + 1];
        if (check(d, B) == 0) ++bad;
        d = v;
        d[2 * k + (it & 1)] = (it & 2) ? NAN : INFINITY;
        if (check(d, B) == 0) ++bad;
        cases += 6;
    }
    // fixed cases: bow-tie, zero area, fold-back onto the previous edge, too few
    const std::vector<double> bow{0, 0, 1, 1, 1, 0, 0, 1};
    const std::vector<double> flat{0, 0, 1, 0, 2, 0};
    const std::vector<double> fold{0, 0, 2, 0, 1, 0, 1, 1};
    const std::vector<double> two{0, 0, 1, 0};
    if (check(bow, 4) == 0 || check(flat, 3) == 0 || check(fold, 4) == 0 || check(two, 2) == 0) ++bad;
    cases += 4;
    std::printf("cases %ld violations %d\n", cases, bad);
    return bad ? 1 : 0;
}
