// Host-side set-up helpers: face matching and the product quadrature.
#include <algorithm>
#include <array>
#include <cmath>
#include <unordered_map>

#include "snx_internal.h"

namespace snx {

namespace {

// Local vertices of face f = 2*axis + side, in increasing local index.
std::array<int, 4> face_vertices(int f) {
    std::array<int, 4> out{};
    int axis = f >> 1, side = f & 1, k = 0;
    for (int j = 0; j < 8; ++j)
        if (((j >> axis) & 1) == side) out[k++] = j;
    return out;
}

struct Key {
    std::array<int, 4> v;
    bool operator==(const Key &o) const { return v == o.v; }
};
struct KeyHash {
    size_t operator()(const Key &k) const {
        uint64_t h = 1469598103934665603ull;
        for (int x : k.v) { h ^= (uint32_t)x; h *= 1099511628211ull; }
        return (size_t)h;
    }
};

}  // namespace

// Matches every cell face with the face of another cell that has the same
// four vertices (the elem_neighbors / face_nodes arrays of Table 1).  A face
// met by more than two cells is a mesh error; an unmatched face is boundary.
int topology(int C, int nvert, const int *cell_vert, std::vector<int> &nbr, std::vector<int> &nbr_face,
             std::vector<unsigned> &perm, std::string &err) {
    nbr.assign((size_t)C * 6, -1);
    nbr_face.assign((size_t)C * 6, -1);
    perm.assign((size_t)C * 6, 0u);
    std::unordered_map<Key, int, KeyHash> first;   // key -> cell*6+face of its first owner
    first.reserve((size_t)C * 4);
    for (int K = 0; K < C; ++K) {
        for (int f = 0; f < 6; ++f) {
            auto fv = face_vertices(f);
            Key key;
            for (int k = 0; k < 4; ++k) {
                int v = cell_vert[(size_t)K * 8 + fv[k]];
                if (v < 0 || v >= nvert) { err = "vertex id out of range"; return SNX_E_ARG; }
                key.v[k] = v;
            }
            std::sort(key.v.begin(), key.v.end());
            if (key.v[0] == key.v[1] || key.v[1] == key.v[2] || key.v[2] == key.v[3]) {
                err = "degenerate face (repeated vertex)";
                return SNX_E_MESH;
            }
            auto it = first.find(key);
            if (it == first.end()) {
                first.emplace(key, K * 6 + f);
                continue;
            }
            int other = it->second;
            if (other < 0) { err = "face shared by more than two cells"; return SNX_E_MESH; }
            int N = other / 6, g = other % 6;
            if (N == K) { err = "cell glued to itself"; return SNX_E_MESH; }
            nbr[(size_t)K * 6 + f] = N; nbr_face[(size_t)K * 6 + f] = g;
            nbr[(size_t)N * 6 + g] = K; nbr_face[(size_t)N * 6 + g] = f;
            it->second = -1;   // a third occurrence is an error
        }
    }
    for (int K = 0; K < C; ++K) {
        for (int f = 0; f < 6; ++f) {
            int N = nbr[(size_t)K * 6 + f];
            if (N < 0) continue;
            auto fv = face_vertices(f);
            unsigned packed = 0;
            for (int k = 0; k < 4; ++k) {
                int v = cell_vert[(size_t)K * 8 + fv[k]];
                int found = -1;
                for (int j = 0; j < 8; ++j)
                    if (cell_vert[(size_t)N * 8 + j] == v) found = j;
                if (found < 0) { err = "matched face vertices disagree"; return SNX_E_MESH; }
                packed |= (unsigned)found << (8 * k);
            }
            perm[(size_t)K * 6 + f] = packed;
        }
    }
    return SNX_OK;
}

// Product quadrature: positive nodes of the 2*npolar-point Gauss-Legendre rule
// (roots of P_m by Newton's method, weights 2 / ((1 - x^2) P_m'(x)^2)) times
// nazim equal azimuthal intervals per octant.
int product_quadrature(int npolar, int nazim, double *omega, double *w) {
    if (npolar < 1 || nazim < 1 || npolar > 32 || nazim > 64 || !omega || !w) return SNX_E_ARG;
    const int m = 2 * npolar;
    const double pi = 3.14159265358979323846;
    std::vector<double> mu(npolar), wmu(npolar);
    for (int i = 0; i < npolar; ++i) {
        // the i-th positive root, counted from the largest, starts near cos(pi (i + 3/4) / (m + 1/2))
        double x = std::cos(pi * (i + 0.75) / (m + 0.5));
        double dP = 1.0;
        for (int it = 0; it < 64; ++it) {
            double Pkm1 = 1.0, Pk = x;   // P_0, P_1
            for (int k = 1; k < m; ++k) {
                double Pkp1 = ((2 * k + 1) * x * Pk - k * Pkm1) / (k + 1);
                Pkm1 = Pk;
                Pk = Pkp1;
            }
            dP = m * (x * Pk - Pkm1) / (x * x - 1.0);
            double step = Pk / dP;
            x -= step;
            if (std::fabs(step) <= 1e-16 * std::fabs(x)) break;
        }
        double Pkm1 = 1.0, Pk = x;
        for (int k = 1; k < m; ++k) {
            double Pkp1 = ((2 * k + 1) * x * Pk - k * Pkm1) / (k + 1);
            Pkm1 = Pk;
            Pk = Pkp1;
        }
        dP = m * (x * Pk - Pkm1) / (x * x - 1.0);
        mu[npolar - 1 - i] = x;                  // ascending
        wmu[npolar - 1 - i] = 2.0 / ((1.0 - x * x) * dP * dP);
    }
    const int per = npolar * nazim;
    for (int o = 0; o < 8; ++o) {
        double sx = (o & 1) ? -1.0 : 1.0, sy = (o & 2) ? -1.0 : 1.0, sz = (o & 4) ? -1.0 : 1.0;
        for (int k = 0; k < npolar; ++k) {
            double sinth = std::sqrt(1.0 - mu[k] * mu[k]);
            for (int j = 0; j < nazim; ++j) {
                double phi = (j + 0.5) * (0.5 * pi) / nazim;
                size_t n = (size_t)o * per + (size_t)k * nazim + j;
                omega[3 * n + 0] = sx * sinth * std::cos(phi);
                omega[3 * n + 1] = sy * sinth * std::sin(phi);
                omega[3 * n + 2] = sz * mu[k];
                w[n] = wmu[k] * (0.5 * pi) / nazim;
            }
        }
    }
    return SNX_OK;
}

}  // namespace snx
