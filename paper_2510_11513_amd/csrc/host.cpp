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

namespace snx {

// Per-direction sweep order (SNX_DESIGNATION_DIRECTION), direction by direction:
//  1. the strongly connected components of the direction's dependency graph
//     (cell K depends on its neighbour across each inflow face), by Tarjan's
//     algorithm with an explicit stack;
//  2. inside a component, the inflow faces whose upwind cell is ranked after
//     the cell (larger Omega . centroid, the centroid being the mean of the
//     eight vertices; the larger cell id on a tie) are lagged;
//  3. the levels of the remaining acyclic graph: a cell's level is one more
//     than the highest level of the upwind cells it still waits for (Kahn's
//     algorithm from the cells without any).
// Then the work items: for every (octant, cell) one item per distinct level
// among the octant's directions, holding those directions, bucketed by level.
int direction_orders(int C, int A, const std::vector<int> &nbr, const std::vector<int> &nbr_face,
                     const std::vector<unsigned char> &amask, const std::vector<double> &xyz,
                     const std::vector<int> &cell_vert, const std::vector<double> &omega, DirHost &out,
                     std::string &err) {
    std::vector<std::array<double, 3>> cen((size_t)C);
    for (int K = 0; K < C; ++K) {
        double c[3] = {0.0, 0.0, 0.0};
        for (int j = 0; j < 8; ++j)
            for (int d = 0; d < 3; ++d) c[d] += xyz[3 * (size_t)cell_vert[(size_t)K * 8 + j] + d] / 8.0;
        cen[K] = {c[0], c[1], c[2]};
    }
    const size_t OCA = (size_t)8 * C * A;
    out.lagbits.assign(OCA, 0);
    out.lagidx.assign(OCA, 0);
    out.lag.clear();
    out.cyclic_directions = 0;
    std::vector<int> level((size_t)A * C);                 // levels of the current octant's directions
    std::vector<int> index(C), low(C), comp(C), onstack(C), stack, todo, waits(C), queue(C);
    std::vector<double> rank(C);
    std::vector<std::vector<std::pair<int, unsigned long long>>> buckets;   // per level: (task, directions)
    for (int o = 0; o < 8; ++o) {
        for (int a = 0; a < A; ++a) {
            const int n = o * A + a;
            const double *om = &omega[3 * (size_t)n];
            auto in = [&](int K) { return (int)amask[((size_t)o * C + K) * A + a]; };
            for (int K = 0; K < C; ++K) {
                rank[K] = om[0] * cen[K][0] + om[1] * cen[K][1] + om[2] * cen[K][2];
                index[K] = -1;
                onstack[K] = 0;
            }
            // 1. Tarjan: todo holds (cell, next face) frames of the depth-first search
            int next = 0, ncomp = 0;
            bool cyclic = false;
            for (int root = 0; root < C; ++root) {
                if (index[root] >= 0) continue;
                todo.assign({root, 0});
                index[root] = low[root] = next++;
                stack.push_back(root);
                onstack[root] = 1;
                while (!todo.empty()) {
                    const int v = todo[todo.size() - 2];
                    int &fi = todo.back();
                    if (fi < 6) {
                        const int f = fi++;
                        const int w = nbr[(size_t)v * 6 + f];
                        if (w < 0 || ((in(v) >> f) & 1)) continue;       // successors: across outflow faces
                        if (index[w] < 0) {
                            index[w] = low[w] = next++;
                            stack.push_back(w);
                            onstack[w] = 1;
                            todo.push_back(w);
                            todo.push_back(0);
                        } else if (onstack[w]) {
                            low[v] = std::min(low[v], index[w]);
                        }
                    } else {
                        todo.resize(todo.size() - 2);
                        if (low[v] == index[v]) {
                            int w, size = 0;
                            do {
                                w = stack.back();
                                stack.pop_back();
                                onstack[w] = 0;
                                comp[w] = ncomp;
                                ++size;
                            } while (w != v);
                            cyclic = cyclic || size > 1;
                            ++ncomp;
                        }
                        if (!todo.empty()) {
                            const int u = todo[todo.size() - 2];
                            low[u] = std::min(low[u], low[v]);
                        }
                    }
                }
            }
            out.cyclic_directions += cyclic;
            // 2. lagged faces and 3. levels
            for (int K = 0; K < C; ++K) {
                int lag = 0, wait = 0;
                for (int f = 0; f < 6; ++f) {
                    const int N = nbr[(size_t)K * 6 + f];
                    if (N < 0 || !((in(K) >> f) & 1)) continue;
                    const bool after = rank[N] > rank[K] || (rank[N] == rank[K] && N > K);
                    if (comp[N] == comp[K] && after) lag |= 1 << f;
                    else ++wait;
                }
                waits[K] = wait;
                const size_t oka = ((size_t)o * C + K) * A + a;
                out.lagbits[oka] = (unsigned char)lag;
                out.lagidx[oka] = (int)out.lag.size();
                for (int f = 0; f < 6; ++f)
                    if ((lag >> f) & 1) out.lag.push_back({o, K, a, f});
            }
            int head = 0, tail = 0;
            int *lev = &level[(size_t)a * C];
            for (int K = 0; K < C; ++K) {
                lev[K] = 0;
                if (!waits[K]) queue[tail++] = K;
            }
            while (head < tail) {
                const int v = queue[head++];
                for (int f = 0; f < 6; ++f) {
                    const int w = nbr[(size_t)v * 6 + f];
                    if (w < 0 || ((in(v) >> f) & 1)) continue;
                    if ((out.lagbits[((size_t)o * C + w) * A + a] >> nbr_face[(size_t)v * 6 + f]) & 1) continue;
                    lev[w] = std::max(lev[w], lev[v] + 1);
                    if (--waits[w] == 0) queue[tail++] = w;
                }
            }
            if (tail != C) {
                err = "a cycle is left after lagging (inconsistent face designation)";
                return SNX_E_CYCLE;
            }
        }
        // work items of this octant: one per (cell, distinct level of its directions)
        for (int K = 0; K < C; ++K) {
            unsigned long long left = A >= 64 ? ~0ull : ((1ull << A) - 1);
            while (left) {
                const int a0 = __builtin_ctzll(left);
                const int l0 = level[(size_t)a0 * C + K];
                unsigned long long dirs = 0;
                for (int a = a0; a < A; ++a)
                    if (((left >> a) & 1) && level[(size_t)a * C + K] == l0) dirs |= 1ull << a;
                left &= ~dirs;
                if ((int)buckets.size() <= l0) buckets.resize(l0 + 1);
                buckets[l0].push_back({8 * K + o, dirs});
            }
        }
    }
    out.items.clear();
    out.dirs.clear();
    out.level_off.assign(1, 0);
    for (const auto &bk : buckets) {
        for (const auto &it : bk) {
            out.items.push_back(it.first);
            out.dirs.push_back(it.second);
        }
        out.level_off.push_back((long long)out.items.size());
    }
    return SNX_OK;
}

}  // namespace snx
