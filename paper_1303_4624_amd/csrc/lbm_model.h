// lbm_model.h - compile-time velocity sets of the 2D 33-velocity (Table 2) and
// 3D 95-velocity (Table 3) on-lattice models of 4th-order accuracy, and of
// the lower-order 3D 19- and 15-velocity sets the paper says the same
// construction yields (paragraph after Formula (10)), shared by the host
// validation code and the HIP kernels of this library.
//
// A model is a list of symmetry groups, each given by an integer
// representative; the group is the orbit of the representative under
// coordinate permutations and sign changes (G_1, G_4, G_8 in 2D and G_1, G_6,
// G_8, G_12, G_24, G_48 in 3D).  The velocities of a group share one weight.
// Canonical order: groups in table order, inside a group ascending integer
// tuples (e_x, e_y[, e_z]).
#pragma once

#include <cstdint>

namespace lbm {

enum class ModelId : int { D2Q33 = 0, D3Q95 = 1, D3Q19 = 2, D3Q15 = 3 };
enum class Prec : int { F64 = 0, F32S = 1 };

struct GroupRep {
    int order;      // number of velocities in the group (table column "group")
    int r[3];       // representative, unused trailing components are 0
};

// Table 2: D2Q33.
inline constexpr GroupRep kD2Q33Reps[8] = {
    {1, {0, 0, 0}}, {4, {1, 0, 0}}, {4, {1, 1, 0}}, {4, {2, 0, 0}},
    {4, {2, 2, 0}}, {4, {3, 0, 0}}, {8, {2, 1, 0}}, {4, {4, 4, 0}}};
inline constexpr double kD2Q33PrintedW[8] = {.161987, .143204, .0338840, .00556112,
                                             8.44799e-5, .00113254, .0128169, 3.45552e-6};
inline constexpr double kD2Q33PrintedC = .819381;

// Table 3: D3Q95.
inline constexpr GroupRep kD3Q95Reps[10] = {
    {1, {0, 0, 0}}, {6, {2, 0, 0}}, {12, {2, 2, 0}}, {8, {2, 2, 2}}, {6, {3, 0, 0}},
    {12, {3, 3, 0}}, {8, {3, 3, 3}}, {24, {2, 2, 5}}, {12, {4, 4, 0}}, {6, {5, 0, 0}}};
inline constexpr double kD3Q95PrintedW[10] = {.206847, .00442257, .0333341, .0128902, .0287920,
                                              .00264319, .000927908, .00106078, .000804376,
                                              .00274697};
inline constexpr double kD3Q95PrintedC = .421803;

// Lower-order 3D sets (order of accuracy m = 2: Formula (5) up to n_max = 4,
// Omega(2, 3) = 4 equations for three group weights and c, Formula (10)).
// The paper names them without tables; their weights are solved on the host
// from a generic start (least squares at c = 1, then Newton).
inline constexpr GroupRep kD3Q19Reps[3] = {{1, {0, 0, 0}}, {6, {1, 0, 0}}, {12, {1, 1, 0}}};
inline constexpr GroupRep kD3Q15Reps[3] = {{1, {0, 0, 0}}, {6, {1, 0, 0}}, {8, {1, 1, 1}}};

template <int D_, int Q_, int G_>
struct VelocityTable {
    static constexpr int D = D_;
    static constexpr int Q = Q_;
    static constexpr int G = G_;
    int e[Q_][3];       // displacement, trailing components 0
    int group[Q_];      // group of each velocity
    int gstart[G_];     // first velocity of each group
    int gsize[G_];
    int e2[G_];         // |e|^2 of the group
    int opp[Q_];        // index of the opposite velocity -e_i
    int emax;           // largest |component|
    bool ok;            // orbit sizes matched the declared group orders
};

namespace detail {

constexpr bool less_tuple(const int* a, const int* b, int D) {
    for (int k = 0; k < D; ++k) {
        if (a[k] != b[k]) return a[k] < b[k];
    }
    return false;
}

constexpr bool equal_tuple(const int* a, const int* b, int D) {
    for (int k = 0; k < D; ++k)
        if (a[k] != b[k]) return false;
    return true;
}

}  // namespace detail

template <int D, int Q, int G>
constexpr VelocityTable<D, Q, G> make_table(const GroupRep (&reps)[G]) {
    VelocityTable<D, Q, G> t{};
    t.ok = true;
    int q = 0;
    int perms[6][3] = {};
    int np = 0;
    for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b)
            for (int c = 0; c < (D == 3 ? D : 1); ++c) {
                if (a == b) continue;
                if (D == 3 && (c == a || c == b)) continue;
                perms[np][0] = a;
                perms[np][1] = b;
                perms[np][2] = (D == 3) ? c : 0;
                ++np;
            }
    for (int g = 0; g < G; ++g) {
        int cand[48][3] = {};
        int nc = 0;
        for (int p = 0; p < np; ++p) {
            for (int s = 0; s < (1 << D); ++s) {
                int v[3] = {0, 0, 0};
                for (int k = 0; k < D; ++k) {
                    int comp = reps[g].r[perms[p][k]];
                    v[k] = ((s >> k) & 1) ? -comp : comp;
                }
                bool dup = false;
                for (int j = 0; j < nc; ++j)
                    if (detail::equal_tuple(cand[j], v, D)) dup = true;
                if (!dup) {
                    for (int k = 0; k < 3; ++k) cand[nc][k] = v[k];
                    ++nc;
                }
            }
        }
        // insertion sort, ascending tuples
        for (int i = 1; i < nc; ++i) {
            for (int j = i; j > 0 && detail::less_tuple(cand[j], cand[j - 1], D); --j) {
                for (int k = 0; k < 3; ++k) {
                    int tmp = cand[j][k];
                    cand[j][k] = cand[j - 1][k];
                    cand[j - 1][k] = tmp;
                }
            }
        }
        if (nc != reps[g].order) t.ok = false;
        t.gstart[g] = q;
        t.gsize[g] = nc;
        int e2 = 0;
        for (int k = 0; k < D; ++k) e2 += reps[g].r[k] * reps[g].r[k];
        t.e2[g] = e2;
        for (int j = 0; j < nc && q < Q; ++j, ++q) {
            for (int k = 0; k < 3; ++k) {
                t.e[q][k] = cand[j][k];
                int m = cand[j][k] < 0 ? -cand[j][k] : cand[j][k];
                if (m > t.emax) t.emax = m;
            }
            t.group[q] = g;
        }
    }
    if (q != Q) t.ok = false;
    for (int i = 0; i < Q; ++i) {
        t.opp[i] = -1;
        for (int j = 0; j < Q; ++j) {
            bool neg = true;
            for (int k = 0; k < 3; ++k)
                if (t.e[j][k] != -t.e[i][k]) neg = false;
            if (neg) t.opp[i] = j;
        }
        if (t.opp[i] < 0) t.ok = false;
    }
    return t;
}

inline constexpr auto kD2Q33 = make_table<2, 33, 8>(kD2Q33Reps);
inline constexpr auto kD3Q95 = make_table<3, 95, 10>(kD3Q95Reps);
inline constexpr auto kD3Q19 = make_table<3, 19, 3>(kD3Q19Reps);
inline constexpr auto kD3Q15 = make_table<3, 15, 3>(kD3Q15Reps);
static_assert(kD2Q33.ok && kD3Q95.ok, "orbit sizes must match Tables 2 and 3");
static_assert(kD3Q19.ok && kD3Q15.ok, "orbit sizes of the lower-order sets");
static_assert(kD2Q33.emax == 4 && kD3Q95.emax == 5, "largest displacement");
static_assert(kD3Q19.emax == 1 && kD3Q15.emax == 1, "largest displacement");

// Largest displacement over the supported models: halo width of the gather.
inline constexpr int kMaxDisp = 5;
inline constexpr int kMaxG = 10;

// Model tags used as template parameters of the kernels.  m is the order of
// accuracy (Formula (5) up to n_max = 2m), N the order of the Hermite
// equilibrium, N = m (the paragraph after Formula (5) asks for N >= m).
struct D2Q33 {
    static constexpr int D = 2, Q = 33, G = 8, m = 4, N = 4;
    static constexpr ModelId id = ModelId::D2Q33;
    static constexpr const auto& table = kD2Q33;
};
struct D3Q95 {
    static constexpr int D = 3, Q = 95, G = 10, m = 4, N = 4;
    static constexpr ModelId id = ModelId::D3Q95;
    static constexpr const auto& table = kD3Q95;
};
struct D3Q19 {
    static constexpr int D = 3, Q = 19, G = 3, m = 2, N = 2;
    static constexpr ModelId id = ModelId::D3Q19;
    static constexpr const auto& table = kD3Q19;
};
struct D3Q15 {
    static constexpr int D = 3, Q = 15, G = 3, m = 2, N = 2;
    static constexpr ModelId id = ModelId::D3Q15;
    static constexpr const auto& table = kD3Q15;
};

}  // namespace lbm
