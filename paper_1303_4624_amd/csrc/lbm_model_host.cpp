// lbm_model_host.cpp - host-side model construction and checks: the weight
// equations of Formula (5) and their Newton solution, used by
// lbm_velocity_set and by the validation in lbm_create.
//
// Built with the host compiler (no device code).  The Newton iteration runs
// in binary128 (__float128): the Jacobian of the weight system has a
// condition number of about 3e6, so a float64 solve leaves errors near 1e-11
// in the weights, a small but systematic change of the model.  In binary128
// the result rounds to the nearest float64 of the exact root.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "lbm_host.h"
#include "lbm_model.h"

namespace lbm {
namespace {

// A compiled model: its velocity table, its order of accuracy m (Formula (5)
// up to n_max = 2m) and the start of the weight solve (the printed table
// values; none for the lower-order sets, which start from least squares).
struct ModelView {
    int D, Q, G, m;
    const int (*e)[3];
    const int* group;
    const int* e2;
    const double* printedW;
    double printedC;
};

template <class M>
ModelView view_of(const double* printedW, double printedC) {
    return {M::D, M::Q, M::G, M::m, M::table.e, M::table.group, M::table.e2, printedW, printedC};
}

ModelView view(ModelId m) {
    switch (m) {
        case ModelId::D2Q33: return view_of<D2Q33>(kD2Q33PrintedW, kD2Q33PrintedC);
        case ModelId::D3Q19: return view_of<D3Q19>(nullptr, 1.0);
        case ModelId::D3Q15: return view_of<D3Q15>(nullptr, 1.0);
        default: return view_of<D3Q95>(kD3Q95PrintedW, kD3Q95PrintedC);
    }
}

// Exponent tuples (a_1 >= ... >= a_D, all even) of the equations of Formula (5)
// up to order 2m: one per partition of q <= m into at most D parts
// (Formula (8)).
void equation_exponents(int D, int m, std::vector<std::vector<int>>& out) {
    out.clear();
    std::vector<int> cur(D, 0);
    // enumerate non-increasing tuples p_1 >= p_2 >= ... >= p_D >= 0, sum <= m
    auto rec = [&](auto&& self, int pos, int maxpart, int rest) -> void {
        if (pos == D) {
            std::vector<int> a(D);
            for (int k = 0; k < D; ++k) a[k] = 2 * cur[k];
            out.push_back(a);
            return;
        }
        for (int p = 0; p <= maxpart && p <= rest; ++p) {
            cur[pos] = p;
            self(self, pos + 1, p, rest - p);
        }
    };
    rec(rec, 0, m, m);
}

// (a - 1)!! / 2^(a/2) for even a: the 1D Gaussian moment normalised to unit mass.
double gauss_moment_1d(int a) {
    double v = 1.0;
    for (int k = a - 1; k > 1; k -= 2) v *= k;
    return v / std::ldexp(1.0, a / 2);
}

// Velocity list of a model: groups in order, each the orbit of its
// representative under coordinate permutations and sign changes, sorted
// ascending inside the group.
struct OrbitModel {
    int D = 0, Q = 0, G = 0;
    std::vector<std::array<int, 3>> e;
    std::vector<int> group;
};

OrbitModel builtin_model(ModelId m) {
    const ModelView v = view(m);
    OrbitModel om;
    om.D = v.D;
    om.Q = v.Q;
    om.G = v.G;
    for (int i = 0; i < v.Q; ++i) {
        om.e.push_back({v.e[i][0], v.e[i][1], v.e[i][2]});
        om.group.push_back(v.group[i]);
    }
    return om;
}

bool make_orbits(int D, int G, const int32_t* reps, OrbitModel& om, std::string& err) {
    om = OrbitModel{};
    om.D = D;
    om.G = G;
    std::vector<std::array<int, 3>> keys;   // sorted |components|, one per orbit
    for (int g = 0; g < G; ++g) {
        std::array<int, 3> r{0, 0, 0};
        for (int k = 0; k < D; ++k) {
            r[k] = reps[g * D + k];
            if (r[k] < -64 || r[k] > 64) {
                err = "representative components must lie in [-64, 64]";
                return false;
            }
        }
        std::array<int, 3> key{0, 0, 0};
        for (int k = 0; k < D; ++k) key[k] = r[k] < 0 ? -r[k] : r[k];
        std::sort(key.begin(), key.begin() + D);
        for (const auto& kk : keys)
            if (kk == key) {
                err = "two representatives generate the same group";
                return false;
            }
        keys.push_back(key);
        std::array<int, 3> perm{0, 1, 2};
        std::vector<std::array<int, 3>> orb;
        do {
            for (int s = 0; s < (1 << D); ++s) {
                std::array<int, 3> v{0, 0, 0};
                for (int k = 0; k < D; ++k) v[k] = ((s >> k) & 1) ? -r[perm[k]] : r[perm[k]];
                if (std::find(orb.begin(), orb.end(), v) == orb.end()) orb.push_back(v);
            }
        } while (std::next_permutation(perm.begin(), perm.begin() + D));
        std::sort(orb.begin(), orb.end());
        for (const auto& v : orb) {
            om.e.push_back(v);
            om.group.push_back(g);
        }
    }
    om.Q = static_cast<int>(om.e.size());
    return true;
}

struct System {
    int G = 0;
    std::vector<std::vector<double>> B;   // B[k][g] = sum over group g of e^a
    std::vector<int> order;               // |a| of equation k
    std::vector<double> rhs;
};

System build_system(const OrbitModel& om, int m) {
    System s;
    s.G = om.G;
    std::vector<std::vector<int>> ex;
    equation_exponents(om.D, m, ex);
    for (const auto& a : ex) {
        std::vector<double> row(om.G, 0.0);
        int ord = 0;
        double r = 1.0;
        for (int k = 0; k < om.D; ++k) {
            ord += a[k];
            r *= gauss_moment_1d(a[k]);
        }
        for (int i = 0; i < om.Q; ++i) {
            double mono = 1.0;
            for (int k = 0; k < om.D; ++k) {
                for (int p = 0; p < a[k]; ++p) mono *= om.e[i][k];
            }
            row[om.group[i]] += mono;
        }
        s.B.push_back(row);
        s.order.push_back(ord);
        s.rhs.push_back(r);
    }
    return s;
}

System build_system(ModelId m) { return build_system(builtin_model(m), view(m).m); }

void residual_and_jacobian(const System& s, const std::vector<double>& W, double c,
                           std::vector<double>& F, std::vector<std::vector<double>>* J) {
    const int n = static_cast<int>(s.rhs.size());
    F.assign(n, 0.0);
    if (J) J->assign(n, std::vector<double>(s.G + 1, 0.0));
    for (int k = 0; k < n; ++k) {
        const double cp = std::pow(c, s.order[k]);
        const double dcp = s.order[k] > 0 ? s.order[k] * std::pow(c, s.order[k] - 1) : 0.0;
        double acc = 0.0, dacc = 0.0;
        for (int g = 0; g < s.G; ++g) {
            acc += W[g] * s.B[k][g];
            if (J) (*J)[k][g] = cp * s.B[k][g];
        }
        dacc = dcp * acc;
        F[k] = cp * acc - s.rhs[k];
        if (J) (*J)[k][s.G] = dacc;
    }
}

double max_residual(const System& s, const std::vector<double>& W, double c) {
    std::vector<double> F;
    residual_and_jacobian(s, W, c, F, nullptr);
    double worst = 0.0;
    for (double f : F) worst = std::fmax(worst, std::fabs(f));
    return worst;
}

using quad = __float128;

quad qabs(quad a) { return a < 0 ? -a : a; }

// Solve the n x n system A x = b (A has n + 1 columns, b in the last) by
// Gaussian elimination with partial pivoting, in binary128.
bool solve_dense(std::vector<std::vector<quad>>& A, std::vector<quad>& x) {
    const int n = static_cast<int>(A.size());
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (qabs(A[r][col]) > qabs(A[piv][col])) piv = r;
        if (A[piv][col] == 0) return false;
        std::swap(A[piv], A[col]);
        for (int r = col + 1; r < n; ++r) {
            const quad f = A[r][col] / A[col][col];
            for (int cc = col; cc <= n; ++cc) A[r][cc] -= f * A[col][cc];
        }
    }
    x.assign(n, 0);
    for (int r = n - 1; r >= 0; --r) {
        quad t = A[r][n];
        for (int cc = r + 1; cc < n; ++cc) t -= A[r][cc] * x[cc];
        x[r] = t / A[r][r];
    }
    return true;
}

// Newton on the square system F(W, c) = 0 of Formula (5), in binary128,
// from x = (W_1..W_G, c).
bool newton(const System& s, std::vector<quad>& x, std::string& err) {
    const int n = static_cast<int>(s.rhs.size());
    const int G = s.G;
    for (int it = 0; it < 80; ++it) {
        std::vector<std::vector<quad>> A(n, std::vector<quad>(n + 1, 0));
        for (int k = 0; k < n; ++k) {
            quad cp = 1, dcp = 0;
            for (int p = 0; p < s.order[k]; ++p) {
                dcp = dcp * x[G] + cp;
                cp *= x[G];
            }
            quad acc = 0;
            for (int g = 0; g < G; ++g) {
                acc += x[g] * static_cast<quad>(s.B[k][g]);
                A[k][g] = cp * static_cast<quad>(s.B[k][g]);
            }
            A[k][G] = dcp * acc;
            A[k][n] = -(cp * acc - static_cast<quad>(s.rhs[k]));
        }
        std::vector<quad> dx;
        if (!solve_dense(A, dx)) {
            err = "singular Jacobian in the weight solve";
            return false;
        }
        quad rel = 0;
        for (int k = 0; k < n; ++k) {
            x[k] += dx[k];
            const quad r = qabs(dx[k]) / qabs(x[k]);
            if (r > rel) rel = r;
        }
        if (rel < static_cast<quad>(1e-30)) return true;
    }
    err = "Newton iteration for the weights did not converge";
    return false;
}

// Least-squares group weights at the speed x[G]: (A^T A) W = A^T rhs with
// A = c^|a| B; written into x[0 .. G).
bool least_squares_weights(const System& s, std::vector<quad>& x, std::string& err) {
    const int n = static_cast<int>(s.rhs.size());
    const int G = s.G;
    std::vector<std::vector<quad>> A(n, std::vector<quad>(G));
    for (int k = 0; k < n; ++k) {
        quad cp = 1;
        for (int p = 0; p < s.order[k]; ++p) cp *= x[G];
        for (int g = 0; g < G; ++g) A[k][g] = cp * static_cast<quad>(s.B[k][g]);
    }
    std::vector<std::vector<quad>> N(G, std::vector<quad>(G + 1, 0));
    for (int i = 0; i < G; ++i) {
        for (int j = 0; j < G; ++j)
            for (int k = 0; k < n; ++k) N[i][j] += A[k][i] * A[k][j];
        for (int k = 0; k < n; ++k) N[i][G] += A[k][i] * static_cast<quad>(s.rhs[k]);
    }
    std::vector<quad> w0;
    if (!solve_dense(N, w0)) {
        err = "singular least-squares system for the initial weights";
        return false;
    }
    for (int g = 0; g < G; ++g) x[g] = w0[g];
    return true;
}

}  // namespace

bool model_from_shape(int D, int Q, ModelId& m) {
    for (ModelId id : {ModelId::D2Q33, ModelId::D3Q95, ModelId::D3Q19, ModelId::D3Q15}) {
        const ModelView v = view(id);
        if (v.D == D && v.Q == Q) {
            m = id;
            return true;
        }
    }
    return false;
}

int model_dim(ModelId m) { return view(m).D; }
int model_q(ModelId m) { return view(m).Q; }
int model_groups(ModelId m) { return view(m).G; }
int model_group_of(ModelId m, int i) { return view(m).group[i]; }
int model_e(ModelId m, int i, int k) { return view(m).e[i][k]; }
int model_e2(ModelId m, int g) { return view(m).e2[g]; }
int model_order(ModelId m) { return view(m).m; }

bool model_matches(ModelId m, const int32_t* e) {
    const ModelView v = view(m);
    for (int i = 0; i < v.Q; ++i)
        for (int k = 0; k < v.D; ++k)
            if (e[i * v.D + k] != v.e[i][k]) return false;
    return true;
}

double model_residual(ModelId m, const double* W, double c) {
    const System s = build_system(m);
    return max_residual(s, std::vector<double>(W, W + s.G), c);
}

bool model_solve(ModelId m, double* W, double* c, std::string& err) {
    const ModelView v = view(m);
    const System s = build_system(m);
    if (static_cast<int>(s.rhs.size()) != v.G + 1) {
        err = "weight system is not square";
        return false;
    }
    std::vector<quad> x(v.G + 1);
    x[v.G] = v.printedC;
    if (v.printedW) {
        for (int g = 0; g < v.G; ++g) x[g] = v.printedW[g];
    } else if (!least_squares_weights(s, x, err)) {
        return false;
    }
    if (!newton(s, x, err)) return false;
    for (int g = 0; g < v.G; ++g) W[g] = static_cast<double>(x[g]);
    *c = static_cast<double>(x[v.G]);
    return true;
}

int equation_count(int m, int D) {
    std::vector<std::vector<int>> ex;
    equation_exponents(D, m, ex);
    return static_cast<int>(ex.size());
}

bool model_build(int D, int m, int G, const int32_t* reps, const double* w_guess, double c_guess,
                 BuiltModel& out, std::string& err) {
    OrbitModel om;
    if (!make_orbits(D, G, reps, om, err)) return false;
    const System s = build_system(om, m);
    const int n = static_cast<int>(s.rhs.size());
    if (n != G + 1) {
        err = "Formula (10) needs G + 1 = Omega(m, D) = " + std::to_string(n) + " unknowns, got " +
              std::to_string(G + 1);
        return false;
    }
    std::vector<quad> x(G + 1);
    x[G] = c_guess;
    if (w_guess) {
        for (int g = 0; g < G; ++g) x[g] = w_guess[g];
    } else if (!least_squares_weights(s, x, err)) {
        return false;
    }
    if (!newton(s, x, err)) return false;
    out.D = D;
    out.Q = om.Q;
    out.G = G;
    out.e = om.e;
    out.group = om.group;
    out.W.assign(G, 0.0);
    for (int g = 0; g < G; ++g) out.W[g] = static_cast<double>(x[g]);
    out.c = static_cast<double>(x[G]);
    out.residual = max_residual(s, out.W, out.c);
    return true;
}

}  // namespace lbm
