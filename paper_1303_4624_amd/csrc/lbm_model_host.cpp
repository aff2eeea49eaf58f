// lbm_model_host.cpp - host-side model construction and checks: the weight
// equations of Formula (5) and their Newton solution, used by
// lbm_velocity_set and by the validation in lbm_create.
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "lbm_host.h"
#include "lbm_model.h"

namespace lbm {
namespace {

struct ModelView {
    int D, Q, G;
    const int (*e)[3];
    const int* group;
    const double* printedW;
    double printedC;
};

ModelView view(ModelId m) {
    if (m == ModelId::D2Q33)
        return {2, 33, 8, kD2Q33.e, kD2Q33.group, kD2Q33PrintedW, kD2Q33PrintedC};
    return {3, 95, 10, kD3Q95.e, kD3Q95.group, kD3Q95PrintedW, kD3Q95PrintedC};
}

// Exponent tuples (a_1 >= ... >= a_D, all even) of the equations of Formula (5)
// up to order 2m = 8: one per partition of q <= 4 into at most D parts.
void equation_exponents(int D, std::vector<std::vector<int>>& out) {
    out.clear();
    std::vector<int> cur(D, 0);
    // enumerate non-increasing tuples p_1 >= p_2 >= ... >= p_D >= 0, sum <= 4
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
    rec(rec, 0, 4, 4);
}

// (a - 1)!! / 2^(a/2) for even a: the 1D Gaussian moment normalised to unit mass.
double gauss_moment_1d(int a) {
    double v = 1.0;
    for (int k = a - 1; k > 1; k -= 2) v *= k;
    return v / std::ldexp(1.0, a / 2);
}

struct System {
    int G = 0;
    std::vector<std::vector<double>> B;   // B[k][g] = sum over group g of e^a
    std::vector<int> order;               // |a| of equation k
    std::vector<double> rhs;
};

System build_system(ModelId m) {
    const ModelView v = view(m);
    System s;
    s.G = v.G;
    std::vector<std::vector<int>> ex;
    equation_exponents(v.D, ex);
    for (const auto& a : ex) {
        std::vector<double> row(v.G, 0.0);
        int ord = 0;
        double r = 1.0;
        for (int k = 0; k < v.D; ++k) {
            ord += a[k];
            r *= gauss_moment_1d(a[k]);
        }
        for (int i = 0; i < v.Q; ++i) {
            double mono = 1.0;
            for (int k = 0; k < v.D; ++k) {
                for (int p = 0; p < a[k]; ++p) mono *= v.e[i][k];
            }
            row[v.group[i]] += mono;
        }
        s.B.push_back(row);
        s.order.push_back(ord);
        s.rhs.push_back(r);
    }
    return s;
}

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

bool solve_dense(std::vector<std::vector<double>> A, std::vector<double> b, std::vector<double>& x) {
    const int n = static_cast<int>(b.size());
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (std::fabs(A[r][col]) > std::fabs(A[piv][col])) piv = r;
        if (A[piv][col] == 0.0) return false;
        std::swap(A[piv], A[col]);
        std::swap(b[piv], b[col]);
        for (int r = col + 1; r < n; ++r) {
            const double f = A[r][col] / A[col][col];
            for (int cc = col; cc < n; ++cc) A[r][cc] -= f * A[col][cc];
            b[r] -= f * b[col];
        }
    }
    x.assign(n, 0.0);
    for (int r = n - 1; r >= 0; --r) {
        double s = b[r];
        for (int cc = r + 1; cc < n; ++cc) s -= A[r][cc] * x[cc];
        x[r] = s / A[r][r];
    }
    return true;
}

}  // namespace

bool model_from_shape(int D, int Q, ModelId& m) {
    if (D == 2 && Q == 33) {
        m = ModelId::D2Q33;
        return true;
    }
    if (D == 3 && Q == 95) {
        m = ModelId::D3Q95;
        return true;
    }
    return false;
}

int model_dim(ModelId m) { return view(m).D; }
int model_q(ModelId m) { return view(m).Q; }
int model_groups(ModelId m) { return view(m).G; }
int model_group_of(ModelId m, int i) { return view(m).group[i]; }
int model_e(ModelId m, int i, int k) { return view(m).e[i][k]; }
int model_e2(ModelId m, int g) {
    return m == ModelId::D2Q33 ? kD2Q33.e2[g] : kD3Q95.e2[g];
}

bool model_matches(ModelId m, const int32_t* e) {
    const ModelView v = view(m);
    for (int i = 0; i < v.Q; ++i)
        for (int k = 0; k < v.D; ++k)
            if (e[i * v.D + k] != v.e[i][k]) return false;
    return true;
}

double model_residual(ModelId m, const double* W, double c) {
    const System s = build_system(m);
    std::vector<double> Wv(W, W + s.G), F;
    residual_and_jacobian(s, Wv, c, F, nullptr);
    double worst = 0.0;
    for (double f : F) worst = std::fmax(worst, std::fabs(f));
    return worst;
}

bool model_solve(ModelId m, double* W, double* c, std::string& err) {
    const ModelView v = view(m);
    const System s = build_system(m);
    if (static_cast<int>(s.rhs.size()) != v.G + 1) {
        err = "weight system is not square";
        return false;
    }
    std::vector<double> x(v.G + 1);
    for (int g = 0; g < v.G; ++g) x[g] = v.printedW[g];
    x[v.G] = v.printedC;
    bool converged = false;
    for (int it = 0; it < 60; ++it) {
        std::vector<double> F, dx;
        std::vector<std::vector<double>> J;
        std::vector<double> Wv(x.begin(), x.begin() + v.G);
        residual_and_jacobian(s, Wv, x[v.G], F, &J);
        for (double& f : F) f = -f;
        if (!solve_dense(J, F, dx)) {
            err = "singular Jacobian in the weight solve";
            return false;
        }
        double rel = 0.0;
        for (int k = 0; k <= v.G; ++k) {
            x[k] += dx[k];
            rel = std::fmax(rel, std::fabs(dx[k]) / std::fmax(std::fabs(x[k]), 1e-300));
        }
        if (rel < 1e-15) {
            converged = true;
            break;
        }
    }
    std::vector<double> Wv(x.begin(), x.begin() + v.G), F;
    residual_and_jacobian(s, Wv, x[v.G], F, nullptr);
    double worst = 0.0;
    for (double f : F) worst = std::fmax(worst, std::fabs(f));
    if (!converged && worst > 1e-13) {
        err = "Newton iteration for the weights did not converge";
        return false;
    }
    for (int g = 0; g < v.G; ++g) W[g] = x[g];
    *c = x[v.G];
    return true;
}

}  // namespace lbm
