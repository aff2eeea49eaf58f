// lbm_model_host.cpp - host-side model construction and checks: the weight
// equations of Formula (5) and their Newton solution, used by
// lbm_velocity_set and by the validation in lbm_create.
//
// Built with the host compiler (no device code).  The Newton iteration runs
// in binary128 (__float128): the Jacobian of the weight system has a
// condition number of about 3e6, so a float64 solve leaves errors near 1e-11
// in the weights, a small but systematic change of the model.  In binary128
// the result rounds to the nearest float64 of the exact root.
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
    using q = __float128;
    const ModelView v = view(m);
    const System s = build_system(m);
    const int n = static_cast<int>(s.rhs.size());
    if (n != v.G + 1) {
        err = "weight system is not square";
        return false;
    }
    std::vector<q> x(v.G + 1);
    for (int g = 0; g < v.G; ++g) x[g] = v.printedW[g];
    x[v.G] = v.printedC;
    auto qabs = [](q a) { return a < 0 ? -a : a; };
    bool converged = false;
    for (int it = 0; it < 80; ++it) {
        // residual and Jacobian in binary128
        std::vector<std::vector<q>> A(n, std::vector<q>(n + 1, 0));
        for (int k = 0; k < n; ++k) {
            q cp = 1, dcp = 0;
            for (int p = 0; p < s.order[k]; ++p) {
                dcp = dcp * x[v.G] + cp;
                cp *= x[v.G];
            }
            q acc = 0;
            for (int g = 0; g < v.G; ++g) {
                acc += x[g] * static_cast<q>(s.B[k][g]);
                A[k][g] = cp * static_cast<q>(s.B[k][g]);
            }
            A[k][v.G] = dcp * acc;
            A[k][n] = -(cp * acc - static_cast<q>(s.rhs[k]));
        }
        // Gaussian elimination with partial pivoting
        for (int col = 0; col < n; ++col) {
            int piv = col;
            for (int r = col + 1; r < n; ++r)
                if (qabs(A[r][col]) > qabs(A[piv][col])) piv = r;
            if (A[piv][col] == 0) {
                err = "singular Jacobian in the weight solve";
                return false;
            }
            std::swap(A[piv], A[col]);
            for (int r = col + 1; r < n; ++r) {
                const q f = A[r][col] / A[col][col];
                for (int cc = col; cc <= n; ++cc) A[r][cc] -= f * A[col][cc];
            }
        }
        std::vector<q> dx(n, 0);
        for (int r = n - 1; r >= 0; --r) {
            q t = A[r][n];
            for (int cc = r + 1; cc < n; ++cc) t -= A[r][cc] * dx[cc];
            dx[r] = t / A[r][r];
        }
        q rel = 0;
        for (int k = 0; k < n; ++k) {
            x[k] += dx[k];
            const q r = qabs(dx[k]) / qabs(x[k]);
            if (r > rel) rel = r;
        }
        if (rel < static_cast<q>(1e-30)) {
            converged = true;
            break;
        }
    }
    if (!converged) {
        err = "Newton iteration for the weights did not converge";
        return false;
    }
    for (int g = 0; g < v.G; ++g) W[g] = static_cast<double>(x[g]);
    *c = static_cast<double>(x[v.G]);
    return true;
}

}  // namespace lbm
