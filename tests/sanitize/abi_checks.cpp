// Host-side checks of the C ABI, built with AddressSanitizer and
// UndefinedBehaviorSanitizer (tests/test_host_sanitizers.py): model tables
// and the Formula (5) solver, the model constructor, context creation and
// every argument check that runs without a device, on valid and invalid
// input.  Prints "ok" and returns 0 when every expectation holds.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <limits>
#include <set>
#include <vector>

#include "lbm.h"

static int g_fail = 0;
#define EXPECT(cond)                                                          \
    do {                                                                      \
        if (!(cond)) {                                                        \
            std::printf("FAIL line %d: %s\n", __LINE__, #cond);               \
            ++g_fail;                                                         \
        }                                                                     \
    } while (0)

namespace {

struct Model {
    int D, Q;
    std::vector<int32_t> e;
    std::vector<double> w;
    double c = 0;
};

Model velocity_set(int D, int Q) {
    Model m{D, Q, std::vector<int32_t>(static_cast<size_t>(Q) * D), std::vector<double>(Q)};
    EXPECT(lbm_velocity_set(D, Q, m.e.data(), m.w.data(), &m.c) == LBM_OK);
    return m;
}

// Group representatives of a canonical velocity list: the first vector of
// each run of vectors with the same multiset of absolute components.
std::vector<int32_t> representatives(const Model& m) {
    std::vector<int32_t> reps;
    std::multiset<int> prev;
    for (int i = 0; i < m.Q; ++i) {
        std::multiset<int> a;
        for (int k = 0; k < m.D; ++k) a.insert(std::abs(m.e[i * m.D + k]));
        if (i == 0 || a != prev)
            for (int k = 0; k < m.D; ++k) reps.push_back(m.e[i * m.D + k]);
        prev = a;
    }
    return reps;
}

lbm_ctx* create(const Model& m, const int64_t* ext, double omega = 1.3,
                int prec = LBM_FP32_SHIFTED, int* status = nullptr) {
    lbm_ctx* ctx = nullptr;
    const int rc = lbm_create(&ctx, m.D, m.Q, m.e.data(), m.w.data(), m.c, ext, omega, prec, 1.0,
                              nullptr);
    if (status) *status = rc;
    return rc == LBM_OK ? ctx : nullptr;
}

void check_models() {
    for (int D = 2; D <= 3; ++D) {
        const int Q = D == 2 ? 33 : 95;
        const Model m = velocity_set(D, Q);
        double s = 0;
        for (double x : m.w) s += x;
        EXPECT(std::fabs(s - 1.0) < 1e-14);
        EXPECT(m.c > 0.3 && m.c < 1.0);
        // constructor from the table's representatives reproduces the weights
        const std::vector<int32_t> reps = representatives(m);
        const int G = static_cast<int>(reps.size()) / D;
        EXPECT(G == (D == 2 ? 8 : 10));
        std::vector<int32_t> e(static_cast<size_t>(Q) * D), grp(Q);
        std::vector<double> w(Q);
        double c = 0, res = 1;
        int q = 0;
        EXPECT(lbm_model_build(D, 4, G, reps.data(), nullptr, m.c * 1.01, Q, e.data(), grp.data(),
                               w.data(), &c, &q, &res) == LBM_OK);
        EXPECT(q == Q && res < 1e-12 && c == m.c && w == m.w && e == m.e);
        // too small an output: Q is still reported
        q = 0;
        EXPECT(lbm_model_build(D, 4, G, reps.data(), nullptr, m.c, Q - 1, e.data(), nullptr,
                               nullptr, nullptr, &q, nullptr) == LBM_E_INVALID);
        EXPECT(q == Q);
        // not square (one group less), repeated group, bad guesses
        EXPECT(lbm_model_build(D, 4, G - 1, reps.data(), nullptr, m.c, Q, nullptr, nullptr,
                               nullptr, nullptr, nullptr, nullptr) == LBM_E_INVALID);
        std::vector<int32_t> rep2 = reps;
        for (int k = 0; k < D; ++k) rep2[D + k] = reps[k + D] == 0 ? 0 : -reps[k + D];
        for (int k = 0; k < D; ++k) rep2[2 * D + k] = rep2[D + k];
        EXPECT(lbm_model_build(D, 4, G, rep2.data(), nullptr, m.c, Q, nullptr, nullptr, nullptr,
                               nullptr, nullptr, nullptr) == LBM_E_INVALID);
        EXPECT(lbm_model_build(D, 4, G, reps.data(), nullptr, -1.0, Q, nullptr, nullptr, nullptr,
                               nullptr, nullptr, nullptr) == LBM_E_INVALID);
        EXPECT(lbm_model_build(D, 4, G, reps.data(), nullptr,
                               std::numeric_limits<double>::quiet_NaN(), Q, nullptr, nullptr,
                               nullptr, nullptr, nullptr, nullptr) == LBM_E_INVALID);
        std::vector<int32_t> big = reps;
        big[D] = 65;   // components are limited to [-64, 64]
        EXPECT(lbm_model_build(D, 4, G, big.data(), nullptr, m.c, Q, nullptr, nullptr, nullptr,
                               nullptr, nullptr, nullptr) == LBM_E_INVALID);
    }
    // the 1D set {0, +-1, +-3} at m = 3 has two roots; the guess selects one
    const int32_t r1[3] = {0, 1, 3};
    double ca = 0, cb = 0;
    int q = 0;
    EXPECT(lbm_model_build(1, 3, 3, r1, nullptr, 0.5, 5, nullptr, nullptr, nullptr, &ca, &q,
                           nullptr) == LBM_OK);
    EXPECT(lbm_model_build(1, 3, 3, r1, nullptr, 1.5, 5, nullptr, nullptr, nullptr, &cb, &q,
                           nullptr) == LBM_OK);
    EXPECT(q == 5 && ca > 0 && cb > 0 && std::fabs(ca - cb) > 1e-3);
    EXPECT(lbm_model_build(4, 2, 2, r1, nullptr, 1.0, 5, nullptr, nullptr, nullptr, nullptr,
                           nullptr, nullptr) == LBM_E_UNSUPPORTED);
    EXPECT(lbm_model_build(1, 3, 3, nullptr, nullptr, 1.0, 5, nullptr, nullptr, nullptr, nullptr,
                           nullptr, nullptr) == LBM_E_INVALID);
    EXPECT(lbm_model_build(1, 3, -1, r1, nullptr, 1.0, 5, nullptr, nullptr, nullptr, nullptr,
                           nullptr, nullptr) == LBM_E_INVALID);
    // equation counts: Table 1's range and outside it
    int cnt = 0;
    for (int D = 1; D <= 8; ++D)
        for (int m = 0; m <= 16; ++m) {
            EXPECT(lbm_equation_count(m, D, &cnt) == LBM_OK);
            EXPECT(cnt >= 1);
        }
    EXPECT(lbm_equation_count(4, 2, &cnt) == LBM_OK && cnt == 9);
    EXPECT(lbm_equation_count(4, 3, &cnt) == LBM_OK && cnt == 11);
    EXPECT(lbm_equation_count(-1, 2, &cnt) == LBM_E_INVALID);
    EXPECT(lbm_equation_count(17, 2, &cnt) == LBM_E_INVALID);
    EXPECT(lbm_equation_count(2, 0, &cnt) == LBM_E_INVALID);
    EXPECT(lbm_equation_count(2, 9, &cnt) == LBM_E_INVALID);
    EXPECT(lbm_equation_count(2, 2, nullptr) == LBM_E_INVALID);
    EXPECT(lbm_velocity_set(3, 27, nullptr, nullptr, nullptr) == LBM_E_UNSUPPORTED);
}

void check_create() {
    const Model m = velocity_set(3, 95);
    const int64_t ext[3] = {6, 4, 20};
    int rc = 0;
    lbm_ctx* ctx = create(m, ext);
    EXPECT(ctx != nullptr);
    size_t pop = 0, scr = 0;
    EXPECT(lbm_workspace_bytes(ctx, &pop, &scr) == LBM_OK);
    EXPECT(pop == 95u * 6 * 4 * 20 * 4 && scr > 0);
    // calls that need bound buffers
    EXPECT(lbm_step(ctx, 1) == LBM_E_STATE);
    EXPECT(lbm_moments(ctx, nullptr, nullptr, nullptr) == LBM_E_STATE);
    double cons[5];
    EXPECT(lbm_conservation(ctx, cons) == LBM_E_STATE);
    EXPECT(lbm_conservation_noalloc(ctx, cons) == LBM_E_STATE);
    EXPECT(lbm_conservation_noalloc(nullptr, cons) == LBM_E_INVALID);
    EXPECT(lbm_init_fields(ctx, nullptr, nullptr, nullptr) == LBM_E_STATE);
    EXPECT(lbm_restore_checkpoint(ctx, 10, 3, 1, nullptr, 0, 0) == LBM_E_STATE);
    // host memory is not device memory (and there is no device here)
    std::vector<char> host(pop + 256);
    EXPECT(lbm_bind(ctx, host.data(), host.data() + 128, host.data()) != LBM_OK);
    EXPECT(lbm_last_error(ctx) != nullptr && lbm_last_error(ctx)[0] != '\0');
    // sizes of checkpoints and adjoint workspaces
    size_t b1 = 0, b2 = 0;
    EXPECT(lbm_checkpoint_bytes(ctx, 200, 20, 1, &b1) == LBM_OK);
    EXPECT(lbm_checkpoint_bytes(ctx, 200, 20, 99, &b2) == LBM_OK && b2 > b1);
    EXPECT(lbm_checkpoint_bytes(ctx, 0, 20, 1, &b1) == LBM_E_INVALID);
    EXPECT(lbm_adjoint_workspace_bytes(ctx, 200, 20, 1, &b1) == LBM_OK);
    EXPECT(lbm_adjoint_workspace_bytes(ctx, 200, 20, 99, &b2) == LBM_OK && b2 < b1);
    EXPECT(lbm_adjoint_workspace_bytes(ctx, 5, 0, 1, &b1) == LBM_E_INVALID);
    // streaming scheme, held planes, graph steps, omega
    const double good[5] = {1.0, 0.0, 0.0, 0.0, 1.0};
    const double bad[5] = {-1.0, 0.0, 0.0, 0.0, 1.0};
    const double nan[5] = {1.0, std::numeric_limits<double>::quiet_NaN(), 0.0, 0.0, 1.0};
    EXPECT(lbm_set_streaming(ctx, 7) == LBM_E_INVALID);
    EXPECT(lbm_set_streaming(ctx, LBM_STREAM_AA) == LBM_OK);
    EXPECT(lbm_set_fixed_planes(ctx, 5, 5, good, good) == LBM_OK);
    EXPECT(lbm_set_fixed_planes(ctx, 15, 6, good, good) == LBM_E_INVALID);
    EXPECT(lbm_set_fixed_planes(ctx, -1, 0, good, good) == LBM_E_INVALID);
    EXPECT(lbm_set_fixed_planes(ctx, 1, 0, nullptr, nullptr) == LBM_E_INVALID);
    EXPECT(lbm_set_fixed_planes(ctx, 1, 1, good, bad) == LBM_E_INVALID);
    EXPECT(lbm_set_fixed_planes(ctx, 1, 1, good, nan) == LBM_E_NONFINITE);
    EXPECT(lbm_set_fixed_planes(ctx, 0, 0, nullptr, nullptr) == LBM_OK);
    EXPECT(lbm_set_streaming(ctx, LBM_STREAM_AB) == LBM_OK);
    EXPECT(lbm_set_graph_steps(ctx, 3) == LBM_E_INVALID);
    EXPECT(lbm_set_graph_steps(ctx, 4) == LBM_E_UNSUPPORTED);   // null stream
    EXPECT(lbm_set_graph_steps(ctx, 0) == LBM_OK);
    EXPECT(lbm_set_omega(ctx, 2.0) == LBM_E_INVALID);
    EXPECT(lbm_set_omega(ctx, std::numeric_limits<double>::infinity()) == LBM_E_INVALID);
    EXPECT(lbm_set_omega(ctx, 1.7) == LBM_OK);
    EXPECT(lbm_destroy(ctx) == LBM_OK);
    EXPECT(lbm_destroy(nullptr) == LBM_OK);

    // rejected models and grids
    Model p = m;
    p.w[3] *= 1.0 + 1e-9;
    EXPECT(create(p, ext, 1.3, LBM_FP64, &rc) == nullptr && rc == LBM_E_INVALID);
    p = m;
    p.c *= 1.001;
    EXPECT(create(p, ext, 1.3, LBM_FP64, &rc) == nullptr && rc == LBM_E_INVALID);
    p = m;
    std::swap(p.e[3], p.e[4]);
    EXPECT(create(p, ext, 1.3, LBM_FP64, &rc) == nullptr && rc == LBM_E_UNSUPPORTED);
    p = m;
    p.Q = 94;
    EXPECT(create(p, ext, 1.3, LBM_FP64, &rc) == nullptr && rc == LBM_E_UNSUPPORTED);
    EXPECT(create(m, ext, 2.0, LBM_FP64, &rc) == nullptr && rc == LBM_E_INVALID);
    EXPECT(create(m, ext, -0.1, LBM_FP64, &rc) == nullptr && rc == LBM_E_INVALID);
    EXPECT(create(m, ext, 1.3, 5, &rc) == nullptr && rc == LBM_E_UNSUPPORTED);
    const int64_t zero[3] = {6, 0, 20};
    const int64_t neg[3] = {6, 4, -3};
    const int64_t huge[3] = {1 << 20, 1 << 20, 4};        // N >= 2^31
    const int64_t slab[3] = {65536, 256, 2};               // one slab above 4 GiB
    for (const int64_t* x : {zero, neg, huge, slab}) {
        EXPECT(create(m, x, 1.3, LBM_FP32_SHIFTED, &rc) == nullptr && rc == LBM_E_INVALID);
    }
    lbm_ctx* out = nullptr;
    EXPECT(lbm_create(&out, 3, 95, nullptr, m.w.data(), m.c, ext, 1.3, LBM_FP64, 1.0, nullptr) ==
           LBM_E_INVALID);
    EXPECT(lbm_create(nullptr, 3, 95, m.e.data(), m.w.data(), m.c, ext, 1.3, LBM_FP64, 1.0,
                      nullptr) == LBM_E_INVALID);
    for (int s = 1; s >= -6; --s) EXPECT(lbm_status_str(s) != nullptr);
    EXPECT(lbm_last_error(nullptr) != nullptr);
}

}  // namespace

int main() {
    check_models();
    check_create();
    if (g_fail == 0) std::printf("ok\n");
    return g_fail == 0 ? 0 : 1;
}
