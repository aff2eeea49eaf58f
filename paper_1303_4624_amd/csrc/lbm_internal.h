// lbm_internal.h - parameters and launchers shared by the C-ABI layer
// (lbm_api.cpp) and the kernels (lbm_kernels.h).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "lbm_model.h"

// Largest block of the row-blocked kernels (launch bounds): the default, and
// float64 storage with the 4th-order sets.
#ifndef LBM_STEP_MAXB
#define LBM_STEP_MAXB 512
#endif
#ifndef LBM_F64_MAXB
#define LBM_F64_MAXB 256
#endif

namespace lbm {

// Largest block of the row-blocked kernels (step, in-place step, adjoint)
// for a set of Q velocities stored in precision p; the kernels' launch
// bounds and the host's launch geometry both take it from here.  Float64
// with Q >= 33 (up to 256 VGPRs per lane) keeps 256 threads; the lower-order
// float64 sets and FP32-shifted take 512 (measured with both limits bound to
// the same buffers: D3Q19 and D3Q15 float64 at 384^3 1.5-1.9 % faster with
// 512, D3Q95 float64 0.1-0.8 % slower).
constexpr int row_block_limit(int Q, Prec p) {
    return (p == Prec::F64 && Q >= 33) ? LBM_F64_MAXB : LBM_STEP_MAXB;
}

// Elements added to every population run of a row (run stride = nx + pad).
#ifndef LBM_RUN_PAD
#define LBM_RUN_PAD 0
#endif
constexpr int kRunPad = LBM_RUN_PAD;

// Rows of at least this many cells get a run stride rounded up to a multiple
// of it (32 elements: every population run starts on a 128-byte line).
// Measured on D3Q95 FP32-shifted: +8 % to +20 % for 376^3, 392^3, 400^3;
// no change where nx is already a multiple.
#ifndef LBM_RUN_ALIGN
#define LBM_RUN_ALIGN 32
#endif
constexpr int kRunAlign = LBM_RUN_ALIGN;

// Rows (consecutive y, same z) whose population runs are interleaved in 3D
// (a power of two),
// when ny is a multiple of it (else 1); 2D rows are long enough alone.
// Measured on D3Q95: 2 rows +0.7 % (FP32-shifted 384^3) and +1.5 % (FP64
// 256^3); on D2Q33 8192^2 grouping lost 3 % (2 rows) to 13 % (8 rows).
#ifndef LBM_ROW_GROUP_SHIFT
#define LBM_ROW_GROUP_SHIFT 1
#endif
constexpr int kRowGroup3DShift = LBM_ROW_GROUP_SHIFT;
constexpr int kRowGroup3D = 1 << kRowGroup3DShift;

// Whole grid rows per block of the row-blocked kernels when a row is a
// multiple of 64 cells and several fit in one block (0: one row per block).
#ifndef LBM_PACK_ROWS
#define LBM_PACK_ROWS 1
#endif
constexpr bool kPackRows = LBM_PACK_ROWS != 0;
// Largest block made of packed rows: forward steps, and the adjoint (whose
// kernels hold more registers, so that large packed blocks leave fewer waves
// per CU).  Measured on D3Q95 FP32-shifted 128^3: forward step +1.1 % with
// 512 against one row per block; adjoint 2 % slower with 512, +0.3 % with 256.
#ifndef LBM_PACK_MAXB
#define LBM_PACK_MAXB 512
#endif
#ifndef LBM_PACK_ADJ_MAXB
#define LBM_PACK_ADJ_MAXB 256
#endif
constexpr int kPackMaxBlock = LBM_PACK_MAXB;
constexpr int kPackAdjMaxBlock = LBM_PACK_ADJ_MAXB;

// A macroscopic state held fixed on boundary planes.
struct FixedState {
    double rho;
    double U[3];
    double T;
};

// Storage forms of the population buffer (see the kernels' PopAt).
constexpr int kFormAB = 0;        // two buffers: run i of cell c
constexpr int kFormSwapped = 1;   // in place, after an even number of steps: run opp(i) of c
constexpr int kFormPushed = 2;    // in place, after an odd number of steps: run i of c + e_i

// Per-context constants, passed to every kernel by value.  Per group only
// the weight W_g and X_g = |e_g|^2 / T0 are arguments (argument values live
// in scalar registers; the kernels form every other coefficient of the
// equilibrium per cell as a polynomial in X).
struct KParams {
    int nx, ny, nz;           // nz = 1 in 2D
    int form;                 // storage form of the state the kernel reads or writes
    int rs;                   // run stride: elements between two population runs of a row
    int rg;                   // rows per group (consecutive y sharing interleaved runs), 1 or 2
    int rg_shift;             // log2(rg)
    int chunks;               // blocks per grid row (x direction)
    int rpb;                  // grid rows per block (> 1 only with chunks = 1, nx % 64 = 0)
    int bx;                   // threads per block (multiple of 64)
    int xcd_cyclic;           // > 0: the forward steps hand the 8 XCDs chunks of this
                              // many blocks in turn; 0: a contiguous range each
    long long N;              // cells
    double omega;             // relaxation frequency
    double omc;               // 1 - omega as used by the kernels (float-rounded for F32S)
    double omega_eff;         // 1 - omc, so that omc + omega_eff = 1 exactly
    double T0;                // reference temperature 1/(2c^2)
    double invT0;             // 1 / T0
    double rho0;              // shift reference (FP32-shifted storage)
    double W[kMaxG];          // group weights
    double X[kMaxG];          // |e_g|^2 / T0 per group
    int hold_lo, hold_hi;     // planes of the slowest axis held at f^eq(hold[0] / hold[1])
    FixedState hold[2];
};

// Launch geometry of the row-blocked kernels: one grid row (fixed y, z) is
// split into `chunks` blocks of `bx` threads.
struct RowLaunch {
    int bx;
    int chunks;
    long long blocks;
};

RowLaunch row_launch(int nx, long long rows, int max_threads);
// Largest block size the row-blocked kernels of a model and precision are
// compiled for (row_block_limit of its Q).
int step_max_threads(ModelId m, Prec p);

// Number of blocks of the grid-stride reduction kernels.
int reduce_blocks(long long N);
constexpr int kReduceThreads = 256;

// Launchers: each returns the hipError_t of the launch.
hipError_t launch_init(ModelId m, Prec p, const KParams& kp, const double* rho, const double* U,
                       const double* T, void* f, hipStream_t s);
hipError_t launch_set_pop(ModelId m, Prec p, const KParams& kp, const double* fin, void* f,
                          hipStream_t s);
hipError_t launch_get_pop(ModelId m, Prec p, const KParams& kp, const void* f, double* fout,
                          hipStream_t s);
// One update step from src into dst.  mom_out != nullptr: also store the
// step's D+2 moments (recomputation for the adjoint).  dst == nullptr (with
// mom_out): gather and store the moments only, no populations (the last
// recomputed step of a segment, whose state the next checkpoint holds).
hipError_t launch_step(ModelId m, Prec p, const KParams& kp, const void* src, void* dst,
                       void* mom_out, hipStream_t s);
// In-place step (AA pattern): push = true reads the swapped form and writes
// the pushed form, push = false the reverse.  mom_out != nullptr: also store
// the step's D+2 moments (as launch_step does; held planes store the moments
// of their held state).
hipError_t launch_step_aa(ModelId m, Prec p, const KParams& kp, void* f, bool push,
                          void* mom_out, hipStream_t s);
// Copy of the state f, stored in form kp.form, into the two-buffer form.
hipError_t launch_to_ab(ModelId m, Prec p, const KParams& kp, const void* f, void* out,
                        hipStream_t s);
// Copy of the two-buffer-form state f into form kp.form (two-buffer or swapped).
hipError_t launch_from_ab(ModelId m, Prec p, const KParams& kp, const void* f, void* out,
                          hipStream_t s);
hipError_t launch_moments(ModelId m, Prec p, const KParams& kp, const void* f, double* rho,
                          double* U, double* T, hipStream_t s);
hipError_t launch_conservation(ModelId m, Prec p, const KParams& kp, const void* f,
                               double* partials, double* out, hipStream_t s);
hipError_t launch_fill_zero(double* p, long long n, hipStream_t s);
// Streaming copy of `bytes` (a multiple of 4; src and dst 16-byte aligned).
hipError_t launch_stream_copy(const void* src, void* dst, size_t bytes, hipStream_t s);
hipError_t launch_lambda_init(ModelId m, Prec p, const KParams& kp, const void* fn,
                              const double* dLdrho, void* lam, double* partK, hipStream_t s);
// mom == nullptr: transposed streaming only (no collision, partA unused).
// mark_state != nullptr: also partM[block] = sum_i mu_i B_i over the block's
// cells, B = mark_state (stored populations, mu the gathered adjoint state).
hipError_t launch_adjoint_step(ModelId m, Prec p, const KParams& kp, const void* lam_src,
                               void* lam_dst, const void* mom, double* partA,
                               const void* mark_state, double* partM, hipStream_t s);
hipError_t launch_dT_init(ModelId m, Prec p, const KParams& kp, const void* lam0,
                          const double* rho, const double* U, const double* T, double* dT,
                          hipStream_t s);
hipError_t launch_sum_partials(const double* part, long long n, int stride, int count,
                               double* out, hipStream_t s);

// The library's static device scratch array (a file-scope __device__ array,
// one copy per GPU, kept until the process ends): its device address on
// `device`, which must be the current device, resolved once per device, and
// its size in bytes.  Used only by lbm_conservation_noalloc.
hipError_t static_scratch(int device, void** ptr, size_t* bytes);

// Sizes used by the API layer for its buffers.
long long step_blocks(ModelId m, Prec p, const KParams& kp);

// The launchers of one model and precision (defined with the kernels in
// lbm_kernels.h, instantiated once per model and precision in its own
// translation unit; the launch_* functions above dispatch to them).
template <class M, Prec P>
struct ModelKernels {
    static hipError_t init(const KParams& kp, const double* rho, const double* U, const double* T,
                           void* f, hipStream_t s);
    static hipError_t set_pop(const KParams& kp, const double* fin, void* f, hipStream_t s);
    static hipError_t get_pop(const KParams& kp, const void* f, double* fout, hipStream_t s);
    static hipError_t step(const KParams& kp, const void* src, void* dst, void* mom_out,
                           hipStream_t s);
    static hipError_t step_aa(const KParams& kp, void* f, bool push, void* mom_out,
                              hipStream_t s);
    static hipError_t to_ab(const KParams& kp, const void* f, void* out, hipStream_t s);
    static hipError_t from_ab(const KParams& kp, const void* f, void* out, hipStream_t s);
    static hipError_t moments(const KParams& kp, const void* f, double* rho, double* U,
                              double* T, hipStream_t s);
    static hipError_t conservation(const KParams& kp, const void* f, double* partials,
                                   hipStream_t s);
    static hipError_t lambda_init(const KParams& kp, const void* fn, const double* dLdrho,
                                  void* lam, double* partK, hipStream_t s);
    static hipError_t adjoint_step(const KParams& kp, const void* lam_src, void* lam_dst,
                                   const void* mom, double* partA, const void* mark_state,
                                   double* partM, hipStream_t s);
    static hipError_t dT_init(const KParams& kp, const void* lam0, const double* rho,
                              const double* U, const double* T, double* dT, hipStream_t s);
};

}  // namespace lbm
