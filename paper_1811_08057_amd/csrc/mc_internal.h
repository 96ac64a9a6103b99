// mc_internal.h -- workspace layouts and kernel launchers behind the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "mc.h"

namespace mc {

constexpr int kMaxRowsPerBlock = 16;
constexpr int64_t kPlainTargetBlocks = 2048;

struct DevState {
    int status;   // kStatus* of the running factorisation
    int bad_step; // first step whose pivot row was zero / non-finite
};

// Device workspace of the plain path (FP64), carved from the caller's
// buffer.  W holds rows 1..n-1 of the matrix being condensed, row stride
// ldw (a multiple of 16 doubles = 128 bytes).
struct PlainWork {
    double* W;
    int64_t ldw;
    double* r[2];    // pivot row / pivot, ping-pong by step parity
    double* piv_val; // pivot of each step
    int* piv_slot;   // slot of each step's pivot in its row
    int* colid;      // original column held by each slot
    int* piv_col;    // optional (caller's, may be null): original column of
                     // each step's pivot
    DevState* state;
};

// Device workspace of the blocked path.  W is the matrix being factored in
// place (row stride ldw); L receives the multipliers of the rows below the
// current panel; the integer arrays track pivot positions and the column
// exchanges.
template <typename T>
struct BlkWork {
    T* W;
    int64_t ldw;
    T* L;          // (n x b), row stride ldl = b
    int64_t ldl;
    int* piv_pos;  // position of each step's pivot in its row (>= step)
    double* piv_val;
    int* perm;     // perm[pos] = original column now at position pos
    int* perm0;    // perm as the panel's first step left it (single-XCD panel)
    int* colsrc;   // source position of each trailing destination position
    int* srcp;     // source position of each panel column s0 + t
    int* moved;    // trailing positions remapped by the previous panel
    // second set of the three above: consecutive panels alternate, so a
    // panel's trailing update can still read its set while the next panel
    // fills the other
    int* colsrc_b;
    int* srcp_b;
    int* moved_b;
    T* dinv;       // inverses of the 16 x 16 diagonal blocks of U11
    int* stepflag; // per panel step: 1 once its pivot row is published
    int* claim;    // [0] panel slot/slice counter, [1] elected XCD, [2] trailing-update tile counter
    // column-split panel: per step parity and slice, a 16-byte pivot
    // candidate record and the candidate's column of the panel rows
    unsigned long long* xrec; // [2][kSplitSlices][2]
    T* xcol;                  // [2][kSplitSlices][kMaxPanel]
    DevState* state;
};

constexpr int64_t kMaxPanel = 128;
constexpr int kSplitSlices = 32; // compute units of one XCD

size_t blocked_workspace_bytes(int64_t n, int dtype, int64_t b);
template <typename T>
BlkWork<T> blocked_carve(void* work, int64_t n, int64_t b,
                         bool with_w = true);
template <typename T>
hipError_t launch_blocked(const T* A, int64_t n, int64_t lda, int64_t b,
                          int update, BlkWork<T> w, mc_result* out,
                          hipStream_t stream, bool factor, bool lookahead,
                          bool serialize = true);

// Column-split panel kernel on (default) or off; returns the previous setting.
int split_panel_set(int on);

size_t plain_workspace_bytes(int64_t n);
PlainWork plain_carve(void* work, int64_t n);
// rule: kRuleMaxAbs (the paper's), kRuleFirstNonzero or kRuleClosestToOne.
hipError_t launch_plain_f64(const double* A, int64_t n, int64_t lda,
                            PlainWork w, mc_result* out, hipStream_t stream,
                            int rule = 0);

// Copy n int32 values on the stream (a kernel, so that graph capture
// records no memory-copy or memset node).
hipError_t launch_copy_i32(int32_t* dst, const int* src, int64_t n,
                           hipStream_t stream);

hipError_t launch_write_result(mc_result* out, double logabsdet, double sign,
                               int64_t info, hipStream_t stream);

// Optional event timing (mc_profile_enable) of two kinds of kernel:
// MC_PROF_UPDATE (the condensation update: the trailing update of the
// blocked path, the per-step loop of the plain path) and MC_PROF_PANEL (the
// panel-chain kernel of the blocked path).
struct ProfMark {
    int slot = -1;
    int kind = 0;
};
ProfMark prof_begin(hipStream_t stream, int kind = MC_PROF_UPDATE);
void prof_end(hipStream_t stream, ProfMark m, int64_t launches,
              double alg_bytes, double alg_flops);

// Workspace of the backward call: Z (n x ldz) holds L^{-1}, then A^{-1}
// before the permuted transpose; ident is the identity column map the
// trailing-update kernel reads.
template <typename T>
struct BwdWork {
    T* Z;
    int64_t ldz;
    int* ident;
    DevState* state;
};

template <typename T>
hipError_t launch_backward(const T* LU, int64_t ld, const int* perm, int64_t n,
                           const double* grad_out, const mc_result* fwd, T* G,
                           int64_t ldg, BwdWork<T> w, hipStream_t st);

// Remember a failing HIP status for mc_last_hip_error(); returns it.
hipError_t note_hip_error(hipError_t e);

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// mc_logdet on a caller-provided workspace with no per-device scheduling
// state: lookahead off, not ordered against other blocked calls, no stream
// or event created.  Same argument checks and numbering as mc_logdet.
mc_status logdet_fixed_work(const void* A, int64_t n, int64_t lda, int dtype,
                            int update, int64_t b, mc_result* out, void* work,
                            size_t work_bytes, void* stream);

} // namespace mc
