// Shared declarations of the HIP library: complex types, status handling,
// per-kernel timing hooks and launch helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "abacus_pw.h"

namespace apw {

// ---------------------------------------------------------------------------
// Complex numbers (interleaved re, im), usable on host and device.
// ---------------------------------------------------------------------------
template <typename T> struct alignas(2 * sizeof(T)) cx {
    T re, im;
};
using z64 = cx<double>;   // complex128
using c32 = cx<float>;    // complex64

template <typename T> __host__ __device__ inline cx<T> mk(T r, T i) { return cx<T>{r, i}; }
template <typename T> __host__ __device__ inline cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> __host__ __device__ inline cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T> __host__ __device__ inline cx<T> operator*(cx<T> a, T s) { return {a.re * s, a.im * s}; }
template <typename T> __host__ __device__ inline cx<T> cmul(cx<T> a, cx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a * conj(b)
template <typename T> __host__ __device__ inline cx<T> cmulc(cx<T> a, cx<T> b) {
    return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
// s * i * a for s = +1 or -1
template <int S, typename T> __host__ __device__ inline cx<T> mul_si(cx<T> a) {
    return S > 0 ? cx<T>{-a.im, a.re} : cx<T>{a.im, -a.re};
}
template <typename TO, typename TI> __host__ __device__ inline cx<TO> cvt(cx<TI> a) {
    return {static_cast<TO>(a.re), static_cast<TO>(a.im)};
}

// ---------------------------------------------------------------------------
// Status handling. Internal functions return int status codes from
// abacus_pw.h; set_error records a message for abacus_pw_last_error.
// ---------------------------------------------------------------------------
int set_error(int code, const std::string &msg);

#define APW_HIP(call)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return ::apw::set_error(ABACUS_PW_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define APW_TRY(expr)                \
    do {                             \
        int s_ = (expr);             \
        if (s_ < 0) return s_;       \
    } while (0)

// ---------------------------------------------------------------------------
// Per-kernel timing (abacus_pw_profile_enable). Launch sites wrap their
// launches in a KernelTimer; when profiling is off it costs one branch.
// ---------------------------------------------------------------------------
void prof_begin(const char *name, hipStream_t s);
void prof_end(hipStream_t s);
// flops (complex products counted as 8 M N K) attributed to the label `name` in the
// current scope, for the kernels enqueued under that label
void prof_count_flops(const char *name, double flops);
extern bool g_prof_on;
// Records made while a ProfScope is alive are labelled "scope:name" (innermost scope;
// a null scope restores plain names), so one kernel can be reported per caller.
extern thread_local const char *t_prof_scope;
struct ProfScope {
    const char *prev;
    explicit ProfScope(const char *scope) : prev(t_prof_scope) { t_prof_scope = scope; }
    ~ProfScope() { t_prof_scope = prev; }
};

struct KernelTimer {
    hipStream_t s;
    KernelTimer(const char *name, hipStream_t st) : s(st) {
        if (g_prof_on) prof_begin(name, s);
    }
    ~KernelTimer() {
        if (g_prof_on) prof_end(s);
    }
};

inline int check_launch(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(ABACUS_PW_EHIP, std::string(what) + ": " + hipGetErrorString(e));
    return ABACUS_PW_OK;
}

inline int ceil_div(int a, int b) { return (a + b - 1) / b; }

// MI355X dispatches consecutive work-groups round-robin over its 8 XCDs, each
// with its own L2. xcd_block() maps the hardware block id of a 3-D grid to a
// logical block id such that logically consecutive blocks run on the same XCD:
// hardware id w runs on XCD w % 8 and takes logical id (w % 8) * (W / 8) + w / 8.
// Blocks beyond the largest multiple of 8 keep their id. Kernels decode the
// logical id with x fastest, so blocks that share operands (consecutive x)
// share an L2.
constexpr int kNumXcd = 8;
__device__ __forceinline__ void xcd_block(int &bx, int &by, int &bz) {
    const int gx = gridDim.x, gy = gridDim.y;
    const int W = gx * gy * gridDim.z;
    const int w = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    const int per = W / kNumXcd;
    const int L = w < per * kNumXcd ? (w % kNumXcd) * per + w / kNumXcd : w;
    bx = L % gx;
    by = (L / gx) % gy;
    bz = L / (gx * gy);
}
inline int64_t ceil_div64(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace apw
