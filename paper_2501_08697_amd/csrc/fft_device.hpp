// Device-side discrete Fourier transforms for the local term of H psi.
//
// Sign convention (the grid transforms of the plane-wave method, Sec. III.A):
// S = +1 is the inverse transform x[j] = sum_k X[k] e^{+2 pi i jk/N} (psi(r)
// from psi(G)), S = -1 the forward one X[k] = sum_j x[j] e^{-2 pi i jk/N}.
// Neither is normalised; the 1/N of the forward grid transform is applied once
// where the result is gathered back onto the sphere.
//
// Two levels:
//  * RegDft<N,S,T>: a length-N DFT held entirely in one thread's registers,
//    natural order in and out. Hand-written butterflies for N = 2, 3, 4, 5 and
//    a compile-time split N = A*B (Cooley-Tukey, twiddles as literals) above.
//  * lds_fft<N,S,...>: many length-N lines resident in LDS, N = A*B with A, B
//    register codelets. Two phases per transform; in each phase a thread owns
//    one (line, sub-index) task and writes only the LDS slots it read, so the
//    only barrier is between the phases. The forward transform takes natural
//    order and leaves frequency k at slot B*(k mod A) + k/A ("digit-permuted");
//    the inverse takes that permuted order and returns natural order. Forward
//    and inverse therefore chain without any reordering pass.
#pragma once

#include "common.hpp"
#include "twiddle_tables.hpp"

namespace apw {

// ------------------------------------------------------------------ splits --
template <int N> struct Split;  // N = A * B, A <= B, both codelet lengths
template <> struct Split<6> { static constexpr int A = 2, B = 3; };
template <> struct Split<8> { static constexpr int A = 2, B = 4; };
template <> struct Split<9> { static constexpr int A = 3, B = 3; };
template <> struct Split<10> { static constexpr int A = 2, B = 5; };
template <> struct Split<12> { static constexpr int A = 3, B = 4; };
template <> struct Split<15> { static constexpr int A = 3, B = 5; };
template <> struct Split<16> { static constexpr int A = 4, B = 4; };

// Splits of the grid lengths into two codelet lengths (LDS level).
template <int N> struct LdsSplit;
#define APW_LDS_SPLIT(n, a, b) \
    template <> struct LdsSplit<n> { static constexpr int A = a, B = b; static_assert(a * b == n, "split"); };
APW_LDS_SPLIT(8, 2, 4)
APW_LDS_SPLIT(12, 3, 4)
APW_LDS_SPLIT(16, 4, 4)
APW_LDS_SPLIT(18, 3, 6)
APW_LDS_SPLIT(20, 4, 5)
APW_LDS_SPLIT(24, 4, 6)
APW_LDS_SPLIT(25, 5, 5)
APW_LDS_SPLIT(27, 3, 9)
APW_LDS_SPLIT(30, 5, 6)
APW_LDS_SPLIT(32, 4, 8)
APW_LDS_SPLIT(36, 6, 6)
APW_LDS_SPLIT(40, 5, 8)
APW_LDS_SPLIT(45, 5, 9)
APW_LDS_SPLIT(48, 6, 8)
APW_LDS_SPLIT(50, 5, 10)
APW_LDS_SPLIT(54, 6, 9)
APW_LDS_SPLIT(60, 6, 10)
APW_LDS_SPLIT(64, 8, 8)
APW_LDS_SPLIT(72, 8, 9)
APW_LDS_SPLIT(75, 5, 15)
APW_LDS_SPLIT(80, 8, 10)
APW_LDS_SPLIT(81, 9, 9)
APW_LDS_SPLIT(90, 9, 10)
APW_LDS_SPLIT(96, 8, 12)
APW_LDS_SPLIT(100, 10, 10)
APW_LDS_SPLIT(108, 9, 12)
APW_LDS_SPLIT(120, 15, 8)
APW_LDS_SPLIT(128, 16, 8)
#undef APW_LDS_SPLIT

// ------------------------------------------------------------ codelets ----
// w = exp(S 2 pi i e / N) from the literal tables; e == 0 is skipped by the
// caller so multiplications by one vanish after unrolling.
template <int N, int S, typename T> __device__ __forceinline__ cx<T> codelet_tw(int e) {
    return cx<T>{static_cast<T>(CodeletTw<N>::c[e]), static_cast<T>(S * CodeletTw<N>::s[e])};
}

template <int N, int S, typename T> struct RegDft {
    static constexpr int A = Split<N>::A, B = Split<N>::B;
    __device__ __forceinline__ static void run(cx<T> *v) {
        cx<T> t[N];
#pragma unroll
        for (int jb = 0; jb < B; ++jb) {
            cx<T> a[A];
#pragma unroll
            for (int ja = 0; ja < A; ++ja) a[ja] = v[jb + B * ja];
            RegDft<A, S, T>::run(a);
#pragma unroll
            for (int ka = 0; ka < A; ++ka) {
                const int e = (jb * ka) % N;
                t[ka * B + jb] = (e == 0) ? a[ka] : cmul(a[ka], codelet_tw<N, S, T>(e));
            }
        }
#pragma unroll
        for (int ka = 0; ka < A; ++ka) {
            cx<T> z[B];
#pragma unroll
            for (int jb = 0; jb < B; ++jb) z[jb] = t[ka * B + jb];
            RegDft<B, S, T>::run(z);
#pragma unroll
            for (int kb = 0; kb < B; ++kb) v[ka + A * kb] = z[kb];
        }
    }
};

template <int S, typename T> struct RegDft<1, S, T> {
    __device__ __forceinline__ static void run(cx<T> *) {}
};

template <int S, typename T> struct RegDft<2, S, T> {
    __device__ __forceinline__ static void run(cx<T> *v) {
        cx<T> a = v[0], b = v[1];
        v[0] = a + b;
        v[1] = a - b;
    }
};

template <int S, typename T> struct RegDft<3, S, T> {
    __device__ __forceinline__ static void run(cx<T> *v) {
        const T h = static_cast<T>(0.8660254037844386);  // sin(2 pi / 3)
        cx<T> t1 = v[1] + v[2], t2 = v[1] - v[2];
        cx<T> m = v[0] - t1 * static_cast<T>(0.5);
        cx<T> r = mul_si<S>(t2 * h);
        v[0] = v[0] + t1;
        v[1] = m + r;
        v[2] = m - r;
    }
};

template <int S, typename T> struct RegDft<4, S, T> {
    __device__ __forceinline__ static void run(cx<T> *v) {
        cx<T> a = v[0] + v[2], b = v[0] - v[2], c = v[1] + v[3], d = mul_si<S>(v[1] - v[3]);
        v[0] = a + c;
        v[2] = a - c;
        v[1] = b + d;
        v[3] = b - d;
    }
};

template <int S, typename T> struct RegDft<5, S, T> {
    __device__ __forceinline__ static void run(cx<T> *v) {
        const T c1 = static_cast<T>(0.30901699437494745);   // cos(2 pi / 5)
        const T c2 = static_cast<T>(-0.8090169943749475);   // cos(4 pi / 5)
        const T s1 = static_cast<T>(0.9510565162951535);    // sin(2 pi / 5)
        const T s2 = static_cast<T>(0.5877852522924731);    // sin(4 pi / 5)
        cx<T> t1 = v[1] + v[4], t2 = v[2] + v[3], t3 = v[1] - v[4], t4 = v[2] - v[3];
        cx<T> x0 = v[0];
        cx<T> a1 = x0 + t1 * c1 + t2 * c2;
        cx<T> a2 = x0 + t1 * c2 + t2 * c1;
        cx<T> b1 = mul_si<S>(t3 * s1 + t4 * s2);
        cx<T> b2 = mul_si<S>(t3 * s2 - t4 * s1);
        v[0] = x0 + t1 + t2;
        v[1] = a1 + b1;
        v[4] = a1 - b1;
        v[2] = a2 + b2;
        v[3] = a2 - b2;
    }
};

// Digit-permuted slot of frequency k for a length-N LDS transform.
template <int N> __host__ __device__ constexpr int perm_slot(int k) {
    return LdsSplit<N>::B * (k % LdsSplit<N>::A) + k / LdsSplit<N>::A;
}

// --------------------------------------------------------------- LDS FFT --
// Transforms `nlines` lines of length N resident in LDS. Element e of line l
// is at lds[base(l) + e * es]. tw[jb * A + ka] = exp(+2 pi i jb ka / N) for
// jb < B, ka < A (the forward transform uses the conjugate). LINES_FAST
// chooses the task order: consecutive threads on consecutive lines (true; use
// when lines are adjacent in memory) or on consecutive sub-indices of one line
// (false; use when a line is contiguous). Ends with a barrier.
template <int N, int S, bool LINES_FAST, typename T, typename Base>
__device__ __forceinline__ void lds_fft(cx<T> *lds, int nlines, Base base, int es, const cx<T> *tw) {
    constexpr int A = LdsSplit<N>::A, B = LdsSplit<N>::B;
    const int tid = threadIdx.x, nthr = blockDim.x;
    if (S < 0) {
        // Phase 1: task (l, jb). a[ja] = x[jb + B ja]; DFT_A; times w^{-jb ka}; back to jb + B ka.
        for (int t = tid; t < nlines * B; t += nthr) {
            const int l = LINES_FAST ? t % nlines : t / B;
            const int jb = LINES_FAST ? t / nlines : t % B;
            cx<T> *p = lds + base(l) + jb * es;
            cx<T> a[A];
#pragma unroll
            for (int ja = 0; ja < A; ++ja) a[ja] = p[B * ja * es];
            RegDft<A, -1, T>::run(a);
            p[0] = a[0];
#pragma unroll
            for (int ka = 1; ka < A; ++ka) {
                cx<T> w = tw[jb * A + ka];
                p[B * ka * es] = cmulc(a[ka], w);
            }
        }
        __syncthreads();
        // Phase 2: task (l, ka). z[jb] = x[B ka + jb]; DFT_B; to slot B ka + kb.
        for (int t = tid; t < nlines * A; t += nthr) {
            const int l = LINES_FAST ? t % nlines : t / A;
            const int ka = LINES_FAST ? t / nlines : t % A;
            cx<T> *p = lds + base(l) + B * ka * es;
            cx<T> z[B];
#pragma unroll
            for (int jb = 0; jb < B; ++jb) z[jb] = p[jb * es];
            RegDft<B, -1, T>::run(z);
#pragma unroll
            for (int kb = 0; kb < B; ++kb) p[kb * es] = z[kb];
        }
        __syncthreads();
    } else {
        // Phase 1: task (l, ka). Z[kb] = x[B ka + kb]; inverse DFT_B; times w^{+jb ka}; back to B ka + jb.
        for (int t = tid; t < nlines * A; t += nthr) {
            const int l = LINES_FAST ? t % nlines : t / A;
            const int ka = LINES_FAST ? t / nlines : t % A;
            cx<T> *p = lds + base(l) + B * ka * es;
            cx<T> z[B];
#pragma unroll
            for (int kb = 0; kb < B; ++kb) z[kb] = p[kb * es];
            RegDft<B, +1, T>::run(z);
            p[0] = z[0];
#pragma unroll
            for (int jb = 1; jb < B; ++jb) p[jb * es] = cmul(z[jb], tw[jb * A + ka]);
        }
        __syncthreads();
        // Phase 2: task (l, jb). a[ka] = x[B ka + jb]; inverse DFT_A; to natural slot jb + B ja.
        for (int t = tid; t < nlines * B; t += nthr) {
            const int l = LINES_FAST ? t % nlines : t / B;
            const int jb = LINES_FAST ? t / nlines : t % B;
            cx<T> *p = lds + base(l) + jb * es;
            cx<T> a[A];
#pragma unroll
            for (int ka = 0; ka < A; ++ka) a[ka] = p[B * ka * es];
            RegDft<A, +1, T>::run(a);
#pragma unroll
            for (int ja = 0; ja < A; ++ja) p[B * ja * es] = a[ja];
        }
        __syncthreads();
    }
}

}  // namespace apw
