// Local-potential term of H psi on the real-space grid (plane-wave KS equation,
// Sec. III.A; V_local of the pseudopotential split, Sec. II.A):
//
//   (V psi)(G) = (1/N) sum_j e^{-iG.r_j} V(r_j) sum_{G'} psi(G') e^{+iG'.r_j}
//
// computed per band as three passes over a pruned grid, all resident in LDS
// while they transform:
//   yz_inv  one work-group per (band, plane m1): scatter the plane's sphere points
//           into an N2 x N3 LDS plane, inverse z transforms on the rows that hold
//           sphere columns, inverse y transforms on every column, store the plane.
//           Only planes m1 in [m1min, m1min + nslab) exist (the "slab").
//   xpass   one work-group per (band, j2): load the slab rows of an N1 x N3 tile,
//           inverse x transform, multiply by V(r), forward x transform, store the
//           slab rows back (in place).
//   yz_fwd  one work-group per (band, plane): forward y, forward z on the column
//           rows, gather the sphere points, write |k+G|^2 psi + (1/N) (V psi).
// HBM traffic per band: psi and H psi once, four passes over the slab
// (nslab * N2 * N3 complex), V once per band tile.
#include "fft_device.hpp"
#include "local.hpp"
#include "plan.hpp"

namespace apw {

template <typename T> __device__ __forceinline__ cx<T> czero() { return cx<T>{T(0), T(0)}; }

int lds_split_host(int n, int *a, int *b);

// A band batch spread over the k-points [k0, k0 + nk) of a call: at every k the
// bands [b0, b0 + bbt) of that k's [nb_total][npw_k] block; off0 = pw_off[k0].
struct BatchArgs {
    int64_t nb_total;
    int64_t off0;
    int b0;
    int bbt;
};

// Block y index -> (k-point, band range inside the batch) for work-groups of bpw bands.
// The planes of one band group are logically consecutive (x = plane), so the
// XCD remap keeps them, and the gathers of that group's psi, on one L2.
__device__ __forceinline__ void batch_block(const KDesc *kd, const BatchArgs &ba, int bpw, KDesc &D, int &k, int &lb0,
                                            int &lb1, int &plane) {
    int by, bz;
    xcd_block(plane, by, bz);
    const int gpk = (ba.bbt + bpw - 1) / bpw;
    k = by / gpk;
    const int g = by - k * gpk;
    D = kd[k];
    lb0 = g * bpw;
    lb1 = min(ba.bbt, lb0 + bpw);
}

constexpr int kMaxT3 = 32;     // widest j3 tile of the x pass
constexpr int kXBands = 4;     // bands per x-pass work-group (FP32)
constexpr int kXBands64 = 8;   // FP64: V is read once per work-group, and 8 bands measured fastest at 72^3 - 128^3
// Threads of a y-z plane work-group. An FP64 plane in LDS allows one group per
// CU, so up to N = 72 it runs 16 waves; larger planes need more registers per
// thread than 1024 threads leave (128 VGPRs), and FP32 planes fit three groups
// of 8 waves per CU, which measured faster than fewer, larger groups.
template <int N, typename T> constexpr int yz_threads() { return sizeof(T) == 8 && N <= 72 ? 1024 : 512; }
constexpr int kYzBandsDefault = 2; // bands per y-z plane work-group

// Copy an N x N plane from LDS to global memory, yz_threads<N, T>() threads, four
// elements per thread in flight (LDS reads first, then the stores).
template <int N, typename T> __device__ __forceinline__ void store_plane(const cx<T> *plane, cx<T> *out, int tid) {
    constexpr int NN = N * N, U = 4, NT = yz_threads<N, T>();
    for (int i0 = tid; i0 < NN; i0 += U * NT) {
        cx<T> v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = plane[min(i0 + u * NT, NN - 1)];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (i0 + u * NT < NN) out[i0 + u * NT] = v[u];
    }
}

// One work-group per (plane s, group of bands). The plane's point list is read
// once into registers; while band b transforms, the sphere values of band b+1
// are already being fetched.
template <int N, typename T, typename TIN>
__global__ __launch_bounds__((yz_threads<N, T>())) void k_yz_inv(const cx<TIN> *__restrict__ psi_all, const KDesc *__restrict__ kd,
                                                       BatchArgs ba, const cx<T> *__restrict__ tw_g,
                                                       cx<T> *__restrict__ slab, int nslab, int bpw) {
    KDesc D;
    int kk, b0, b1;
    int s;
    batch_block(kd, ba, bpw, D, kk, b0, b1, s);
    const int *__restrict__ pt_off = D.pt_off, *__restrict__ pt_g = D.pt_g, *__restrict__ pt_pos = D.pt_pos;
    const int *__restrict__ row_off = D.row_off, *__restrict__ row_list = D.row_list;
    const cx<TIN> *psi = psi_all + ba.nb_total * (D.pw_off - ba.off0) + (int64_t)ba.b0 * D.npw;
    const int64_t ldpsi = D.npw;
    slab += (int64_t)kk * ba.bbt * nslab * (int64_t)(N * N);
    constexpr int MAXP = 4096 / yz_threads<N, T>();   // sphere points per thread held in registers
    extern __shared__ __align__(16) unsigned char smem[];
    cx<T> *plane = reinterpret_cast<cx<T> *>(smem);
    cx<T> *tw = plane + N * N;
    int *rows = reinterpret_cast<int *>(tw + N);   // the plane's z-column rows (times N), read once
    const int tid = threadIdx.x, nthr = blockDim.x;
    for (int i = tid; i < N; i += nthr) tw[i] = tw_g[i];
    const int r0 = row_off[s], nr = row_off[s + 1] - r0;
    for (int i = tid; i < nr; i += nthr) rows[i] = row_list[r0 + i] * N;
    const int p0 = pt_off[s], p1 = pt_off[s + 1];
    // gi = -1 marks an unused slot; gc is a valid index for every slot, so the
    // loads are issued unconditionally (one wait for all of them, not one each)
    int gi[MAXP], gc[MAXP], lp[MAXP];
    cx<TIN> pre[MAXP];
#pragma unroll
    for (int q = 0; q < MAXP; ++q) {
        const int p = p0 + tid + q * nthr;
        const int pc = p1 > p0 ? min(p, p1 - 1) : 0;
        gc[q] = pt_g[pc];
        gi[q] = p < p1 ? gc[q] : -1;
        lp[q] = pt_pos[pc];
    }
#pragma unroll
    for (int q = 0; q < MAXP; ++q) pre[q] = psi[b0 * ldpsi + gc[q]];
    for (int b = b0; b < b1; ++b) {
        for (int i = tid; i < N * N; i += nthr) plane[i] = czero<T>();
        __syncthreads();
#pragma unroll
        for (int q = 0; q < MAXP; ++q)
            if (gi[q] >= 0) plane[lp[q]] = cvt<T>(pre[q]);
        for (int p = p0 + MAXP * nthr + tid; p < p1; p += nthr) plane[pt_pos[p]] = cvt<T>(psi[b * ldpsi + pt_g[p]]);
        __syncthreads();
        if (b + 1 < b1) {
#pragma unroll
            for (int q = 0; q < MAXP; ++q) pre[q] = psi[(b + 1) * ldpsi + gc[q]];
        }
        lds_fft<N, +1, false>(plane, nr, [=](int l) { return rows[l]; }, 1, tw);
        lds_fft<N, +1, true>(plane, N, [](int l) { return l; }, N, tw);
        cx<T> *out = slab + ((int64_t)b * nslab + s) * (int64_t)(N * N);
        store_plane<N>(plane, out, tid);
        __syncthreads();
    }
}

// One work-group per (j2, a tile of T3 consecutive j3 columns, a group of bands):
// inverse x transform, x V(r), forward x transform, with N1 = A B split as in
// lds_fft. Per band and column the work is three thread phases:
//   I  task (c, ka): the B slab values of slots B ka + kb come straight from
//      HBM; inverse DFT_B, twiddle, to LDS.
//   F  task (c, jb): the A values of slots jb + B ka from LDS; inverse DFT_A
//      gives x(j1) at j1 = jb + B ja; times V(j1, j2, j3) (held in registers
//      for the whole band group); forward DFT_A on the same values; twiddle;
//      back to the same LDS slots.
//   O  task (c, ka): slots B ka + jb from LDS; forward DFT_B; the slots that
//      belong to the slab go straight to HBM.
// So each element crosses LDS twice per band (once per transpose) and there
// are three barriers per band. The next band's phase-I values are fetched as
// soon as phase I has consumed the current ones, behind phases F and O. The tile width keeps w3 max(A, B) <= 256,
// so every thread owns at most one task per phase.
template <int N1, typename T, typename TV>
__global__ __launch_bounds__(256) void k_xpass(cx<T> *__restrict__ slab, int nslab, int N2, int N3, int T3, int nt3,
                                               int nbands, int bpw, const int *__restrict__ row_to_slab,
                                               const TV *__restrict__ vloc, const cx<T> *__restrict__ tw_g) {
    constexpr int A = LdsSplit<N1>::A, B = LdsSplit<N1>::B;
    extern __shared__ __align__(16) unsigned char smem[];
    cx<T> *tile = reinterpret_cast<cx<T> *>(smem);       // [N1 slots][T3]
    cx<T> *tw = tile + N1 * T3;
    int *r2s = reinterpret_cast<int *>(tw + N1);
    const int j2 = blockIdx.x / nt3, c0 = (blockIdx.x - j2 * nt3) * T3;
    const int w3 = min(T3, N3 - c0);
    const int b0 = blockIdx.y * bpw, b1 = min(nbands, b0 + bpw);
    const int tid = threadIdx.x;
    const int64_t plane = (int64_t)N2 * N3;
    const int64_t bstride = (int64_t)nslab * plane;
    for (int i = tid; i < N1; i += blockDim.x) {
        tw[i] = tw_g[i];
        r2s[i] = row_to_slab[i];
    }
    __syncthreads();
    // task of this thread in the (c, ka) phases and in the (c, jb) phase
    const int c = w3 > 0 ? tid % w3 : 0;
    const int ka = tid / w3;           // valid when tid < w3 * A
    const int jb = tid / w3;           // valid when tid < w3 * B
    const bool has_ka = tid < w3 * A, has_jb = tid < w3 * B;
    cx<T> *base = slab + (int64_t)j2 * N3 + c0 + c;
    T vr[A];
    int src[B];   // slab offset of each row (< 2^31: at most 128^3 points per band)
#pragma unroll
    for (int ja = 0; ja < A; ++ja)
        vr[ja] = has_jb ? static_cast<T>(vloc[(int64_t)(jb + B * ja) * plane + (int64_t)j2 * N3 + c0 + c]) : T(0);
#pragma unroll
    for (int kb = 0; kb < B; ++kb) {
        const int sl = has_ka ? r2s[B * ka + kb] : -1;
        src[kb] = sl >= 0 ? (int)(sl * plane) : -1;
    }
    // phase-I values in flight: the next band's, and at N1 >= 120 also the one after
    // (there the lines are long and few work-groups fit a CU, so one band of lookahead
    // left the loads exposed; the second costs 32 VGPRs, which the shorter lengths
    // would pay with a wave per SIMD)
    constexpr bool kDeep = N1 >= 120;
    cx<T> pre[B], pre2[kDeep ? B : 1];
#pragma unroll
    for (int kb = 0; kb < B; ++kb) pre[kb] = (has_ka && src[kb] >= 0) ? base[b0 * bstride + src[kb]] : czero<T>();
    if constexpr (kDeep) {
#pragma unroll
        for (int kb = 0; kb < B; ++kb)
            pre2[kb] = (has_ka && src[kb] >= 0 && b0 + 1 < b1) ? base[(b0 + 1) * bstride + src[kb]] : czero<T>();
    }
    for (int b = b0; b < b1; ++b) {
        if (has_ka) {
            cx<T> z[B];
#pragma unroll
            for (int kb = 0; kb < B; ++kb) z[kb] = pre[kb];
            if constexpr (kDeep) {
                // the band after next is fetched now, behind phases F and O of this band and the next
#pragma unroll
                for (int kb = 0; kb < B; ++kb) pre[kb] = pre2[kb];
                if (b + 2 < b1) {
#pragma unroll
                    for (int kb = 0; kb < B; ++kb)
                        if (src[kb] >= 0) pre2[kb] = base[(b + 2) * bstride + src[kb]];
                }
            } else if (b + 1 < b1) {
                // the next band's values are fetched now, behind phases F and O
#pragma unroll
                for (int kb = 0; kb < B; ++kb)
                    if (src[kb] >= 0) pre[kb] = base[(b + 1) * bstride + src[kb]];
            }
            RegDft<B, +1, T>::run(z);
            tile[(B * ka) * T3 + c] = z[0];
#pragma unroll
            for (int q = 1; q < B; ++q) tile[(B * ka + q) * T3 + c] = cmul(z[q], tw[q * A + ka]);
        }
        __syncthreads();
        if (has_jb) {
            cx<T> a[A];
#pragma unroll
            for (int q = 0; q < A; ++q) a[q] = tile[(jb + B * q) * T3 + c];
            RegDft<A, +1, T>::run(a);
#pragma unroll
            for (int q = 0; q < A; ++q) a[q] = a[q] * vr[q];
            RegDft<A, -1, T>::run(a);
            tile[jb * T3 + c] = a[0];
#pragma unroll
            for (int q = 1; q < A; ++q) tile[(jb + B * q) * T3 + c] = cmulc(a[q], tw[jb * A + q]);
        }
        __syncthreads();
        if (has_ka) {
            cx<T> z[B];
#pragma unroll
            for (int q = 0; q < B; ++q) z[q] = tile[(B * ka + q) * T3 + c];
            RegDft<B, -1, T>::run(z);
#pragma unroll
            for (int kb = 0; kb < B; ++kb)
                if (src[kb] >= 0) base[b * bstride + src[kb]] = z[kb];
        }
        __syncthreads();
    }
}

// One work-group per (plane s, group of bands); the next band's plane is
// fetched into registers while the current one transforms, and so is this
// band's psi at the plane's sphere points (whose indices and |k+G|^2 are read
// once for all bands).
template <int N, typename T, typename TIO>
__global__ __launch_bounds__((yz_threads<N, T>())) void k_yz_fwd(const cx<T> *__restrict__ slab, int nslab,
                                                       const KDesc *__restrict__ kd, BatchArgs ba,
                                                       const cx<T> *__restrict__ tw_g, const cx<TIO> *__restrict__ psi_all,
                                                       cx<TIO> *__restrict__ hpsi_all, double inv_n, int bpw) {
    KDesc D;
    int kk, b0, b1;
    int s;
    batch_block(kd, ba, bpw, D, kk, b0, b1, s);
    const int *__restrict__ pt_off = D.pt_off, *__restrict__ pt_g = D.pt_g, *__restrict__ pt_pos = D.pt_pos;
    const int *__restrict__ row_off = D.row_off, *__restrict__ row_list = D.row_list;
    const double *__restrict__ kin = D.kin;
    const int64_t koff = ba.nb_total * (D.pw_off - ba.off0) + (int64_t)ba.b0 * D.npw;
    const cx<TIO> *psi = psi_all + koff;
    cx<TIO> *hpsi = hpsi_all + koff;
    const int64_t ld = D.npw;
    slab += (int64_t)kk * ba.bbt * nslab * (int64_t)(N * N);
    constexpr int NT = yz_threads<N, T>();
    constexpr int MAXQ = (N * N + NT - 1) / NT;
    extern __shared__ __align__(16) unsigned char smem[];
    cx<T> *plane = reinterpret_cast<cx<T> *>(smem);
    cx<T> *tw = plane + N * N;
    int *rows = reinterpret_cast<int *>(tw + N);   // the plane's z-column rows (times N), read once
    const int tid = threadIdx.x, nthr = blockDim.x;
    for (int i = tid; i < N; i += nthr) tw[i] = tw_g[i];
    const int r0 = row_off[s], nr = row_off[s + 1] - r0;
    for (int i = tid; i < nr; i += nthr) rows[i] = row_list[r0 + i] * N;
    cx<T> pre[MAXQ];
    {
        const cx<T> *in = slab + ((int64_t)b0 * nslab + s) * (int64_t)(N * N);
#pragma unroll
        for (int q = 0; q < MAXQ; ++q) {
            const int i = tid + q * NT;
            pre[q] = i < N * N ? in[i] : czero<T>();
        }
    }
    const int p0 = pt_off[s], p1 = pt_off[s + 1];
    const TIO sc = static_cast<TIO>(inv_n);
    // the plane's first MAXP * nthr sphere points: index, LDS slot and |k+G|^2
    // held in registers for every band (clamped to point 0 where a slot is unused)
    constexpr int MAXP = 4;
    int gi[MAXP], lp[MAXP];
    TIO kq[MAXP];
#pragma unroll
    for (int q = 0; q < MAXP; ++q) {
        const int p = min(p0 + tid + q * nthr, p1 - 1);
        gi[q] = p >= p0 ? pt_g[p] : 0;
        lp[q] = p >= p0 ? pt_pos[p] : 0;
    }
#pragma unroll
    for (int q = 0; q < MAXP; ++q) kq[q] = static_cast<TIO>(kin[gi[q]]);
    for (int b = b0; b < b1; ++b) {
#pragma unroll
        for (int q = 0; q < MAXQ; ++q) {
            const int i = tid + q * NT;
            if (i < N * N) plane[i] = pre[q];
        }
        __syncthreads();
        const cx<TIO> *x = psi + b * ld;
        cx<TIO> *y = hpsi + b * ld;
        cx<TIO> xq[MAXP];   // this band's psi at the thread's points, fetched behind the transforms
#pragma unroll
        for (int q = 0; q < MAXP; ++q) xq[q] = x[gi[q]];
        if (b + 1 < b1) {
            const cx<T> *in = slab + ((int64_t)(b + 1) * nslab + s) * (int64_t)(N * N);
#pragma unroll
            for (int q = 0; q < MAXQ; ++q) {
                const int i = tid + q * NT;
                if (i < N * N) pre[q] = in[i];
            }
        }
        lds_fft<N, -1, true>(plane, N, [](int l) { return l; }, N, tw);
        lds_fft<N, -1, false>(plane, nr, [=](int l) { return rows[l]; }, 1, tw);
#pragma unroll
        for (int q = 0; q < MAXP; ++q)
            if (p0 + tid + q * nthr < p1) {
                const cx<TIO> v = cvt<TIO>(plane[lp[q]]);
                y[gi[q]] = cx<TIO>{kq[q] * xq[q].re + sc * v.re, kq[q] * xq[q].im + sc * v.im};
            }
        for (int p = p0 + MAXP * nthr + tid; p < p1; p += nthr) {
            const int g = pt_g[p];
            const cx<TIO> v = cvt<TIO>(plane[pt_pos[p]]);
            const TIO kg = static_cast<TIO>(kin[g]);
            const cx<TIO> xg = x[g];
            y[g] = cx<TIO>{kg * xg.re + sc * v.re, kg * xg.im + sc * v.im};
        }
        __syncthreads();
    }
}

// Compact-row variants of the plane passes for planes too large for LDS (and
// for higher occupancy): only the nr rows of the plane that hold sphere columns
// are kept in LDS (rows[r][j3], r = position in the plane's row list); the y
// transforms run through an N2 x C chunk buffer, C consecutive j3 at a time.
// The two phases of each chunk's y transform are written out here rather than
// taken from lds_fft, so that they read and write the compact rows and the slab
// themselves: the inverse's first phase takes its inputs from the compact rows
// (slots without a row are zero) and its second phase stores the natural-order
// outputs to the slab; the forward's second phase writes the slots that have a
// row straight into the compact rows. A chunk then costs two (inverse) or three
// (forward) barriers instead of five and four, and no zero or copy passes.
// These planes leave room for one work-group per CU, so nothing else on the CU
// covers a global load's latency: both kernels keep the next loads in flight
// behind the current work (the next band's sphere values in the inverse pass;
// the next chunk's slab values and this band's psi in the forward pass).
template <int N, typename T, typename TIN, int NT>
__global__ __launch_bounds__(NT) void k_yz_inv_c(const cx<TIN> *__restrict__ psi_all, const KDesc *__restrict__ kd,
                                                 BatchArgs ba, const cx<T> *__restrict__ tw_g,
                                                 cx<T> *__restrict__ slab, int nslab, int bpw, int rows_max, int C) {
    KDesc D;
    int kk, b0, b1;
    int s;
    batch_block(kd, ba, bpw, D, kk, b0, b1, s);
    const int *__restrict__ pt_off = D.pt_off, *__restrict__ pt_g = D.pt_g, *__restrict__ pt_pos = D.pt_pos;
    const int *__restrict__ row_off = D.row_off, *__restrict__ row_list = D.row_list;
    const cx<TIN> *psi = psi_all + ba.nb_total * (D.pw_off - ba.off0) + (int64_t)ba.b0 * D.npw;
    const int64_t ldpsi = D.npw;
    slab += (int64_t)kk * ba.bbt * nslab * (int64_t)(N * N);
    extern __shared__ __align__(16) unsigned char smem[];
    cx<T> *rows = reinterpret_cast<cx<T> *>(smem);
    cx<T> *ybuf = rows + rows_max * N;
    cx<T> *tw = ybuf + N * C;
    int *map = reinterpret_cast<int *>(tw + N);
    const int tid = threadIdx.x;
    const int r0 = row_off[s], nr = row_off[s + 1] - r0;
    const int p0 = pt_off[s], p1 = pt_off[s + 1];
    constexpr int A = LdsSplit<N>::A, B = LdsSplit<N>::B;
    for (int i = tid; i < N; i += NT) {
        tw[i] = tw_g[i];
        map[i] = -1;
    }
    __syncthreads();
    for (int r = tid; r < nr; r += NT) map[row_list[r0 + r]] = r;
    // the plane's first MAXP * NT sphere points: psi index and compact-row LDS position,
    // held in registers for every band (point p1 - 1 stands in for unused slots); fewer
    // per thread at 1024 threads, whose FP64 transforms leave no registers for more
    constexpr int MAXP = NT >= 1024 ? (sizeof(T) == 8 && N >= 128 ? 0 : 1) : 4;
    int gc[MAXP > 0 ? MAXP : 1], pos[MAXP > 0 ? MAXP : 1];
#pragma unroll
    for (int q = 0; q < MAXP; ++q) {
        const int p = p1 > p0 ? min(p0 + tid + q * NT, p1 - 1) : 0;
        gc[q] = pt_g[p];
        pos[q] = pt_pos[p];
    }
    cx<TIN> pre[MAXP > 0 ? MAXP : 1];
#pragma unroll
    for (int q = 0; q < MAXP; ++q) pre[q] = psi[b0 * ldpsi + gc[q]];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < MAXP; ++q) {
        const int slot = pos[q] / N;
        pos[q] = p0 + tid + q * NT < p1 ? map[slot] * N + (pos[q] - slot * N) : -1;
    }
    for (int b = b0; b < b1; ++b) {
        for (int i = tid; i < nr * N; i += NT) rows[i] = czero<T>();
        __syncthreads();
#pragma unroll
        for (int q = 0; q < MAXP; ++q)
            if (pos[q] >= 0) rows[pos[q]] = cvt<T>(pre[q]);
        for (int p = p0 + MAXP * NT + tid; p < p1; p += NT) {
            const int ps = pt_pos[p], slot = ps / N;
            rows[map[slot] * N + (ps - slot * N)] = cvt<T>(psi[b * ldpsi + pt_g[p]]);
        }
        __syncthreads();
        if (b + 1 < b1) {
#pragma unroll
            for (int q = 0; q < MAXP; ++q) pre[q] = psi[(b + 1) * ldpsi + gc[q]];
        }
        lds_fft<N, +1, false>(rows, nr, [](int l) { return l * N; }, 1, tw);
        cx<T> *out = slab + ((int64_t)b * nslab + s) * (int64_t)(N * N);
        for (int c0 = 0; c0 < N; c0 += C) {
            const int w = min(C, N - c0);
            // phase 1, task (c, ka): slots B ka + kb of column c0 + c from the compact rows,
            // inverse DFT_B, twiddle, to ybuf slots B ka + jb
            for (int t = tid; t < w * A; t += NT) {
                const int c = t % w, ka = t / w;
                cx<T> z[B];
#pragma unroll
                for (int kb = 0; kb < B; ++kb) {
                    const int r = map[B * ka + kb];
                    z[kb] = r >= 0 ? rows[r * N + c0 + c] : czero<T>();
                }
                RegDft<B, +1, T>::run(z);
                ybuf[(B * ka) * C + c] = z[0];
#pragma unroll
                for (int jb = 1; jb < B; ++jb) ybuf[(B * ka + jb) * C + c] = cmul(z[jb], tw[jb * A + ka]);
            }
            __syncthreads();
            // phase 2, task (c, jb): inverse DFT_A of slots B ka + jb; j2 = jb + B ja goes to the slab
            for (int t = tid; t < w * B; t += NT) {
                const int c = t % w, jb = t / w;
                cx<T> a[A];
#pragma unroll
                for (int ka = 0; ka < A; ++ka) a[ka] = ybuf[(B * ka + jb) * C + c];
                RegDft<A, +1, T>::run(a);
#pragma unroll
                for (int ja = 0; ja < A; ++ja) out[(jb + B * ja) * N + c0 + c] = a[ja];
            }
            __syncthreads();
        }
    }
}

template <int N, typename T, typename TIO, int NT>
__global__ __launch_bounds__(NT) void k_yz_fwd_c(const cx<T> *__restrict__ slab, int nslab,
                                                 const KDesc *__restrict__ kd, BatchArgs ba,
                                                 const cx<T> *__restrict__ tw_g, const cx<TIO> *__restrict__ psi_all,
                                                 cx<TIO> *__restrict__ hpsi_all, double inv_n, int bpw, int rows_max,
                                                 int C) {
    KDesc D;
    int kk, b0, b1;
    int s;
    batch_block(kd, ba, bpw, D, kk, b0, b1, s);
    const int *__restrict__ pt_off = D.pt_off, *__restrict__ pt_g = D.pt_g, *__restrict__ pt_pos = D.pt_pos;
    const int *__restrict__ row_off = D.row_off, *__restrict__ row_list = D.row_list;
    const double *__restrict__ kin = D.kin;
    const int64_t koff = ba.nb_total * (D.pw_off - ba.off0) + (int64_t)ba.b0 * D.npw;
    const cx<TIO> *psi = psi_all + koff;
    cx<TIO> *hpsi = hpsi_all + koff;
    const int64_t ld = D.npw;
    slab += (int64_t)kk * ba.bbt * nslab * (int64_t)(N * N);
    extern __shared__ __align__(16) unsigned char smem[];
    cx<T> *rows = reinterpret_cast<cx<T> *>(smem);
    cx<T> *ybuf = rows + rows_max * N;
    cx<T> *tw = ybuf + N * C;
    int *map = reinterpret_cast<int *>(tw + N);
    const int tid = threadIdx.x;
    const int r0 = row_off[s], nr = row_off[s + 1] - r0;
    const int p0 = pt_off[s], p1 = pt_off[s + 1];
    const TIO sc = static_cast<TIO>(inv_n);
    constexpr int A = LdsSplit<N>::A, B = LdsSplit<N>::B;
    for (int i = tid; i < N; i += NT) {
        tw[i] = tw_g[i];
        map[i] = -1;
    }
    __syncthreads();
    for (int r = tid; r < nr; r += NT) map[row_list[r0 + r]] = r;
    // slab values of one chunk (N2 x w): the first MAXQ per thread are fetched ahead
    constexpr int MAXQ = NT >= 1024 ? 1 : 4;
    const int nchunk = (N + C - 1) / C;
    cx<T> pre[MAXQ];
    // slab index of the thread's q-th value of chunk ci of band b (-1: none); a plain
    // function of registers, so the prefetch array stays in registers
    auto src_of = [=](int b, int ci, int q) -> int64_t {
        const int c0 = ci * C, w = min(C, N - c0), i = tid + q * NT;
        if (i >= N * w) return -1;
        const int j2 = i / w, c = i - j2 * w;
        return ((int64_t)b * nslab + s) * (int64_t)(N * N) + j2 * N + c0 + c;
    };
#pragma unroll
    for (int q = 0; q < MAXQ; ++q) {
        const int64_t o = src_of(b0, 0, q);
        pre[q] = o >= 0 ? slab[o] : czero<T>();
    }
    // the plane's first MAXP * NT sphere points: psi index and compact-row position
    constexpr int MAXP = NT >= 1024 ? 1 : 4;
    int gi[MAXP], pos[MAXP];
#pragma unroll
    for (int q = 0; q < MAXP; ++q) {
        const int p = p1 > p0 ? min(p0 + tid + q * NT, p1 - 1) : 0;
        gi[q] = pt_g[p];
        pos[q] = pt_pos[p];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < MAXP; ++q) {
        const int slot = pos[q] / N;
        pos[q] = p0 + tid + q * NT < p1 ? map[slot] * N + (pos[q] - slot * N) : -1;
    }
    for (int b = b0; b < b1; ++b) {
        const cx<TIO> *x = psi + b * ld;
        cx<TIO> *y = hpsi + b * ld;
        const cx<T> *in = slab + ((int64_t)b * nslab + s) * (int64_t)(N * N);
        for (int ci = 0; ci < nchunk; ++ci) {
            const int c0 = ci * C, w = min(C, N - c0);
#pragma unroll
            for (int q = 0; q < MAXQ; ++q) {
                const int i = tid + q * NT;
                if (i < N * w) ybuf[(i / w) * C + (i % w)] = pre[q];
            }
            for (int i = tid + MAXQ * NT; i < N * w; i += NT) {
                const int j2 = i / w, c = i - j2 * w;
                ybuf[j2 * C + c] = in[j2 * N + c0 + c];
            }
            __syncthreads();
            // the next chunk (or the next band's first chunk) is fetched behind this one
            const int nb_ = ci + 1 < nchunk ? b : b + 1, nc_ = ci + 1 < nchunk ? ci + 1 : 0;
#pragma unroll
            for (int q = 0; q < MAXQ; ++q) {
                const int64_t o = nb_ < b1 ? src_of(nb_, nc_, q) : -1;
                pre[q] = o >= 0 ? slab[o] : czero<T>();
            }
            // phase 1, task (c, jb): forward DFT_A of natural j2 = jb + B ja, twiddle, back in place
            for (int t = tid; t < w * B; t += NT) {
                const int c = t % w, jb = t / w;
                cx<T> a[A];
#pragma unroll
                for (int ja = 0; ja < A; ++ja) a[ja] = ybuf[(jb + B * ja) * C + c];
                RegDft<A, -1, T>::run(a);
                ybuf[jb * C + c] = a[0];
#pragma unroll
                for (int ka = 1; ka < A; ++ka) ybuf[(jb + B * ka) * C + c] = cmulc(a[ka], tw[jb * A + ka]);
            }
            __syncthreads();
            // phase 2, task (c, ka): forward DFT_B of slots B ka + jb; output slot B ka + kb
            // goes to its compact row when the plane has one there
            for (int t = tid; t < w * A; t += NT) {
                const int c = t % w, ka = t / w;
                cx<T> z[B];
#pragma unroll
                for (int jb = 0; jb < B; ++jb) z[jb] = ybuf[(B * ka + jb) * C + c];
                RegDft<B, -1, T>::run(z);
#pragma unroll
                for (int kb = 0; kb < B; ++kb) {
                    const int r = map[B * ka + kb];
                    if (r >= 0) rows[r * N + c0 + c] = z[kb];
                }
            }
            __syncthreads();
        }
        // this band's psi and |k+G|^2 at the thread's points, fetched behind the z transforms
        cx<TIO> xq[MAXP];
        TIO kq[MAXP];
#pragma unroll
        for (int q = 0; q < MAXP; ++q) {
            xq[q] = x[gi[q]];
            kq[q] = static_cast<TIO>(kin[gi[q]]);
        }
        lds_fft<N, -1, false>(rows, nr, [](int l) { return l * N; }, 1, tw);
#pragma unroll
        for (int q = 0; q < MAXP; ++q)
            if (pos[q] >= 0) {
                const cx<TIO> v = cvt<TIO>(rows[pos[q]]);
                y[gi[q]] = cx<TIO>{kq[q] * xq[q].re + sc * v.re, kq[q] * xq[q].im + sc * v.im};
            }
        for (int p = p0 + MAXP * NT + tid; p < p1; p += NT) {
            const int g = pt_g[p], ps = pt_pos[p], slot = ps / N;
            const cx<TIO> v = cvt<TIO>(rows[map[slot] * N + (ps - slot * N)]);
            const TIO kg = static_cast<TIO>(kin[g]);
            const cx<TIO> xg = x[g];
            y[g] = cx<TIO>{kg * xg.re + sc * v.re, kg * xg.im + sc * v.im};
        }
        __syncthreads();
    }
}

template <int N, typename T, typename TIO, int NT>
__global__ __launch_bounds__(NT) void k_yz_fwd_d(const cx<T> *__restrict__ slab, int nslab,
                                                 const KDesc *__restrict__ kd, BatchArgs ba,
                                                 const cx<T> *__restrict__ tw_g, const cx<TIO> *__restrict__ psi_all,
                                                 cx<TIO> *__restrict__ hpsi_all, double inv_n, int bpw, int rows_max,
                                                 int C) {
    KDesc D;
    int kk, b0, b1;
    int s;
    batch_block(kd, ba, bpw, D, kk, b0, b1, s);
    const int *__restrict__ pt_off = D.pt_off, *__restrict__ pt_g = D.pt_g, *__restrict__ pt_pos = D.pt_pos;
    const int *__restrict__ row_off = D.row_off, *__restrict__ row_list = D.row_list;
    const double *__restrict__ kin = D.kin;
    const int64_t koff = ba.nb_total * (D.pw_off - ba.off0) + (int64_t)ba.b0 * D.npw;
    const cx<TIO> *psi = psi_all + koff;
    cx<TIO> *hpsi = hpsi_all + koff;
    const int64_t ld = D.npw;
    slab += (int64_t)kk * ba.bbt * nslab * (int64_t)(N * N);
    extern __shared__ __align__(16) unsigned char smem[];
    cx<T> *rows = reinterpret_cast<cx<T> *>(smem);
    cx<T> *ybuf = rows + rows_max * N;
    cx<T> *tw = ybuf + N * C;
    int *map = reinterpret_cast<int *>(tw + N);
    const int tid = threadIdx.x;
    const int r0 = row_off[s], nr = row_off[s + 1] - r0;
    const int p0 = pt_off[s], p1 = pt_off[s + 1];
    const TIO sc = static_cast<TIO>(inv_n);
    constexpr int A = LdsSplit<N>::A, B = LdsSplit<N>::B;
    for (int i = tid; i < N; i += NT) {
        tw[i] = tw_g[i];
        map[i] = -1;
    }
    __syncthreads();
    for (int r = tid; r < nr; r += NT) map[row_list[r0 + r]] = r;
    // the first phase of each chunk's forward y transform (task (c, jb): the A values at
    // j2 = jb + B ja of column c0 + c) loads its values straight from the slab; the next
    // chunk's (or the next band's first chunk's) are fetched while this one transforms
    const int nchunk = (N + C - 1) / C;
    cx<T> pre[A];
    // slab offset of this thread's phase-1 column in chunk ci of band b (-1: no task)
    auto col_of = [=](int b, int ci) -> int64_t {
        const int c0 = ci * C, w = min(C, N - c0);
        if (tid >= w * B) return -1;
        const int c = tid % w, jb = tid / w;
        return ((int64_t)b * nslab + s) * (int64_t)(N * N) + jb * N + c0 + c;
    };
    {
        const int64_t o = col_of(b0, 0);
#pragma unroll
        for (int ja = 0; ja < A; ++ja) pre[ja] = o >= 0 ? slab[o + (int64_t)B * ja * N] : czero<T>();
    }
    // the plane's first MAXP * NT sphere points: psi index and compact-row position
    constexpr int MAXP = NT >= 1024 ? 1 : 4;
    int gi[MAXP], pos[MAXP];
#pragma unroll
    for (int q = 0; q < MAXP; ++q) {
        const int p = p1 > p0 ? min(p0 + tid + q * NT, p1 - 1) : 0;
        gi[q] = pt_g[p];
        pos[q] = pt_pos[p];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < MAXP; ++q) {
        const int slot = pos[q] / N;
        pos[q] = p0 + tid + q * NT < p1 ? map[slot] * N + (pos[q] - slot * N) : -1;
    }
    for (int b = b0; b < b1; ++b) {
        const cx<TIO> *x = psi + b * ld;
        cx<TIO> *y = hpsi + b * ld;
        for (int ci = 0; ci < nchunk; ++ci) {
            const int c0 = ci * C, w = min(C, N - c0);
            // phase 1, task (c, jb): forward DFT_A of natural j2 = jb + B ja, twiddle, to ybuf
            // (one task per thread: w B <= C B <= NT, checked by the launcher)
            if (tid < w * B) {
                const int c = tid % w, jb = tid / w;
                cx<T> a[A];
#pragma unroll
                for (int ja = 0; ja < A; ++ja) a[ja] = pre[ja];
                const int nb_ = ci + 1 < nchunk ? b : b + 1, nc_ = ci + 1 < nchunk ? ci + 1 : 0;
                const int64_t o = nb_ < b1 ? col_of(nb_, nc_) : -1;
#pragma unroll
                for (int ja = 0; ja < A; ++ja) pre[ja] = o >= 0 ? slab[o + (int64_t)B * ja * N] : czero<T>();
                RegDft<A, -1, T>::run(a);
                ybuf[jb * C + c] = a[0];
#pragma unroll
                for (int ka = 1; ka < A; ++ka) ybuf[(jb + B * ka) * C + c] = cmulc(a[ka], tw[jb * A + ka]);
            } else if (ci + 1 == nchunk && b + 1 < b1) {
                // threads without a task in this chunk may have one in the next band's first chunk
                const int64_t o = col_of(b + 1, 0);
#pragma unroll
                for (int ja = 0; ja < A; ++ja) pre[ja] = o >= 0 ? slab[o + (int64_t)B * ja * N] : czero<T>();
            }
            __syncthreads();
            // phase 2, task (c, ka): forward DFT_B of slots B ka + jb; output slot B ka + kb
            // goes to its compact row when the plane has one there
            for (int t = tid; t < w * A; t += NT) {
                const int c = t % w, ka = t / w;
                cx<T> z[B];
#pragma unroll
                for (int jb = 0; jb < B; ++jb) z[jb] = ybuf[(B * ka + jb) * C + c];
                RegDft<B, -1, T>::run(z);
#pragma unroll
                for (int kb = 0; kb < B; ++kb) {
                    const int r = map[B * ka + kb];
                    if (r >= 0) rows[r * N + c0 + c] = z[kb];
                }
            }
            __syncthreads();
        }
        // this band's psi and |k+G|^2 at the thread's points, fetched behind the z transforms
        cx<TIO> xq[MAXP];
        TIO kq[MAXP];
#pragma unroll
        for (int q = 0; q < MAXP; ++q) {
            xq[q] = x[gi[q]];
            kq[q] = static_cast<TIO>(kin[gi[q]]);
        }
        lds_fft<N, -1, false>(rows, nr, [](int l) { return l * N; }, 1, tw);
#pragma unroll
        for (int q = 0; q < MAXP; ++q)
            if (pos[q] >= 0) {
                const cx<TIO> v = cvt<TIO>(rows[pos[q]]);
                y[gi[q]] = cx<TIO>{kq[q] * xq[q].re + sc * v.re, kq[q] * xq[q].im + sc * v.im};
            }
        for (int p = p0 + MAXP * NT + tid; p < p1; p += NT) {
            const int g = pt_g[p], ps = pt_pos[p], slot = ps / N;
            const cx<TIO> v = cvt<TIO>(rows[map[slot] * N + (ps - slot * N)]);
            const TIO kg = static_cast<TIO>(kin[g]);
            const cx<TIO> xg = x[g];
            y[g] = cx<TIO>{kg * xg.re + sc * v.re, kg * xg.im + sc * v.im};
        }
        __syncthreads();
    }
}

// Adjoint of the local term with respect to V: for one (j2, j3 tile) and the
// contiguous band range [g bpw, (g + 1) bpw) of the batch, inverse x transforms
// of the psi and dY planes and acc(r) += Re(conj(gamma_b(r)) psi_b(r)); part[g]
// holds the running sum (overwritten when first != 0). The transform is the
// two-level one of k_density_x, applied to the sequence psi_bs, dY_bs,
// psi_bs+1, ...: each source's phase-I values are fetched while the previous
// source transforms, and psi's real-space values wait in registers for dY's.
// Bands are summed in a fixed order.
template <int N1, typename T>
__global__ __launch_bounds__(256) void k_gradv_x(const cx<T> *__restrict__ slab_x, const cx<T> *__restrict__ slab_y,
                                                 int nslab, int N2, int N3, int T3, int nt3, int nbands, int bpw,
                                                 const int *__restrict__ row_to_slab, const cx<T> *__restrict__ tw_g,
                                                 double *__restrict__ part, int first) {
    constexpr int A = LdsSplit<N1>::A, B = LdsSplit<N1>::B;
    extern __shared__ __align__(16) unsigned char smem[];
    cx<T> *tile = reinterpret_cast<cx<T> *>(smem);       // [N1 slots][T3]
    cx<T> *tw = tile + N1 * T3;
    int *r2s = reinterpret_cast<int *>(tw + N1);
    const int j2 = blockIdx.x / nt3, c0 = (blockIdx.x - j2 * nt3) * T3;
    const int w3 = min(T3, N3 - c0);
    const int g = blockIdx.y, bs = g * bpw, be = min(nbands, bs + bpw);
    const int tid = threadIdx.x;
    const int64_t plane = (int64_t)N2 * N3;
    const int64_t bstride = (int64_t)nslab * plane;
    for (int i = tid; i < N1; i += blockDim.x) {
        tw[i] = tw_g[i];
        r2s[i] = row_to_slab[i];
    }
    __syncthreads();
    const int c = w3 > 0 ? tid % w3 : 0;
    const int ka = tid / w3, jb = tid / w3;
    const bool has_ka = tid < w3 * A, has_jb = tid < w3 * B;
    const int64_t col = (int64_t)j2 * N3 + c0 + c;
    int src[B];   // slab offset of each row (< 2^31: at most 128^3 points per band)
#pragma unroll
    for (int kb = 0; kb < B; ++kb) {
        const int sl = has_ka ? r2s[B * ka + kb] : -1;
        src[kb] = sl >= 0 ? (int)(sl * plane) : -1;
    }
    // source t: psi (t even) or dY (t odd) of band bs + t / 2
    const int nt = 2 * max(0, be - bs);
    auto source = [&](int t) { return ((t & 1) ? slab_y : slab_x) + (int64_t)(bs + (t >> 1)) * bstride + col; };
    double acc[A];
    cx<T> xr[A];
#pragma unroll
    for (int q = 0; q < A; ++q) {
        acc[q] = 0.0;
        xr[q] = czero<T>();
    }
    cx<T> pre[B];
    {
        const cx<T> *p0 = source(0);
#pragma unroll
        for (int kb = 0; kb < B; ++kb) pre[kb] = (has_ka && src[kb] >= 0 && nt > 0) ? p0[src[kb]] : czero<T>();
    }
    for (int t = 0; t < nt; ++t) {
        if (has_ka) {
            cx<T> z[B];
#pragma unroll
            for (int kb = 0; kb < B; ++kb) z[kb] = pre[kb];
            if (t + 1 < nt) {
                const cx<T> *pn = source(t + 1);
#pragma unroll
                for (int kb = 0; kb < B; ++kb)
                    if (src[kb] >= 0) pre[kb] = pn[src[kb]];
            }
            RegDft<B, +1, T>::run(z);
            tile[(B * ka) * T3 + c] = z[0];
#pragma unroll
            for (int q = 1; q < B; ++q) tile[(B * ka + q) * T3 + c] = cmul(z[q], tw[q * A + ka]);
        }
        __syncthreads();
        if (has_jb) {
            cx<T> a[A];
#pragma unroll
            for (int q = 0; q < A; ++q) a[q] = tile[(jb + B * q) * T3 + c];
            RegDft<A, +1, T>::run(a);
            if ((t & 1) == 0) {
#pragma unroll
                for (int q = 0; q < A; ++q) xr[q] = a[q];
            } else {
#pragma unroll
                for (int q = 0; q < A; ++q)
                    acc[q] += (double)a[q].re * (double)xr[q].re + (double)a[q].im * (double)xr[q].im;
            }
        }
        __syncthreads();
    }
    if (has_jb) {
#pragma unroll
        for (int q = 0; q < A; ++q) {
            double *o = part + (int64_t)g * N1 * plane + (int64_t)(jb + B * q) * plane + col;
            *o = first ? acc[q] : *o + acc[q];
        }
    }
}

// Band density: for one (j2, j3 tile) and the contiguous band range
// [g bpw, (g + 1) bpw) of the batch, inverse x transforms of the psi planes
// and acc(r) += w_b |psi_b(r)|^2, w_b = occ[k][b0 + b] for the virtual band
// (k, b); part[g] holds the running sum (overwritten when first != 0). The
// transform is the two-level one of k_xpass without its forward half: phase I
// takes the B values of slots B ka + kb from HBM, inverse DFT_B, twiddle, to
// LDS; phase F takes the A values of slots jb + B q, inverse DFT_A gives
// psi(j1) at j1 = jb + B q, and the thread adds w |psi|^2 into its registers
// for those A points. The next band's phase-I values are fetched as soon as
// phase I has consumed the current ones; two barriers per band. Bands are
// summed in a fixed order.
template <int N1, typename T>
__global__ __launch_bounds__(256) void k_density_x(const cx<T> *__restrict__ slab, int nslab, int N2, int N3, int T3,
                                                   int nt3, int nbands, int bpw, const int *__restrict__ row_to_slab,
                                                   const cx<T> *__restrict__ tw_g, const double *__restrict__ occ,
                                                   int nb, int b0, int bbt, double *__restrict__ part, int first) {
    constexpr int A = LdsSplit<N1>::A, B = LdsSplit<N1>::B;
    extern __shared__ __align__(16) unsigned char smem[];
    cx<T> *tile = reinterpret_cast<cx<T> *>(smem);       // [N1 slots][T3]
    cx<T> *tw = tile + N1 * T3;
    int *r2s = reinterpret_cast<int *>(tw + N1);
    const int j2 = blockIdx.x / nt3, c0 = (blockIdx.x - j2 * nt3) * T3;
    const int w3 = min(T3, N3 - c0);
    const int g = blockIdx.y, bs = g * bpw, be = min(nbands, bs + bpw);
    const int tid = threadIdx.x;
    const int64_t plane = (int64_t)N2 * N3;
    const int64_t bstride = (int64_t)nslab * plane;
    for (int i = tid; i < N1; i += blockDim.x) {
        tw[i] = tw_g[i];
        r2s[i] = row_to_slab[i];
    }
    __syncthreads();
    const int c = w3 > 0 ? tid % w3 : 0;
    const int ka = tid / w3, jb = tid / w3;
    const bool has_ka = tid < w3 * A, has_jb = tid < w3 * B;
    const cx<T> *base = slab + (int64_t)j2 * N3 + c0 + c;
    int src[B];   // slab offset of each row (< 2^31: at most 128^3 points per band)
#pragma unroll
    for (int kb = 0; kb < B; ++kb) {
        const int sl = has_ka ? r2s[B * ka + kb] : -1;
        src[kb] = sl >= 0 ? (int)(sl * plane) : -1;
    }
    double acc[A];
#pragma unroll
    for (int q = 0; q < A; ++q) acc[q] = 0.0;
    cx<T> pre[B];
#pragma unroll
    for (int kb = 0; kb < B; ++kb)
        pre[kb] = (has_ka && src[kb] >= 0 && bs < be) ? base[bs * bstride + src[kb]] : czero<T>();
    for (int b = bs; b < be; ++b) {
        if (has_ka) {
            cx<T> z[B];
#pragma unroll
            for (int kb = 0; kb < B; ++kb) z[kb] = pre[kb];
            if (b + 1 < be) {
#pragma unroll
                for (int kb = 0; kb < B; ++kb)
                    if (src[kb] >= 0) pre[kb] = base[(b + 1) * bstride + src[kb]];
            }
            RegDft<B, +1, T>::run(z);
            tile[(B * ka) * T3 + c] = z[0];
#pragma unroll
            for (int q = 1; q < B; ++q) tile[(B * ka + q) * T3 + c] = cmul(z[q], tw[q * A + ka]);
        }
        __syncthreads();
        if (has_jb) {
            const int kk = b / bbt;
            const double w = occ[(int64_t)kk * nb + b0 + (b - kk * bbt)];
            cx<T> a[A];
#pragma unroll
            for (int q = 0; q < A; ++q) a[q] = tile[(jb + B * q) * T3 + c];
            RegDft<A, +1, T>::run(a);
#pragma unroll
            for (int q = 0; q < A; ++q)
                acc[q] += w * ((double)a[q].re * (double)a[q].re + (double)a[q].im * (double)a[q].im);
        }
        __syncthreads();
    }
    if (has_jb) {
#pragma unroll
        for (int q = 0; q < A; ++q) {
            double *o = part + (int64_t)g * N1 * plane + (int64_t)(jb + B * q) * plane + (int64_t)j2 * N3 + c0 + c;
            *o = first ? acc[q] : *o + acc[q];
        }
    }
}

// out[j] = scale * sum_{g < G} part[g][j]   (fixed order)
__global__ void k_gradv_reduce(int64_t n, int G, const double *__restrict__ part, double *__restrict__ out, double inv_n) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int g = 0; g < G; ++g) s += part[(int64_t)g * n + j];
        out[j] = s * inv_n;
    }
}

// ------------------------------------------------------------ launchers ----
template <typename K> static int allow_lds(K kernel, size_t bytes) {
    APW_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    return ABACUS_PW_OK;
}

constexpr size_t kLdsLimit = 160 * 1024;

// LDS bytes of the compact-row plane kernels with chunk width C.
template <int N, typename T> static size_t compact_lds(int rows_max, int C) {
    return (size_t)(rows_max * N + N * C + N) * sizeof(cx<T>) + (size_t)N * sizeof(int);
}

// Chunk width for the compact kernels: the widest C <= 32 that fits (prefers two
// work-groups per CU when that still allows C >= 8). 0 when nothing fits.
template <int N, typename T> static int compact_chunk(int rows_max) {
    for (int C = std::min(32, N); C >= 8; C -= 8)
        if (compact_lds<N, T>(rows_max, C) <= kLdsLimit / 2) return C;
    for (int C = std::min(32, N); C >= 4; C -= 4)
        if (compact_lds<N, T>(rows_max, C) <= kLdsLimit) return C;
    return 0;
}

// One launch of a plane pass over the k-points [k0, k0 + nkb) of the batch ba.
template <int N, typename T, typename TIO>
static int launch_yz(bool inverse, const Plan &P, int k0, int nkb, const BatchArgs &ba, const void *psi,
                     void *hpsi, void *slab, hipStream_t st) {
    const size_t lds_full = (size_t)(N * N + N) * sizeof(cx<T>) + (size_t)N * sizeof(int);   // plane, twiddles, rows
    const int Cc = compact_chunk<N, T>(P.max_rows);
    const bool full_fits = lds_full <= kLdsLimit;
    const bool compact = g_yz_mode == 2 || !full_fits;
    if (compact && Cc == 0) return set_error(ABACUS_PW_EBAD_FFT_SIZE, "y-z plane rows do not fit in LDS at this precision");
    const cx<T> *tw = static_cast<const cx<T> *>(sizeof(T) == 8 ? P.tw64[2] : P.tw32[2]);
    const KDesc *kd = P.kdesc + k0;
    const int bpw = std::min(ba.bbt, g_yz_bands > 0 ? g_yz_bands : kYzBandsDefault);
    const dim3 grid(P.nslab, nkb * ceil_div(ba.bbt, bpw));
    if (compact) {
        const size_t lds = compact_lds<N, T>(P.max_rows, Cc);
        // threads per work-group: the compact planes hold one or two work-groups per
        // CU, so more waves per group hide more of the memory latency
        // default: 512 threads for the inverse pass (6% faster than 1024 at 120^3 FP64), and for
        // the forward pass the direct form below where its first phase has 128 to 512 tasks,
        // else 1024 threads (1024 measured 1.5x faster than 256 at 128^3 FP64)
        const int nt = g_yz_threads > 0 ? g_yz_threads : (inverse ? 512 : 1024);
        const int sel = nt == 256 ? 0 : (nt == 512 ? 1 : 2);
        auto inv = sel == 0 ? k_yz_inv_c<N, T, TIO, 256> : (sel == 1 ? k_yz_inv_c<N, T, TIO, 512> : k_yz_inv_c<N, T, TIO, 1024>);
        auto fwd = sel == 0 ? k_yz_fwd_c<N, T, TIO, 256> : (sel == 1 ? k_yz_fwd_c<N, T, TIO, 512> : k_yz_fwd_c<N, T, TIO, 1024>);
        const dim3 block(nt);
        if (inverse) {
            static bool once[3] = {false, false, false};
            if (!once[sel]) {
                APW_TRY(allow_lds(inv, kLdsLimit));
                once[sel] = true;
            }
            KernelTimer kt("yz_inv", st);
            hipLaunchKernelGGL(inv, grid, block, lds, st, static_cast<const cx<TIO> *>(psi), kd, ba, tw,
                               static_cast<cx<T> *>(slab), P.nslab, bpw, P.max_rows, Cc);
            return check_launch("yz_inv_c");
        }
        static bool once[3] = {false, false, false};
        if (!once[sel]) {
            APW_TRY(allow_lds(fwd, kLdsLimit));
            once[sel] = true;
        }
        KernelTimer kt("yz_fwd", st);
        // the direct forward pass: its first phase loads the slab itself (one barrier less
        // per chunk); at 120^3 FP64 (16 columns x 8 tasks) it took the pass from 3.87 to
        // 3.12 ms, at 128^3 (8 x 8 tasks) it is no faster
        const int tasks1 = Cc * LdsSplit<N>::B;
        if (g_yz_threads == 0 && tasks1 >= 128 && tasks1 <= 512) {
            static bool once_d = false;
            if (!once_d) {
                APW_TRY(allow_lds(k_yz_fwd_d<N, T, TIO, 512>, kLdsLimit));
                once_d = true;
            }
            hipLaunchKernelGGL((k_yz_fwd_d<N, T, TIO, 512>), grid, dim3(512), lds, st, static_cast<const cx<T> *>(slab),
                               P.nslab, kd, ba, tw, static_cast<const cx<TIO> *>(psi), static_cast<cx<TIO> *>(hpsi),
                               1.0 / (double)P.N, bpw, P.max_rows, Cc);
            return check_launch("yz_fwd_d");
        }
        hipLaunchKernelGGL(fwd, grid, block, lds, st, static_cast<const cx<T> *>(slab), P.nslab, kd, ba, tw,
                           static_cast<const cx<TIO> *>(psi), static_cast<cx<TIO> *>(hpsi), 1.0 / (double)P.N, bpw,
                           P.max_rows, Cc);
        return check_launch("yz_fwd_c");
    }
    if (inverse) {
        static bool once = false;
        if (!once) {
            APW_TRY(allow_lds(k_yz_inv<N, T, TIO>, lds_full));
            once = true;
        }
        KernelTimer kt("yz_inv", st);
        hipLaunchKernelGGL((k_yz_inv<N, T, TIO>), grid, dim3(yz_threads<N, T>()), lds_full, st,
                           static_cast<const cx<TIO> *>(psi), kd, ba, tw, static_cast<cx<T> *>(slab), P.nslab, bpw);
        return check_launch("yz_inv");
    }
    static bool once = false;
    if (!once) {
        APW_TRY(allow_lds(k_yz_fwd<N, T, TIO>, lds_full));
        once = true;
    }
    KernelTimer kt("yz_fwd", st);
    hipLaunchKernelGGL((k_yz_fwd<N, T, TIO>), grid, dim3(yz_threads<N, T>()), lds_full, st, static_cast<const cx<T> *>(slab),
                       P.nslab, kd, ba, tw, static_cast<const cx<TIO> *>(psi), static_cast<cx<TIO> *>(hpsi),
                       1.0 / (double)P.N, bpw);
    return check_launch("yz_fwd");
}

// j3 tile width of the x pass, T3 * max(A, B) <= 256 (one task per thread and phase) and
// T3 <= 32. When N3 is a multiple of 8 the slab rows start on 128-byte boundaries, and a
// multiple of 8 columns keeps every row segment a whole number of cache lines (at 120^3
// the divisor 15 read 240-byte segments across three lines, 1.39x the algorithmic bytes),
// even if the last tile is ragged (a divisor of N3 within 3/4 of the widest such width is
// taken instead); otherwise the widest divisor of N3, else the bound.
static int xpass_tile(int n1, int n3) {
    int a, b;
    lds_split_host(n1, &a, &b);
    const int cap = std::min(kMaxT3, 256 / std::max(a, b));   // one task per thread in both phases
    if (n3 % 8 == 0 && cap >= 8) {
        const int top = std::min(cap / 8 * 8, n3);   // widest multiple of 8; a divisor of N3 within 3/4 of it wins
        for (int t = top; 4 * t >= 3 * top; t -= 8)
            if (n3 % t == 0) return t;
        return top;
    }
    for (int t = cap; t >= 4; --t)
        if (n3 % t == 0) return t;
    return std::min(cap, n3);
}

template <int N1, typename T>
static int launch_x(const Plan &P, const void *vloc, void *slab, int nbands, hipStream_t st) {
    const int T3 = xpass_tile(N1, P.N3), nt3 = ceil_div(P.N3, T3);
    const size_t lds = (size_t)(N1 * T3 + N1) * sizeof(cx<T>) + (size_t)N1 * sizeof(int);
    static bool once = false;
    if (!once) {
        APW_TRY(allow_lds(k_xpass<N1, T, T>, kLdsLimit));
        once = true;
    }
    const cx<T> *tw = static_cast<const cx<T> *>(sizeof(T) == 8 ? P.tw64[0] : P.tw32[0]);
    const int bpw = g_x_bands > 0 ? g_x_bands : (sizeof(T) == 8 ? kXBands64 : kXBands);
    dim3 grid(P.N2 * nt3, ceil_div(nbands, bpw));
    KernelTimer kt("xpass", st);
    hipLaunchKernelGGL((k_xpass<N1, T, T>), grid, dim3(256), lds, st, static_cast<cx<T> *>(slab), P.nslab, P.N2,
                       P.N3, T3, nt3, nbands, bpw, P.row_to_slab, static_cast<const T *>(vloc), tw);
    return check_launch("xpass");
}

#define APW_LENGTHS(X) \
    X(8) X(12) X(16) X(18) X(20) X(24) X(27) X(30) X(32) X(36) X(40) X(45) X(48) X(54) X(60) X(64) X(72) X(80) \
    X(81) X(90) X(96) X(100) X(108) X(120) X(128)

int local_length_supported(int n) {
    switch (n) {
#define APW_CASE(n) case n:
        APW_LENGTHS(APW_CASE)
#undef APW_CASE
        return 1;
        default:
            return 0;
    }
}

template <typename T, typename TIO>
static int dispatch_yz(bool inverse, const Plan &P, int k0, int nkb, const BatchArgs &ba, const void *psi, void *hpsi,
                       void *slab, hipStream_t st) {
    switch (P.N3) {
#define APW_CASE(n) \
    case n: return launch_yz<n, T, TIO>(inverse, P, k0, nkb, ba, psi, hpsi, slab, st);
        APW_LENGTHS(APW_CASE)
#undef APW_CASE
        default:
            return set_error(ABACUS_PW_EBAD_FFT_SIZE, "unsupported grid length");
    }
}

template <typename T>
static int dispatch_x(const Plan &P, const void *vloc, void *slab, int nbands, hipStream_t st) {
    switch (P.N1) {
#define APW_CASE(n) \
    case n: return launch_x<n, T>(P, vloc, slab, nbands, st);
        APW_LENGTHS(APW_CASE)
#undef APW_CASE
        default:
            return set_error(ABACUS_PW_EBAD_FFT_SIZE, "unsupported grid length");
    }
}

int local_supported(const Plan &P, int fft_prec) {
    if (!local_length_supported(P.N1) || !local_length_supported(P.N2) || !local_length_supported(P.N3))
        return set_error(ABACUS_PW_EBAD_FFT_SIZE, "grid length without a transform");
    if (P.N2 != P.N3) return set_error(ABACUS_PW_EBAD_FFT_SIZE, "the plane transform needs N2 == N3");
    const size_t cb = fft_prec == 0 ? 16 : 8;
    const size_t need = ((size_t)P.max_rows * P.N3 + (size_t)P.N3 * 4 + P.N3) * cb + (size_t)P.N3 * 4;
    if (need > kLdsLimit) return set_error(ABACUS_PW_EBAD_FFT_SIZE, "y-z plane rows do not fit in LDS at this precision");
    return ABACUS_PW_OK;
}

size_t local_slab_bytes(const Plan &P, int fft_prec, int nbands) {
    return (size_t)nbands * (size_t)P.nslab * (size_t)P.N2 * (size_t)P.N3 * (fft_prec == 0 ? 16 : 8);
}


template <int N1, typename T>
static int launch_gradv(const Plan &P, const void *sx, const void *sy, int nbands, double *part, int G, int first,
                        hipStream_t st) {
    const int T3 = xpass_tile(N1, P.N3), nt3 = ceil_div(P.N3, T3);
    const size_t lds = (size_t)(N1 * T3 + N1) * sizeof(cx<T>) + (size_t)N1 * sizeof(int);
    static bool once = false;
    if (!once) {
        APW_TRY(allow_lds(k_gradv_x<N1, T>, kLdsLimit));
        once = true;
    }
    const cx<T> *tw = static_cast<const cx<T> *>(sizeof(T) == 8 ? P.tw64[0] : P.tw32[0]);
    KernelTimer kt("gradv_x", st);
    hipLaunchKernelGGL((k_gradv_x<N1, T>), dim3(P.N2 * nt3, G), dim3(256), lds, st, static_cast<const cx<T> *>(sx),
                       static_cast<const cx<T> *>(sy), P.nslab, P.N2, P.N3, T3, nt3, nbands, ceil_div(nbands, G),
                       P.row_to_slab, tw, part, first);
    return check_launch("gradv_x");
}

template <int N1, typename T>
static int launch_density(const Plan &P, const void *slab, int nbands, const double *occ, int nb, int b0, int bbt,
                          double *part, int G, int first, hipStream_t st) {
    const int T3 = xpass_tile(N1, P.N3), nt3 = ceil_div(P.N3, T3);
    const size_t lds = (size_t)(N1 * T3 + N1) * sizeof(cx<T>) + (size_t)N1 * sizeof(int);
    static bool once = false;
    if (!once) {
        APW_TRY(allow_lds(k_density_x<N1, T>, kLdsLimit));
        once = true;
    }
    const cx<T> *tw = static_cast<const cx<T> *>(sizeof(T) == 8 ? P.tw64[0] : P.tw32[0]);
    KernelTimer kt("density_x", st);
    hipLaunchKernelGGL((k_density_x<N1, T>), dim3(P.N2 * nt3, G), dim3(256), lds, st,
                       static_cast<const cx<T> *>(slab), P.nslab, P.N2, P.N3, T3, nt3, nbands, ceil_div(nbands, G),
                       P.row_to_slab, tw, occ, nb, b0, bbt, part, first);
    return check_launch("density_x");
}

int local_inverse_planes(const Plan &P, int k0, int k1, int nb, int b0, int bbt, int fft_prec, int io_prec,
                         const void *psi, void *slab, hipStream_t st) {
    const BatchArgs ba{nb, P.pw_off[k0], b0, bbt};
    const int nkb = k1 - k0;
    if (fft_prec == 0) return dispatch_yz<double, double>(true, P, k0, nkb, ba, psi, nullptr, slab, st);
    if (io_prec == 1) return dispatch_yz<float, float>(true, P, k0, nkb, ba, psi, nullptr, slab, st);
    return dispatch_yz<float, double>(true, P, k0, nkb, ba, psi, nullptr, slab, st);
}

int local_gradv_accumulate(const Plan &P, int fft_prec, const void *slab_x, const void *slab_y, int nbands,
                           double *part, int G, int first, hipStream_t st) {
    switch (P.N1) {
#define APW_CASE(n)                                                                                     \
    case n:                                                                                             \
        return fft_prec == 0 ? launch_gradv<n, double>(P, slab_x, slab_y, nbands, part, G, first, st) \
                             : launch_gradv<n, float>(P, slab_x, slab_y, nbands, part, G, first, st);
        APW_LENGTHS(APW_CASE)
#undef APW_CASE
        default:
            return set_error(ABACUS_PW_EBAD_FFT_SIZE, "unsupported grid length");
    }
}

int local_density_accumulate(const Plan &P, int fft_prec, const void *slab, int nbands, const double *occ, int nb,
                             int b0, int bbt, double *part, int G, int first, hipStream_t st) {
    switch (P.N1) {
#define APW_CASE(n)                                                                                                  \
    case n:                                                                                                          \
        return fft_prec == 0 ? launch_density<n, double>(P, slab, nbands, occ, nb, b0, bbt, part, G, first, st)     \
                             : launch_density<n, float>(P, slab, nbands, occ, nb, b0, bbt, part, G, first, st);
        APW_LENGTHS(APW_CASE)
#undef APW_CASE
        default:
            return set_error(ABACUS_PW_EBAD_FFT_SIZE, "unsupported grid length");
    }
}

int local_sum_parts(const Plan &P, const double *part, int G, double scale, double *out, hipStream_t st) {
    KernelTimer kt("gradv_reduce", st);
    const int64_t blocks = std::min<int64_t>(ceil_div64(P.N, 256), 8192);
    hipLaunchKernelGGL(k_gradv_reduce, dim3((unsigned)blocks), dim3(256), 0, st, (int64_t)P.N, G, part, out, scale);
    return check_launch("gradv_reduce");
}

int local_term(const Plan &P, int k0, int k1, int fft_prec, int io_prec, const void *vloc, const void *psi,
               void *hpsi, int nb, void *slab, int band_batch, hipStream_t st,
               const std::function<int(int, int)> &after_batch) {
    const int nkb = k1 - k0;
    for (int b0 = 0; b0 < nb; b0 += band_batch) {
        const BatchArgs ba{nb, P.pw_off[k0], b0, std::min(band_batch, nb - b0)};
        const int nv = nkb * ba.bbt;   // (k, band) planes sets in this batch
        if (fft_prec == 0) {
            APW_TRY((dispatch_yz<double, double>(true, P, k0, nkb, ba, psi, nullptr, slab, st)));
            APW_TRY((dispatch_x<double>(P, vloc, slab, nv, st)));
            APW_TRY((dispatch_yz<double, double>(false, P, k0, nkb, ba, psi, hpsi, slab, st)));
        } else if (io_prec == 1) {
            APW_TRY((dispatch_yz<float, float>(true, P, k0, nkb, ba, psi, nullptr, slab, st)));
            APW_TRY((dispatch_x<float>(P, vloc, slab, nv, st)));
            APW_TRY((dispatch_yz<float, float>(false, P, k0, nkb, ba, psi, hpsi, slab, st)));
        } else {
            APW_TRY((dispatch_yz<float, double>(true, P, k0, nkb, ba, psi, nullptr, slab, st)));
            APW_TRY((dispatch_x<float>(P, vloc, slab, nv, st)));
            APW_TRY((dispatch_yz<float, double>(false, P, k0, nkb, ba, psi, hpsi, slab, st)));
        }
        if (after_batch) APW_TRY(after_batch(b0, ba.bbt));
    }
    return ABACUS_PW_OK;
}

}  // namespace apw

namespace apw {

// Host view of the LDS split (N = A * B) of every compiled length.
int lds_split_host(int n, int *a, int *b) {
    switch (n) {
#define APW_CASE(n)              \
    case n:                      \
        *a = LdsSplit<n>::A;     \
        *b = LdsSplit<n>::B;     \
        return 1;
        APW_LENGTHS(APW_CASE)
#undef APW_CASE
        default:
            *a = *b = 0;
            return 0;
    }
}

}  // namespace apw
