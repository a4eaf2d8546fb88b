// Density transform on the FFT grid (Sec. III.A): the reciprocal-space density
//
//   rho(G) = (1/N) sum_j rho(r_j) e^{-i G.r_j},   N = N1 N2 N3,
//
// the grid form of rho(G) = (1/Omega) int rho(r) e^{-iG.r} dr, from the
// real-space density of abacus_pw_density. It is a full forward 3-D transform
// (the density sphere reaches 2 Gmax, so no axis can be pruned), done as three
// passes, one per axis, each a batch of LDS-resident two-level transforms:
//
//   pass z  one work-group per kRowsZ consecutive (j1, j2) rows: load the real
//           rows, transform along j3, store complex rows (natural order).
//   pass y  one work-group per (j1, j3 tile): transform along j2, in place.
//   pass x  one work-group per (j2, j3 tile): transform along j1, times 1/N,
//           in place, or gathered straight into the output for a G list.
//
// Each pass reads and writes the grid once (88 N bytes in all for FP64). The
// LDS transforms leave frequency k in a digit-permuted slot; every pass reads
// its outputs back in natural order, so the grid is in natural order between
// passes. Twiddles are generated on the device (sincospi), so the transform
// needs no plan and no tables.
//
// With a G list the passes run on a work grid that the library allocates per
// device on first use; for the whole grid they run in the output itself.
#include <mutex>

#include "fft_device.hpp"
#include "plan.hpp"

namespace apw {

int local_length_supported(int n);   // local.hip

namespace {

constexpr int kRowsZ = 16;    // rows per work-group of the z pass
constexpr int kTileYX = 16;   // j3 columns per work-group of the y and x passes
constexpr int kThreadsDG = 256;

// tw[jb * A + ka] = exp(+2 pi i jb ka / N) in LDS, as lds_fft expects.
template <int N> __device__ __forceinline__ void make_twiddles(z64 *tw) {
    constexpr int A = LdsSplit<N>::A, B = LdsSplit<N>::B;
    for (int t = threadIdx.x; t < A * B; t += blockDim.x) {
        const int jb = t / A, ka = t - jb * A;
        const int e = (jb * ka) % N;
        double s, c;
        sincospi(2.0 * (double)e / (double)N, &s, &c);
        tw[t] = z64{c, s};
    }
}

// Pass z: rows r = (j1 N2 + j2) of length N3 (contiguous). Real input.
template <int N>
__global__ __launch_bounds__(kThreadsDG) void k_dg_z(const double *__restrict__ rho, z64 *__restrict__ out, int64_t nrows) {
    __shared__ z64 lds[kRowsZ * N];
    __shared__ z64 tw[N];
    make_twiddles<N>(tw);
    const int64_t r0 = (int64_t)blockIdx.x * kRowsZ;
    const int nr = nrows - r0 < kRowsZ ? (int)(nrows - r0) : kRowsZ;
    for (int t = threadIdx.x; t < kRowsZ * N; t += blockDim.x) {
        const int l = t / N;
        lds[t] = z64{l < nr ? rho[(r0 + l) * N + (t - l * N)] : 0.0, 0.0};
    }
    __syncthreads();
    lds_fft<N, -1, false>(lds, kRowsZ, [](int l) { return l * N; }, 1, static_cast<const z64 *>(tw));
    for (int t = threadIdx.x; t < nr * N; t += blockDim.x) {
        const int l = t / N, k = t - l * N;
        out[(r0 + l) * N + k] = lds[l * N + perm_slot<N>(k)];
    }
}

// Pass along a strided axis of length N: line (o, j3) has its elements at
// o * so + e * se + j3, e < N. One work-group per (o, tile of kTileYX j3); the
// transformed lines go back in place, times `scale`.
template <int N>
__global__ __launch_bounds__(kThreadsDG) void k_dg_strided(z64 *__restrict__ g, int n3, int64_t so, int64_t se,
                                                          int ntile, double scale) {
    __shared__ z64 lds[kTileYX * N];
    __shared__ z64 tw[N];
    make_twiddles<N>(tw);
    const int o = blockIdx.x / ntile, j0 = (blockIdx.x - o * ntile) * kTileYX;
    const int nt = min(kTileYX, n3 - j0);
    z64 *base = g + (int64_t)o * so + j0;
    for (int t = threadIdx.x; t < kTileYX * N; t += blockDim.x) {
        const int e = t / kTileYX, c = t - e * kTileYX;
        lds[t] = c < nt ? base[(int64_t)e * se + c] : z64{0.0, 0.0};
    }
    __syncthreads();
    lds_fft<N, -1, true>(lds, kTileYX, [](int l) { return l; }, kTileYX, static_cast<const z64 *>(tw));
    for (int t = threadIdx.x; t < kTileYX * N; t += blockDim.x) {
        const int k = t / kTileYX, c = t - k * kTileYX;
        if (c < nt) {
            const z64 v = lds[perm_slot<N>(k) * kTileYX + c];
            base[(int64_t)k * se + c] = z64{v.re * scale, v.im * scale};
        }
    }
}

// rhog[i] = grid[(m1 mod N1, m2 mod N2, m3 mod N3)] for the Miller triples of the G list.
__global__ void k_dg_gather(const z64 *__restrict__ grid, const int *__restrict__ miller, int64_t ng, int n1, int n2,
                            int n3, z64 *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ng) return;
    int a = miller[3 * i] % n1, b = miller[3 * i + 1] % n2, c = miller[3 * i + 2] % n3;
    a += a < 0 ? n1 : 0;
    b += b < 0 ? n2 : 0;
    c += c < 0 ? n3 : 0;
    out[i] = grid[((int64_t)a * n2 + b) * n3 + c];
}

#define APW_DG_LENGTHS(X) \
    X(8) X(12) X(16) X(18) X(20) X(24) X(27) X(30) X(32) X(36) X(40) X(45) X(48) X(54) X(60) X(64) X(72) X(80) \
    X(81) X(90) X(96) X(100) X(108) X(120) X(128)

int launch_z(int n3, const double *rho, z64 *out, int64_t nrows, hipStream_t st) {
    const dim3 grid((unsigned)ceil_div64(nrows, kRowsZ)), block(kThreadsDG);
    switch (n3) {
#define APW_CASE(n) \
    case n: hipLaunchKernelGGL(k_dg_z<n>, grid, block, 0, st, rho, out, nrows); break;
        APW_DG_LENGTHS(APW_CASE)
#undef APW_CASE
        default: return set_error(ABACUS_PW_EBAD_FFT_SIZE, "unsupported grid length");
    }
    return check_launch("density_g z pass");
}

int launch_strided(int n, z64 *g, int nouter, int n3, int64_t so, int64_t se, double scale, hipStream_t st) {
    const int ntile = ceil_div(n3, kTileYX);
    const dim3 grid((unsigned)(nouter * ntile)), block(kThreadsDG);
    switch (n) {
#define APW_CASE(len) \
    case len: hipLaunchKernelGGL(k_dg_strided<len>, grid, block, 0, st, g, n3, so, se, ntile, scale); break;
        APW_DG_LENGTHS(APW_CASE)
#undef APW_CASE
        default: return set_error(ABACUS_PW_EBAD_FFT_SIZE, "unsupported grid length");
    }
    return check_launch("density_g strided pass");
}

#undef APW_DG_LENGTHS

// The three passes on the grid g (natural order in and out); rho is read by the first.
int transform(const int *n, const double *rho, z64 *g, hipStream_t st) {
    const int64_t N = (int64_t)n[0] * n[1] * n[2];
    KernelTimer kt("density_g", st);
    APW_TRY(launch_z(n[2], rho, g, (int64_t)n[0] * n[1], st));
    APW_TRY(launch_strided(n[1], g, n[0], n[2], (int64_t)n[1] * n[2], n[2], 1.0, st));
    return launch_strided(n[0], g, n[1], n[2], n[2], (int64_t)n[1] * n[2], 1.0 / (double)N, st);
}

int check_args(const int *fft, const double *rho, int ng, const int *miller_g, const void *rhog) {
    if (!fft || !rho || !rhog) return set_error(ABACUS_PW_ENULL_ARG, "fft, rho and rhog are required");
    for (int i = 0; i < 3; ++i)
        if (!local_length_supported(fft[i]))
            return set_error(ABACUS_PW_EBAD_FFT_SIZE, "grid length without a transform in this library");
    const int64_t N = (int64_t)fft[0] * fft[1] * fft[2];
    if (ng < 0) return set_error(ABACUS_PW_EBAD_SHAPE, "ng must be >= 0");
    if (!miller_g && (int64_t)ng != N) return set_error(ABACUS_PW_EBAD_SHAPE, "without a G list ng must equal N1 N2 N3");
    return ABACUS_PW_OK;
}

int gather(const int *fft, const z64 *grid, int ng, const int *miller_g, void *rhog, hipStream_t st) {
    if (ng == 0) return ABACUS_PW_OK;
    KernelTimer kt("density_g_gather", st);
    hipLaunchKernelGGL(k_dg_gather, dim3((unsigned)ceil_div64(ng, 256)), dim3(256), 0, st, grid, miller_g, (int64_t)ng,
                       fft[0], fft[1], fft[2], static_cast<z64 *>(rhog));
    return check_launch("density_g gather");
}

// Work grid of the allocating entry point, one per device, grown as needed.
constexpr int kMaxDevicesDG = 64;
std::mutex g_dg_mu;
DeviceBuffer g_dg_work[kMaxDevicesDG];

// Fixed work grid of abacus_pw_density_g_noalloc: the largest grid the library
// transforms (128^3 points, 32 MiB of complex128), a copy on every device the
// library runs on, held until the process ends. In host code `scratch` names a
// host-side stand-in: its device address comes from hipGetSymbolAddress, taken
// once per device (with that device current) and kept in g_na_ptr.
constexpr int64_t kNoAllocMaxPoints = 128 * 128 * 128;
static __device__ __align__(256) z64 scratch[kNoAllocMaxPoints];
std::mutex g_na_mu;
void *g_na_ptr[kMaxDevicesDG] = {};

int noalloc_work(z64 **out) {
    int dev = 0;
    APW_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevicesDG) return set_error(ABACUS_PW_EINTERNAL, "device index out of range");
    std::lock_guard<std::mutex> l(g_na_mu);
    if (!g_na_ptr[dev]) {
        void *ptr = nullptr;
        APW_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return set_error(ABACUS_PW_EHIP, "no device address for the fixed work grid");
        g_na_ptr[dev] = ptr;
    }
    *out = static_cast<z64 *>(g_na_ptr[dev]);
    return ABACUS_PW_OK;
}

}  // namespace

}  // namespace apw

using namespace apw;

extern "C" int abacus_pw_density_g(const int *fft, const double *rho, int ng, const int *miller_g, void *rhog,
                                   void *stream) {
    try {
        APW_TRY(check_args(fft, rho, ng, miller_g, rhog));
        hipStream_t st = static_cast<hipStream_t>(stream);
        if (!miller_g) return transform(fft, rho, static_cast<z64 *>(rhog), st);
        int dev = 0;
        APW_HIP(hipGetDevice(&dev));
        if (dev < 0 || dev >= kMaxDevicesDG) return set_error(ABACUS_PW_EINTERNAL, "device index out of range");
        const size_t bytes = sizeof(z64) * (size_t)fft[0] * fft[1] * fft[2];
        z64 *work = nullptr;
        {
            std::lock_guard<std::mutex> l(g_dg_mu);
            if (g_dg_work[dev].bytes < bytes) {
                // the old grid may still be read by work enqueued earlier
                APW_HIP(hipDeviceSynchronize());
                APW_TRY(g_dg_work[dev].ensure(bytes));
            }
            work = g_dg_work[dev].as<z64>();
        }
        APW_TRY(transform(fft, rho, work, st));
        return gather(fft, work, ng, miller_g, rhog, st);
    } catch (...) {
        return set_error(ABACUS_PW_EINTERNAL, "internal error");
    }
}

extern "C" int abacus_pw_density_g_noalloc(const int *fft, const double *rho, int ng, const int *miller_g, void *rhog,
                                           void *stream) {
    try {
        APW_TRY(check_args(fft, rho, ng, miller_g, rhog));
        hipStream_t st = static_cast<hipStream_t>(stream);
        if (!miller_g) return transform(fft, rho, static_cast<z64 *>(rhog), st);
        if ((int64_t)fft[0] * fft[1] * fft[2] > kNoAllocMaxPoints)
            return set_error(ABACUS_PW_EBAD_SHAPE, "grid larger than the fixed work grid (2,097,152 points)");
        z64 *work = nullptr;
        APW_TRY(noalloc_work(&work));
        APW_TRY(transform(fft, rho, work, st));
        return gather(fft, work, ng, miller_g, rhog, st);
    } catch (...) {
        return set_error(ABACUS_PW_EINTERNAL, "internal error");
    }
}
