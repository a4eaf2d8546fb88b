// Plan construction: validation of the problem statement, the sphere <-> grid
// tables of every k-point, kinetic factors, transform twiddles and D-block
// tables, uploaded once and cached per geometry.
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "local.hpp"

namespace apw {

int lds_split_host(int n, int *a, int *b);   // local_tables.cpp

int g_band_batch = 0;
int g_splitk_chunk = 0;
int g_yz_bands = 0;
int g_x_bands = 0;
int g_yz_mode = 0;
int g_overlap = 0;
int g_yz_threads = 0;

DeviceBuffer::~DeviceBuffer() {
    if (ptr) (void)hipFree(ptr);
}

// Kernels enqueued by an earlier call may still read the plan's tables and work
// space; its buffers are released only after the device has drained them.
Plan::~Plan() { (void)hipDeviceSynchronize(); }

int DeviceBuffer::ensure(size_t n) {
    if (n <= bytes && ptr) return ABACUS_PW_OK;
    if (ptr) {
        APW_HIP(hipFree(ptr));
        ptr = nullptr;
        bytes = 0;
    }
    if (n == 0) n = 256;
    APW_HIP(hipMalloc(&ptr, n));
    bytes = n;
    return ABACUS_PW_OK;
}

int validate_problem_shallow(const abacus_pw_problem *p) {
    if (!p) return set_error(ABACUS_PW_ENULL_ARG, "problem is NULL");
    if (!p->kpts || !p->npw || !p->miller || !p->vloc)
        return set_error(ABACUS_PW_ENULL_ARG, "kpts, npw, miller and vloc are required");
    for (int i = 0; i < 3; ++i)
        if (p->fft[i] < 1) return set_error(ABACUS_PW_EBAD_FFT_SIZE, "grid lengths must be positive");
    if (p->nk < 1) return set_error(ABACUS_PW_EBAD_SHAPE, "nk must be >= 1");
    for (int k = 0; k < p->nk; ++k)
        if (p->npw[k] < 1) return set_error(ABACUS_PW_EBAD_SHAPE, "every npw must be >= 1");
    if (p->nproj < 0 || p->natom < 0) return set_error(ABACUS_PW_EBAD_SHAPE, "negative nproj or natom");
    if (p->nproj > 0) {
        if (!p->beta || !p->dmat || !p->proj_atom_offset)
            return set_error(ABACUS_PW_ENULL_ARG, "beta, dmat and proj_atom_offset are required when nproj > 0");
        if (p->natom < 1) return set_error(ABACUS_PW_EBAD_SHAPE, "nproj > 0 needs natom >= 1");
        if (p->proj_atom_offset[0] != 0 || p->proj_atom_offset[p->natom] != p->nproj)
            return set_error(ABACUS_PW_EBAD_SHAPE, "proj_atom_offset must run from 0 to nproj");
        for (int a = 0; a < p->natom; ++a)
            if (p->proj_atom_offset[a + 1] <= p->proj_atom_offset[a])
                return set_error(ABACUS_PW_EBAD_SHAPE, "every atom block needs at least one projector");
    }
    if (!(p->ecutwfc > 0.0) || !std::isfinite(p->ecutwfc)) return set_error(ABACUS_PW_EBAD_SHAPE, "ecutwfc must be > 0");
    const double det = p->lattice[0] * (p->lattice[4] * p->lattice[8] - p->lattice[5] * p->lattice[7]) -
                       p->lattice[1] * (p->lattice[3] * p->lattice[8] - p->lattice[5] * p->lattice[6]) +
                       p->lattice[2] * (p->lattice[3] * p->lattice[7] - p->lattice[4] * p->lattice[6]);
    if (!(std::fabs(det) > 0.0) || !std::isfinite(det)) return set_error(ABACUS_PW_EBAD_SHAPE, "singular lattice");
    return ABACUS_PW_OK;
}

// ---------------------------------------------------------------- cache ----
namespace {

struct Key {
    double lattice[9];
    int fft[3];
    double ecut;
    int nk;
    std::vector<double> kpts;
    std::vector<int> npw;
    const int *miller;
    uint64_t miller_hash;
    int nproj, natom;
    std::vector<int> offs;
    int device;
    bool operator==(const Key &o) const {
        return std::memcmp(lattice, o.lattice, sizeof lattice) == 0 && std::memcmp(fft, o.fft, sizeof fft) == 0 &&
               ecut == o.ecut && nk == o.nk && kpts == o.kpts && npw == o.npw && miller == o.miller &&
               miller_hash == o.miller_hash && nproj == o.nproj && natom == o.natom && offs == o.offs &&
               device == o.device;
    }
};

// FNV-1a over every Miller triple (about 1 ms per million triples): a caller
// that reorders or edits the map in the same buffer gets a new plan.
uint64_t miller_fnv(const int *m, int64_t n) {
    uint64_t h = 1469598103934665603ull;
    for (int64_t i = 0; i < 3 * n; ++i) {
        h ^= (uint32_t)m[i];
        h *= 1099511628211ull;
    }
    return h;
}

struct Entry {
    Key key;
    std::shared_ptr<Plan> plan;
    uint64_t last_use;
};

std::mutex g_mu;
std::vector<Entry> g_cache;
uint64_t g_clock = 0;
constexpr size_t kMaxPlans = 6;

Key make_key(const abacus_pw_problem *p) {
    Key k;
    std::memcpy(k.lattice, p->lattice, sizeof k.lattice);
    std::memcpy(k.fft, p->fft, sizeof k.fft);
    k.ecut = p->ecutwfc;
    k.nk = p->nk;
    k.kpts.assign(p->kpts, p->kpts + 3 * p->nk);
    k.npw.assign(p->npw, p->npw + p->nk);
    int64_t tot = 0;
    for (int i = 0; i < p->nk; ++i) tot += p->npw[i];
    k.miller = p->miller;
    k.miller_hash = miller_fnv(p->miller, tot);
    k.nproj = p->nproj;
    k.natom = p->natom;
    if (p->nproj > 0) k.offs.assign(p->proj_atom_offset, p->proj_atom_offset + p->natom + 1);
    int dev = 0;
    (void)hipGetDevice(&dev);
    k.device = dev;
    return k;
}

// Appends a typed array to a byte image (16-byte aligned), returning its offset.
template <typename T> size_t put(std::vector<unsigned char> &img, const std::vector<T> &v) {
    size_t off = (img.size() + 15) / 16 * 16;
    img.resize(off + v.size() * sizeof(T));
    if (!v.empty()) std::memcpy(img.data() + off, v.data(), v.size() * sizeof(T));
    return off;
}

int wrap(int m, int n) {
    int r = m % n;
    return r < 0 ? r + n : r;
}

int perm_slot_host(int k, int n) {
    int a, b;
    lds_split_host(n, &a, &b);
    return b * (k % a) + k / a;
}

int build_plan(const abacus_pw_problem *p, Plan &P, hipStream_t st) {
    std::memcpy(P.lattice, p->lattice, sizeof P.lattice);
    P.N1 = p->fft[0];
    P.N2 = p->fft[1];
    P.N3 = p->fft[2];
    P.N = (int64_t)P.N1 * P.N2 * P.N3;
    for (int i = 0; i < 3; ++i) {
        int a, b;
        if (!lds_split_host(p->fft[i], &a, &b))
            return set_error(ABACUS_PW_EBAD_FFT_SIZE,
                             "grid length " + std::to_string(p->fft[i]) + " has no transform in this library");
    }
    // reciprocal vectors: a_i . b_j = 2 pi delta_ij
    const double *a = p->lattice;
    const double c23[3] = {a[4] * a[8] - a[5] * a[7], a[5] * a[6] - a[3] * a[8], a[3] * a[7] - a[4] * a[6]};
    const double c31[3] = {a[7] * a[2] - a[8] * a[1], a[8] * a[0] - a[6] * a[2], a[6] * a[1] - a[7] * a[0]};
    const double c12[3] = {a[1] * a[5] - a[2] * a[4], a[2] * a[3] - a[0] * a[5], a[0] * a[4] - a[1] * a[3]};
    const double vol = a[0] * c23[0] + a[1] * c23[1] + a[2] * c23[2];
    const double tp = 6.283185307179586476925286766559;
    for (int c = 0; c < 3; ++c) {
        P.recip[c] = tp * c23[c] / vol;
        P.recip[3 + c] = tp * c31[c] / vol;
        P.recip[6 + c] = tp * c12[c] / vol;
    }
    P.nk = p->nk;
    P.npw.assign(p->npw, p->npw + p->nk);
    P.pw_off.assign(p->nk + 1, 0);
    for (int k = 0; k < p->nk; ++k) P.pw_off[k + 1] = P.pw_off[k] + p->npw[k];
    P.npw_total = P.pw_off[p->nk];
    P.max_npw = *std::max_element(P.npw.begin(), P.npw.end());
    P.nproj = p->nproj;
    P.natom = p->natom;
    if (p->nproj > 0) P.proj_atom_offset.assign(p->proj_atom_offset, p->proj_atom_offset + p->natom + 1);

    // sphere checks and slab extent
    int m1min = 1 << 30, m1max = -(1 << 30);
    std::vector<unsigned char> seen((size_t)P.N);
    for (int k = 0; k < p->nk; ++k) {
        std::fill(seen.begin(), seen.end(), 0);
        const int *mk = p->miller + 3 * P.pw_off[k];
        const double *kv = p->kpts + 3 * k;
        for (int g = 0; g < p->npw[k]; ++g) {
            const int *m = mk + 3 * g;
            for (int c = 0; c < 3; ++c)
                if (2 * std::abs(m[c]) + 1 > p->fft[c])
                    return set_error(ABACUS_PW_EBAD_FFT_SIZE, "the G-sphere does not fit the grid (2|m|+1 > N)");
            double q[3];
            for (int c = 0; c < 3; ++c) q[c] = kv[c] + m[0] * P.recip[c] + m[1] * P.recip[3 + c] + m[2] * P.recip[6 + c];
            const double kg2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2];
            if (!(kg2 < p->ecutwfc)) return set_error(ABACUS_PW_EBAD_SPHERE, "a Miller triple has |k+G|^2 >= ecutwfc");
            const int64_t idx = ((int64_t)wrap(m[0], P.N1) * P.N2 + wrap(m[1], P.N2)) * P.N3 + wrap(m[2], P.N3);
            if (seen[idx]) return set_error(ABACUS_PW_EBAD_SPHERE, "duplicate Miller triple");
            seen[idx] = 1;
            m1min = std::min(m1min, m[0]);
            m1max = std::max(m1max, m[0]);
        }
    }
    P.m1min = m1min;
    P.nslab = m1max - m1min + 1;

    // per-k plane tables
    std::vector<unsigned char> img;
    struct Offs {
        size_t pt_off, pt_g, pt_pos, row_off, row_list, kin, kin32;
    };
    std::vector<Offs> koffs(p->nk);
    for (int k = 0; k < p->nk; ++k) {
        const int *mk = p->miller + 3 * P.pw_off[k];
        const double *kv = p->kpts + 3 * k;
        const int npw = p->npw[k];
        std::vector<int> cnt(P.nslab + 1, 0);
        for (int g = 0; g < npw; ++g) cnt[mk[3 * g] - m1min + 1]++;
        std::vector<int> pt_off(P.nslab + 1, 0);
        for (int s = 0; s < P.nslab; ++s) pt_off[s + 1] = pt_off[s] + cnt[s + 1];
        std::vector<int> fill(pt_off.begin(), pt_off.end() - 1), pt_g(npw), pt_pos(npw);
        for (int g = 0; g < npw; ++g) {
            const int *m = mk + 3 * g;
            const int s = m[0] - m1min;
            const int pos = perm_slot_host(wrap(m[1], P.N2), P.N2) * P.N3 + perm_slot_host(wrap(m[2], P.N3), P.N3);
            pt_g[fill[s]] = g;
            pt_pos[fill[s]] = pos;
            fill[s]++;
        }
        std::vector<int> row_off(P.nslab + 1, 0), row_list;
        for (int s = 0; s < P.nslab; ++s) {
            std::vector<int> rows;
            for (int q = pt_off[s]; q < pt_off[s + 1]; ++q) rows.push_back(pt_pos[q] / P.N3);
            std::sort(rows.begin(), rows.end());
            rows.erase(std::unique(rows.begin(), rows.end()), rows.end());
            row_list.insert(row_list.end(), rows.begin(), rows.end());
            P.max_rows = std::max(P.max_rows, (int)rows.size());
            row_off[s + 1] = (int)row_list.size();
        }
        std::vector<double> kin(npw);
        std::vector<float> kin32(npw);
        for (int g = 0; g < npw; ++g) {
            const int *m = mk + 3 * g;
            double q[3];
            for (int c = 0; c < 3; ++c) q[c] = kv[c] + m[0] * P.recip[c] + m[1] * P.recip[3 + c] + m[2] * P.recip[6 + c];
            kin[g] = q[0] * q[0] + q[1] * q[1] + q[2] * q[2];
            kin32[g] = (float)kin[g];
        }
        koffs[k].pt_off = put(img, pt_off);
        koffs[k].pt_g = put(img, pt_g);
        koffs[k].pt_pos = put(img, pt_pos);
        koffs[k].row_off = put(img, row_off);
        koffs[k].row_list = put(img, row_list);
        koffs[k].kin = put(img, kin);
        koffs[k].kin32 = put(img, kin32);
    }
    // LDS row of frequency i1 -> slab index
    std::vector<int> r2s(P.N1, -1);
    for (int s = 0; s < P.nslab; ++s) r2s[perm_slot_host(wrap(m1min + s, P.N1), P.N1)] = s;
    const size_t o_r2s = put(img, r2s);
    // twiddles tw[jb*A + ka] = exp(+2 pi i jb ka / N), long double then rounded
    size_t o_tw64[3], o_tw32[3];
    for (int ax = 0; ax < 3; ++ax) {
        const int n = p->fft[ax];
        int A, B;
        lds_split_host(n, &A, &B);
        std::vector<double> t64(2 * n);
        std::vector<float> t32(2 * n);
        const long double pi2 = 6.283185307179586476925286766559005768L;
        for (int jb = 0; jb < B; ++jb)
            for (int ka = 0; ka < A; ++ka) {
                const long e = ((long)jb * ka) % n;
                const long double ang = pi2 * (long double)e / (long double)n;
                const long double c = cosl(ang), s = sinl(ang);
                t64[2 * (jb * A + ka)] = (double)c;
                t64[2 * (jb * A + ka) + 1] = (double)s;
                t32[2 * (jb * A + ka)] = (float)c;
                t32[2 * (jb * A + ka) + 1] = (float)s;
            }
        o_tw64[ax] = put(img, t64);
        o_tw32[ax] = put(img, t32);
    }
    // D blocks
    std::vector<int> blo(std::max(1, p->nproj)), bn(std::max(1, p->nproj)), bdoff(std::max(1, p->nproj));
    int64_t doff = 0;
    for (int at = 0; at < p->natom && p->nproj > 0; ++at) {
        const int lo = p->proj_atom_offset[at], n = p->proj_atom_offset[at + 1] - lo;
        for (int i = lo; i < lo + n; ++i) {
            blo[i] = lo;
            bn[i] = n;
            bdoff[i] = (int)doff;
        }
        doff += (int64_t)n * n;
    }
    P.dmat_len = doff;
    const size_t o_blo = put(img, blo), o_bn = put(img, bn), o_bdoff = put(img, bdoff);

    APW_TRY(P.tables.ensure(img.size()));
    APW_HIP(hipMemcpy(P.tables.ptr, img.data(), img.size(), hipMemcpyHostToDevice));
    auto at = [&](size_t off) { return static_cast<unsigned char *>(P.tables.ptr) + off; };
    P.k.resize(p->nk);
    for (int k = 0; k < p->nk; ++k) {
        KTables &K = P.k[k];
        K.npw = p->npw[k];
        K.pw_off = P.pw_off[k];
        K.pt_off = reinterpret_cast<const int *>(at(koffs[k].pt_off));
        K.pt_g = reinterpret_cast<const int *>(at(koffs[k].pt_g));
        K.pt_pos = reinterpret_cast<const int *>(at(koffs[k].pt_pos));
        K.row_off = reinterpret_cast<const int *>(at(koffs[k].row_off));
        K.row_list = reinterpret_cast<const int *>(at(koffs[k].row_list));
        K.kin = reinterpret_cast<const double *>(at(koffs[k].kin));
        K.kin32 = reinterpret_cast<const float *>(at(koffs[k].kin32));
    }
    {
        std::vector<KDesc> kd(p->nk);
        for (int k = 0; k < p->nk; ++k) {
            const KTables &K = P.k[k];
            kd[k] = KDesc{K.pt_off, K.pt_g, K.pt_pos, K.row_off, K.row_list, K.kin, K.pw_off, K.npw, 0};
        }
        APW_TRY(P.kdesc_buf.ensure(sizeof(KDesc) * kd.size()));
        APW_HIP(hipMemcpy(P.kdesc_buf.ptr, kd.data(), sizeof(KDesc) * kd.size(), hipMemcpyHostToDevice));
        P.kdesc = P.kdesc_buf.as<const KDesc>();
    }
    P.row_to_slab = reinterpret_cast<const int *>(at(o_r2s));
    for (int ax = 0; ax < 3; ++ax) {
        P.tw64[ax] = at(o_tw64[ax]);
        P.tw32[ax] = at(o_tw32[ax]);
    }
    P.proj_blk_lo = reinterpret_cast<const int *>(at(o_blo));
    P.proj_blk_n = reinterpret_cast<const int *>(at(o_bn));
    P.proj_blk_doff = reinterpret_cast<const int *>(at(o_bdoff));

    // operator data checks (once per plan): V finite, D finite and symmetric. The
    // copies run on the caller's stream, behind whatever it has enqueued that
    // writes V or D.
    {
        std::vector<double> v((size_t)P.N);
        APW_HIP(hipMemcpyAsync(v.data(), p->vloc, sizeof(double) * (size_t)P.N, hipMemcpyDeviceToHost, st));
        APW_HIP(hipStreamSynchronize(st));
        for (double x : v)
            if (!std::isfinite(x)) return set_error(ABACUS_PW_ENONFINITE, "V_loc has a NaN or Inf");
    }
    if (p->nproj > 0) {
        std::vector<double> d((size_t)P.dmat_len);
        APW_HIP(hipMemcpyAsync(d.data(), p->dmat, sizeof(double) * (size_t)P.dmat_len, hipMemcpyDeviceToHost, st));
        APW_HIP(hipStreamSynchronize(st));
        int64_t o = 0;
        for (int at2 = 0; at2 < p->natom; ++at2) {
            const int n = p->proj_atom_offset[at2 + 1] - p->proj_atom_offset[at2];
            double mx = 0.0;
            for (int64_t q = 0; q < (int64_t)n * n; ++q) {
                if (!std::isfinite(d[o + q])) return set_error(ABACUS_PW_ENONFINITE, "D has a NaN or Inf");
                mx = std::max(mx, std::fabs(d[o + q]));
            }
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < i; ++j)
                    if (std::fabs(d[o + i * n + j] - d[o + j * n + i]) > 1e-14 * mx)
                        return set_error(ABACUS_PW_EBAD_D, "a D block is not symmetric");
            o += (int64_t)n * n;
        }
    }
    return ABACUS_PW_OK;
}

}  // namespace

int get_plan(const abacus_pw_problem *p, hipStream_t st, std::shared_ptr<Plan> &out) {
    APW_TRY(validate_problem_shallow(p));
    Key key = make_key(p);
    std::lock_guard<std::mutex> lock(g_mu);
    for (auto &e : g_cache)
        if (e.key == key) {
            e.last_use = ++g_clock;
            out = e.plan;
            return ABACUS_PW_OK;
        }
    auto plan = std::make_shared<Plan>();
    APW_TRY(build_plan(p, *plan, st));
    if (g_cache.size() >= kMaxPlans) {
        // an evicted plan lives on while a caller still holds it
        auto it = std::min_element(g_cache.begin(), g_cache.end(),
                                   [](const Entry &a, const Entry &b) { return a.last_use < b.last_use; });
        g_cache.erase(it);
    }
    g_cache.push_back(Entry{std::move(key), plan, ++g_clock});
    out = std::move(plan);
    return ABACUS_PW_OK;
}

int find_plan(const abacus_pw_problem *p, std::shared_ptr<Plan> &out) {
    APW_TRY(validate_problem_shallow(p));
    Key key = make_key(p);
    std::lock_guard<std::mutex> lock(g_mu);
    for (auto &e : g_cache)
        if (e.key == key) {
            e.last_use = ++g_clock;
            out = e.plan;
            return ABACUS_PW_OK;
        }
    out.reset();
    return ABACUS_PW_OK;
}

int plan_reset_all() {
    std::lock_guard<std::mutex> lock(g_mu);
    APW_HIP(hipDeviceSynchronize());
    g_cache.clear();
    return ABACUS_PW_OK;
}

}  // namespace apw
