// gke_plan.cpp -- the C ABI declared in include/gke.h: plan state machine,
// workspace carving, host-built tables and the launch sequence of the two
// scans (Sections "Step 1", "Step 2", "Step 3").
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/gke.h"
#include "gke_internal.h"
#include "tile_groups.h"

using gke::cx;

// Tables of one slab of output rows in the general modes (mirror average,
// FULLR domains or slabs).
struct SlabTables {
    int y1b = 0, y1e = 0;          // output rows [y1b, y1e)
    std::vector<int> rows;         // planes with accumulators (sorted, unique)
    std::vector<int> rowplane;     // rows padded to a multiple of 16 (row tiles)
    std::vector<int> rowidx;       // [ny] index in rows, -1 if absent
    std::vector<int> ta, tb;       // tile pairs (row tile, column tile)
    std::vector<int> sb;           // their groups of four (split rank-k), twelve ints each
    std::vector<int> pairs;        // pair codes in compact order
    std::vector<int> opairs;       // output pairs Y1 | Y2 << 16 in layout order
    int ntp = 0, npair_tiles = 0, npair = 0;
};

struct gke_plan_s {
    gke::Dims d{};
    std::vector<double> y;
    int dtype = GKE_DTYPE_F64;
    int prec = GKE_PREC_FP64;
    int chunk = 64;
    int pair_batch = 0;  // pairs per finalize batch (0 = all)
    int mirror = 0, domain = GKE_DOMAIN_ALLPAIRS_HALFRX, slab_rows = 0;
    int residual = 0;              // mid holds one more plane for the budget residual
    int step1 = 0;                 // buffers of the Step-1 reconstruction (gke_reconstruct)
    // block shapes chosen by an autotuner (0: the built-in rule) and their limits
    int tune_zplanes = 0, tune_kzpairs = 0, tune_kxtrans = 0;
    int max_zplanes = 1, max_kzpairs = 2, max_kxtrans = 1;
    int us[2][4] = {{0, 0, 1, 1}, {0, 0, 1, 1}};   // rx, rz undersampling: t1 t2 s1 s2
    std::vector<int> h_rzk, h_rzinv, h_rxk;        // kept separations (output rows, columns)
    // host outputs: device staging buffers of the maps, copied to the caller's
    // host arrays on a stream of the library's own
    int host_stage = 0;            // staging buffers (GKE_OPT_HOST_STAGING: 0, 1 or 2)
    char *stage = nullptr;         // host_stage buffers of stage_bytes
    size_t stage_bytes = 0, stage_slot = 0;   // a buffer holds 15 slots (14 maps, residual)
    int stage_next = 0;
    bool stage_used[2] = {false, false};
    hipStream_t copy_stream = nullptr;
    hipEvent_t ev_ready[2] = {nullptr, nullptr}, ev_copied[2] = {nullptr, nullptr};
    // notification once a finalize's maps are complete where the caller reads them
    gke_slab_fn slab_fn = nullptr;
    void *slab_user = nullptr;
    bool general = false;          // mirror, a FULLR domain or slabs
    std::vector<SlabTables> slabs;
    int cur_slab = 0;
    std::vector<int> h_rowplane;   // identity row planes of the all-pairs mode
    hipStream_t stream = nullptr;
    char *ws = nullptr;
    size_t ws_bytes = 0;

    // host copies of the tables (kept alive for the async uploads)
    std::vector<cx<double>> h_twx, h_twz;
    std::vector<cx<float>> h_twx32, h_twz32;
    std::vector<double> h_w5, h_w2;
    std::vector<int> h_j0, h_ta, h_tb, h_sb, h_pairs, h_pidx;

    // carved device pointers
    cx<double> *twx = nullptr, *twz = nullptr;
    cx<float> *twx32 = nullptr, *twz32 = nullptr;
    double *w5 = nullptr, *w2 = nullptr;
    cx<double> *s1vel = nullptr, *s1prod = nullptr, *s1ph = nullptr, *s1b = nullptr;
    double *s1u = nullptr;
    int *j0 = nullptr, *ta = nullptr, *tb = nullptr, *sblk = nullptr, *pairs = nullptr,
        *pidx = nullptr;
    int *rowplane = nullptr, *rowidx = nullptr, *opairs = nullptr;
    int *rzk = nullptr, *rzinv = nullptr, *rxk = nullptr;
    double *mf = nullptr, *band = nullptr;
    size_t mstride = 0;            // doubles per term map in mf
    double *sums1 = nullptr, *prof = nullptr, *momp = nullptr, *r0 = nullptr, *gxz = nullptr;
    double *gy1 = nullptr;   // split path: <|D u'|^2> per plane from the first scan
    void *inter = nullptr;  // cx<double> (FP64) or cx<float> (split-BF16)
    void *spec = nullptr;   // cx<double> (FP64) or gke::SplitRec records (split-BF16)
    cx<double> *acc = nullptr, *mid = nullptr;
    gke::Tables tab{};

    long long n1 = 0;          // first-scan snapshots
    long long n2 = 0;          // second-scan snapshots
    int pending = 0;           // snapshots in the current chunk
    long long chunks_done = 0;
    bool second_scan = false;
    bool means_from_host = false;
    std::string err;

    // graphs of gke_accumulate_batch: the launches of n snapshots captured once
    // and replayed while the pointers and the starting scan state match
    struct BatchGraph {
        hipGraphExec_t exec = nullptr;
        std::vector<const void *> ptrs;
        int n = 0, pending0 = 0, pending1 = 0;
        bool second = false, acc0 = false;
        long long dchunks = 0, used = 0;
    };
    std::vector<BatchGraph> graphs;    // at most kMaxGraphs
    long long graph_clock = 0;
    hipStream_t capture_stream = nullptr;

    // optional HIP-event timing of every launch
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;   // created once, reused
    std::vector<std::pair<int, int>> ev_used;  // (kernel family, pool index of start)
    double t_ms[GKE_NKERNELS] = {};
    int64_t t_n[GKE_NKERNELS] = {};
};

static std::string g_plan_error;

namespace {

gke_status fail(gke_plan_t p, gke_status s, const std::string &msg)
{
    if (p) p->err = msg;
    else g_plan_error = msg;
    return s;
}

#define GKE_HIP(plan, call)                                                         \
    do {                                                                            \
        hipError_t e_ = (call);                                                     \
        if (e_ != hipSuccess)                                                       \
            return fail(plan, GKE_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

bool factors_235(int n)
{
    for (int f : {2, 3, 5})
        while (n % f == 0) n /= f;
    return n == 1;
}

// Radices of an LDS transform: the powers of two first (8s, then 4s, then a
// 2), then 5s and 3s.  After a first pass of 8 (or 4, 2) the later passes have
// p >= 8 (or, for n = 4 or 2 times an odd number, odd radices), so their lanes
// write runs of consecutive outputs; the first pass's stride-R writes go
// through the swizzle (swz, when n is a multiple of 8).
gke::FftPlanDev radix_plan(int n)
{
    gke::FftPlanDev pl{};
    pl.n = n;
    int m = n, k = 0;
    int e2 = 0;
    while (m % 2 == 0) { ++e2; m /= 2; }
    while (e2 >= 3 && e2 != 4) { pl.radix[k++] = 8; e2 -= 3; }
    while (e2 >= 2) { pl.radix[k++] = 4; e2 -= 2; }
    if (e2 == 1) pl.radix[k++] = 2;
    while (m % 5 == 0) { pl.radix[k++] = 5; m /= 5; }
    while (m % 3 == 0) { pl.radix[k++] = 3; m /= 3; }
    pl.npass = k;
    pl.swz = k > 1 && n % 8 == 0 && pl.radix[0] % 2 == 0 ? 1 : 0;
    return pl;
}

// The twiddle table of a plan: for every pass after the first (radix R after
// radices of product p), the block [j - 1][k], j = 1..R-1, k = 0..p-1, of
// exp(-2 pi i j k / (p R)); n - R_first entries, zero-filled to n.
std::vector<cx<double>> twiddles(const gke::FftPlanDev &pl)
{
    std::vector<cx<double>> t(pl.n, cx<double>{0.0, 0.0});
    size_t off = 0;
    int p = 1;
    for (int ps = 0; ps < pl.npass; ++ps) {
        const int R = pl.radix[ps];
        if (p > 1) {
            for (int j = 1; j < R; ++j)
                for (int k = 0; k < p; ++k) {
                    const double a = 2.0 * M_PI * (double)(j * k) / (double)(p * R);
                    t[off + (size_t)(j - 1) * p + k] = cx<double>{std::cos(a), -std::sin(a)};
                }
            off += (size_t)p * (R - 1);
        }
        p *= R;
    }
    return t;
}

// First-derivative weights at x0 on the nodes x[0..n) by Fornberg's recurrence
// (B. Fornberg, Math. Comp. 51 (1988) 699-706), derivative orders 0 and 1.
void fornberg_d1(double x0, const double *x, int n, double *w)
{
    std::vector<double> c0(n, 0.0), c1(n, 0.0);
    double a = 1.0, xd = x[0] - x0;
    c0[0] = 1.0;
    for (int i = 1; i < n; ++i) {
        double b = 1.0;
        const double xd_prev = xd;
        xd = x[i] - x0;
        for (int j = 0; j < i; ++j) {
            const double dx = x[i] - x[j];
            b *= dx;
            if (j == i - 1) {
                c1[i] = a * (c0[i - 1] - xd_prev * c1[i - 1]) / b;
                c0[i] = -a * xd_prev * c0[i - 1] / b;
            }
            c1[j] = (xd * c1[j] - c0[j]) / dx;
            c0[j] = xd * c0[j] / dx;
        }
        a = b;
    }
    for (int i = 0; i < n; ++i) w[i] = c1[i];
}

// Second-derivative weights at x0 on the nodes x[0..n) by the same recurrence
// carried to derivative order 2.
void fornberg_d2(double x0, const double *x, int n, double *w)
{
    std::vector<double> c(3 * (size_t)n, 0.0);   // c[i * 3 + order]
    double c1 = 1.0, c4 = x[0] - x0;
    c[0] = 1.0;
    for (int i = 1; i < n; ++i) {
        const int mn = std::min(i, 2);
        double c2 = 1.0;
        const double c5 = c4;
        c4 = x[i] - x0;
        for (int j = 0; j < i; ++j) {
            const double c3 = x[i] - x[j];
            c2 *= c3;
            if (j == i - 1) {
                for (int k = mn; k >= 1; --k)
                    c[i * 3 + k] = c1 * (k * c[(i - 1) * 3 + k - 1] - c5 * c[(i - 1) * 3 + k]) / c2;
                c[i * 3] = -c1 * c5 * c[(i - 1) * 3] / c2;
            }
            for (int k = mn; k >= 1; --k)
                c[j * 3 + k] = (c4 * c[j * 3 + k] - k * c[j * 3 + k - 1]) / c3;
            c[j * 3] = c4 * c[j * 3] / c3;
        }
        c1 = c2;
    }
    for (int i = 0; i < n; ++i) w[i] = c[i * 3 + 2];
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }
// pair extents of acc and mid rows: whole 128-byte lines of complex FP64
template <typename I>
I round8(I n) { return (n + 7) & ~(I)7; }

// Bracket one launch with HIP events when timing is on.
template <typename F>
hipError_t timed(gke_plan_t p, int kind, F &&launch)
{
    if (!p->timing) return launch();
    const size_t need = 2 * (p->ev_used.size() + 1);
    while (p->ev_pool.size() < need) {
        hipEvent_t e;
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return r;
        p->ev_pool.push_back(e);
    }
    const int i0 = (int)(2 * p->ev_used.size());
    hipError_t r = hipEventRecord(p->ev_pool[i0], p->stream);
    if (r != hipSuccess) return r;
    r = launch();
    if (r != hipSuccess) return r;
    r = hipEventRecord(p->ev_pool[i0 + 1], p->stream);
    if (r != hipSuccess) return r;
    p->ev_used.emplace_back(kind, i0);
    return hipSuccess;
}

// Fold the recorded event pairs into the per-family totals (stream synced).
hipError_t collect_timings(gke_plan_t p)
{
    for (const auto &u : p->ev_used) {
        float ms = 0.f;
        hipError_t r = hipEventElapsedTime(&ms, p->ev_pool[u.second], p->ev_pool[u.second + 1]);
        if (r != hipSuccess) return r;
        p->t_ms[u.first] += ms;
        p->t_n[u.first] += 1;
    }
    p->ev_used.clear();
    return hipSuccess;
}

// Output rows and the Y2 range of row j1 in the plan's domain.
int domain_rows(gke_plan_t p)
{
    return p->domain == GKE_DOMAIN_FUNDAMENTAL_FULLR ? (p->d.ny - 1) / 2 + 1 : p->d.ny;
}
void domain_cols(gke_plan_t p, int j1, int &c0, int &c1)
{
    const int ny = p->d.ny;
    c0 = p->domain == GKE_DOMAIN_ALLPAIRS_HALFRX ? 0 : j1;
    c1 = p->domain == GKE_DOMAIN_FUNDAMENTAL_FULLR ? ny - j1 : ny;
}

// Tables of every slab (general modes): rows with accumulators = the slab's
// output rows, their five-point stencil rows and, with the mirror average,
// the reflections of both; tile pairs = every row tile against every column
// tile (ordered pairs); remainder pairs = every row against the last
// Ny mod 16 planes.
void build_slabs(gke_plan_t p)
{
    const gke::Dims &d = p->d;
    const int ny = d.ny, nrows = domain_rows(p);
    const int R = p->slab_rows > 0 ? std::min(p->slab_rows, nrows) : nrows;
    p->slabs.clear();
    for (int y1b = 0; y1b < nrows; y1b += R) {
        SlabTables t;
        t.y1b = y1b;
        t.y1e = std::min(nrows, y1b + R);
        std::vector<char> in(ny, 0);
        for (int j = t.y1b; j < t.y1e; ++j) {
            in[j] = 1;
            for (int a = 0; a < 5; ++a) in[p->h_j0[j] + a] = 1;
        }
        if (p->mirror)
            for (int j = 0; j < ny; ++j)
                if (in[j]) in[ny - 1 - j] = 2 | in[ny - 1 - j];
        t.rowidx.assign(ny, -1);
        for (int j = 0; j < ny; ++j)
            if (in[j]) {
                t.rowidx[j] = (int)t.rows.size();
                t.rows.push_back(j);
            }
        t.rowplane = t.rows;
        while (t.rowplane.size() % 16) t.rowplane.push_back(t.rows.back());
        const int nrt = d.ntile > 0 ? (int)t.rowplane.size() / 16 : 0;
        for (int rt = 0; rt < nrt; ++rt)
            for (int ct = 0; ct < d.ntile; ++ct) {
                t.ta.push_back(rt);
                t.tb.push_back(ct);
                for (int i = 0; i < 16; ++i)
                    for (int k = 0; k < 16; ++k)
                        t.pairs.push_back(t.rowplane[16 * rt + i] | (16 * ct + k) << 12);
            }
        t.ntp = (int)t.ta.size();
        t.npair_tiles = 256 * t.ntp;
        t.sb = gke::group_tile_pairs(t.ta, t.tb, t.ntp, false);
        for (int r : t.rows)
            for (int c = 16 * d.ntile; c < ny; ++c) t.pairs.push_back(r | c << 12);
        t.npair = (int)t.pairs.size();
        if (t.ta.empty()) {
            t.ta.push_back(0);
            t.tb.push_back(0);
        }
        for (int j1 = t.y1b; j1 < t.y1e; ++j1) {
            int c0, c1;
            domain_cols(p, j1, c0, c1);
            for (int j2 = c0; j2 < c1; ++j2) t.opairs.push_back(j1 | j2 << 16);
        }
        p->slabs.push_back(std::move(t));
    }
}

// Separations kept by the two-threshold undersampling (Section "Undersampling
// and parallelisation": full resolution below the first threshold, every s1-th
// point between the thresholds, every s2-th above the second), per direction:
// a grid index n of signed separation k (k = n, or n - N past N/2) is kept iff
// |k| < t1, or |k| < t2 and |k| is a multiple of s1, or |k| >= t2 and |k| is a
// multiple of s2.  The set is symmetric in the sign of k.
bool kept(int k, const int *u)
{
    const int m = k < 0 ? -k : k;
    if (m < u[0]) return true;
    return m < u[1] ? m % u[2] == 0 : m % u[3] == 0;
}

// Output rows (rz) and columns (rx: 0..Nx/2 in the half-plane domains, 0..Nx-1
// in the full-r ones) of the plan's maps.
void build_samples(gke_plan_t p)
{
    gke::Dims &d = p->d;
    p->h_rzk.clear();
    p->h_rzinv.assign(d.nz, -1);
    for (int q = 0; q < d.nz; ++q)
        if (kept(q <= d.nz / 2 ? q : q - d.nz, p->us[1])) {
            p->h_rzinv[q] = (int)p->h_rzk.size();
            p->h_rzk.push_back(q);
        }
    const int width = p->domain == GKE_DOMAIN_ALLPAIRS_HALFRX ? d.nkx : d.nx;
    p->h_rxk.clear();
    for (int c = 0; c < width; ++c)
        if (kept(c <= d.nx / 2 ? c : c - d.nx, p->us[0])) p->h_rxk.push_back(c);
    d.nqo = (int)p->h_rzk.size();
    d.npo = (int)p->h_rxk.size();
}

// Precision-dependent shapes of the z pass: the row groups of the
// x-transformed layout it reads, its block shape (the smaller one when the
// transforms are FP32, on the split path, and it still holds eight planes,
// measured faster there; the 512-thread one for FP64) and the planes per
// block (spread evenly over the blocks).
void set_zpass_shape(gke::Dims &d)
{
    // rows of one run of the x-transformed layout: 64-byte runs for the z pass
    // (4 rows of FP64 or 8 of FP32 complex) even when an x-pass block holds fewer
    const int zg_min = d.prec == gke::PREC_BF16X3 ? 8 : 4;
    d.zg = d.zb;
    while (d.zg < zg_min && d.nz % (2 * d.zg) == 0) d.zg *= 2;
    d.nzg = d.nz / d.zg;
    const size_t cap = std::min<size_t>(gke::LDS_BUDGET / 16 - std::max(d.nx, d.nz), gke::FFT_CAP);
    const size_t cap_small = std::min<size_t>(cap, gke::SMALL_CAP);
    const size_t sz = gke::fft_stride(d.nz);
    // split path: the record z pass transforms the four snapshots of a quad
    // together (512 threads); FP64: one snapshot, the smaller block when its
    // cap still holds eight planes
    const bool split = d.prec == gke::PREC_BF16X3;
    d.zpblk = !split && cap_small / sz >= 8 ? gke::SMALL_BLOCK : gke::FFT_BLOCK;
    const size_t capz = d.zpblk == gke::SMALL_BLOCK ? cap_small : cap;
    int jmax = std::max(1, (int)std::min<size_t>(64, capz / (split ? 4 * sz : sz)));
    if (d.zplanes > 0) jmax = std::min(jmax, d.zplanes);   // an autotuned bound
    d.njb = (d.ny + jmax - 1) / jmax;
    d.jb = (d.ny + d.njb - 1) / d.njb;
    d.nqs = (d.chunk + 3) / 4;
    // plane slots per snapshot row (FP64: 8 planes of 16 bytes per line) or per
    // record row (split: 32-byte records, a 16-plane tile on four whole lines)
    d.nys = d.prec == gke::PREC_BF16X3 ? (d.ny + 15) & ~15 : round8(d.ny);
}

// bytes of one buffer of x-transformed rows
size_t inter_bytes(const gke::Dims &d)
{
    const size_t esz = d.prec == gke::PREC_BF16X3 ? sizeof(cx<float>) : sizeof(cx<double>);
    return esz * (size_t)d.ny * d.nzg * gke::NFIELD * d.nkx * d.zg;
}

// Workspace layout; with base != nullptr also assigns the pointers.
size_t layout(gke_plan_t p, char *base)
{
    const gke::Dims &d = p->d;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align256(off + bytes);
        return base ? base + o : nullptr;
    };
    // table and accumulator extents: all pairs, or the largest slab
    size_t ntp = std::max(d.ntp, 1), npair = d.npair, nrowp = p->h_rowplane.size();
    size_t nrows = 0, nopairs = 1, nsb = std::max<size_t>(p->h_sb.size() / 12, 1);
    if (p->general) {
        ntp = npair = nrowp = nsb = 1;
        for (const auto &t : p->slabs) {
            ntp = std::max(ntp, t.ta.size());
            nsb = std::max(nsb, t.sb.size() / 12);
            npair = std::max(npair, (size_t)t.npair);
            nrowp = std::max(nrowp, t.rowplane.size());
            nrows = std::max(nrows, t.rows.size());
            nopairs = std::max(nopairs, t.opairs.size());
        }
    }
    const size_t pbt = (p->pair_batch > 0 && (size_t)p->pair_batch < npair) ? p->pair_batch : npair;
    p->twx = (cx<double> *)take(sizeof(cx<double>) * d.nx);
    p->twz = (cx<double> *)take(sizeof(cx<double>) * d.nz);
    p->twx32 = (cx<float> *)take(sizeof(cx<float>) * d.nx);
    p->twz32 = (cx<float> *)take(sizeof(cx<float>) * d.nz);
    p->w5 = (double *)take(sizeof(double) * 5 * d.ny);
    p->w2 = (double *)take(sizeof(double) * 5 * d.ny);
    p->j0 = (int *)take(sizeof(int) * d.ny);
    p->ta = (int *)take(sizeof(int) * ntp);
    p->tb = (int *)take(sizeof(int) * ntp);
    p->sblk = (int *)take(sizeof(int) * 12 * nsb);
    p->pairs = (int *)take(sizeof(int) * npair);
    p->pidx = (int *)take(sizeof(int) * d.ny * d.ny);
    p->rowplane = (int *)take(sizeof(int) * nrowp);
    p->rowidx = (int *)take(sizeof(int) * d.ny);
    p->opairs = (int *)take(sizeof(int) * nopairs);
    p->rzk = (int *)take(sizeof(int) * d.nz);
    p->rzinv = (int *)take(sizeof(int) * d.nz);
    p->rxk = (int *)take(sizeof(int) * d.nx);
    p->sums1 = (double *)take(sizeof(double) * 5 * d.ny * gke::NSPLIT);
    p->prof = (double *)take(sizeof(double) * gke::NPROF * d.ny);
    p->momp = (double *)take(sizeof(double) * d.ny * gke::NMOMP * d.nzb);
    p->r0 = (double *)take(sizeof(double) * d.ny * 5);
    p->gxz = (double *)take(sizeof(double) * d.ny);
    p->gy1 = (double *)take(sizeof(double) * d.ny);
    // split path: four x-transformed buffers of cx<float> (one per snapshot of
    // a quad) and records of four snapshots; FP64: one buffer, cx<double>
    const bool split = d.prec == gke::PREC_BF16X3;
    p->inter = take(inter_bytes(d) * (split ? 4 : 1));
    p->spec = take(split ? sizeof(gke::SplitRec) * (size_t)d.nk * gke::NFIELD * d.nqs * d.nys
                         : sizeof(cx<double>) * (size_t)d.nk * gke::NFIELD * d.chunk * d.nys);
    p->acc = (cx<double> *)take(sizeof(cx<double>) * (size_t)gke::NSPEC * d.nk * round8(npair));
    const size_t nmid = gke::NMID + (p->residual && !p->general ? 1 : 0);
    p->mid = (cx<double> *)take(sizeof(cx<double>) * nmid * d.nkx * d.nz * round8(pbt));
    p->mstride = nrows * d.ny * (size_t)d.nz * d.nx;
    p->mf = (double *)take(sizeof(double) * gke::NSTORED * p->mstride);
    p->band = (double *)take(p->general ? sizeof(double) * (size_t)d.nk * 5 * d.ny : 0);
    // staging for host outputs: 15 slots per buffer, each one FP64 map of the
    // largest output (all pairs, or the largest slab) over the kept separations
    const size_t npo_pairs = p->general ? nopairs : (size_t)d.ny * d.ny;
    p->stage_slot = align256(sizeof(double) * npo_pairs * (size_t)d.nqo * d.npo);
    p->stage_bytes = 15 * p->stage_slot;
    p->stage = (char *)take(p->host_stage * p->stage_bytes);
    // Step 1: velocity (3) and product (6) spectra, the pressure spectrum and
    // the pivot rows of its elimination
    const size_t cf = p->step1 ? (size_t)d.ny * d.nk : 0;
    p->s1vel = (cx<double> *)take(sizeof(cx<double>) * 3 * cf);
    p->s1prod = (cx<double> *)take(sizeof(cx<double>) * 6 * cf);
    p->s1ph = (cx<double> *)take(sizeof(cx<double>) * cf);
    p->s1b = (cx<double> *)take(sizeof(cx<double>) * cf);
    p->s1u = (double *)take(sizeof(double) * 9 * cf);
    return off;
}

// Make slab s current: upload its tables, set the pair extents.
gke_status select_slab(gke_plan_t p, int s)
{
    const SlabTables &t = p->slabs[s];
    hipStream_t st = p->stream;
    GKE_HIP(p, hipMemcpyAsync(p->rowplane, t.rowplane.data(), sizeof(int) * t.rowplane.size(), hipMemcpyHostToDevice, st));
    GKE_HIP(p, hipMemcpyAsync(p->rowidx, t.rowidx.data(), sizeof(int) * t.rowidx.size(), hipMemcpyHostToDevice, st));
    GKE_HIP(p, hipMemcpyAsync(p->ta, t.ta.data(), sizeof(int) * t.ta.size(), hipMemcpyHostToDevice, st));
    GKE_HIP(p, hipMemcpyAsync(p->tb, t.tb.data(), sizeof(int) * t.tb.size(), hipMemcpyHostToDevice, st));
    if (!t.sb.empty())
        GKE_HIP(p, hipMemcpyAsync(p->sblk, t.sb.data(), sizeof(int) * t.sb.size(), hipMemcpyHostToDevice, st));
    if (t.npair > 0)
        GKE_HIP(p, hipMemcpyAsync(p->pairs, t.pairs.data(), sizeof(int) * t.npair, hipMemcpyHostToDevice, st));
    if (!t.opairs.empty())
        GKE_HIP(p, hipMemcpyAsync(p->opairs, t.opairs.data(), sizeof(int) * t.opairs.size(), hipMemcpyHostToDevice, st));
    GKE_HIP(p, hipStreamSynchronize(st));
    p->d.ntp = t.ntp;
    p->d.nsb = (int)t.sb.size() / 12;
    p->d.npair_tiles = t.npair_tiles;
    p->d.npair = t.npair;
    p->d.pstr = round8(t.npair);
    p->cur_slab = s;
    return GKE_OK;
}

// split path: z transforms of the snapshots of quad q (ng of them) into records
gke_status zfft_quad(gke_plan_t p, int q, int ng)
{
    const size_t istride = inter_bytes(p->d) / sizeof(cx<float>);
    GKE_HIP(p, timed(p, GKE_K_ZFFT_PACK, [&] {
        return gke::launch_zfft_rec(p->stream, p->d, p->tab, p->inter, istride, q, ng,
                                    (gke::SplitRec *)p->spec);
    }));
    return GKE_OK;
}

// The slab notification: a host function enqueued on the stream where the
// finalize's outputs complete; it runs on a HIP runtime thread and frees its note.
struct SlabNote {
    gke_slab_fn fn;
    void *user;
    int slab;
};
void run_slab_note(void *data)
{
    SlabNote *n = static_cast<SlabNote *>(data);
    n->fn(n->slab, n->user);
    delete n;
}
gke_status notify_slab(gke_plan_t p, hipStream_t st)
{
    SlabNote *n = new (std::nothrow) SlabNote{p->slab_fn, p->slab_user, p->general ? p->cur_slab : 0};
    if (!n) return fail(p, GKE_ERR_OOM, "no host memory for the slab notification");
    const hipError_t e = hipLaunchHostFunc(st, run_slab_note, n);
    if (e != hipSuccess) {
        delete n;
        return fail(p, GKE_ERR_HIP, std::string("hipLaunchHostFunc: ") + hipGetErrorString(e));
    }
    return GKE_OK;
}

gke_status launch_flush(gke_plan_t p)
{
    if (p->pending == 0) return GKE_OK;
    const int accumulate = p->chunks_done > 0 ? 1 : 0;
    const bool split = p->d.prec == gke::PREC_BF16X3;
    if (split && (p->pending & 3)) {   // the last, partial quad
        const gke_status s = zfft_quad(p, p->pending >> 2, p->pending & 3);
        if (s != GKE_OK) return s;
    }
    const auto *s64 = (const cx<double> *)p->spec;
    const auto *s16 = (const gke::SplitRec *)p->spec;
    if (p->d.ntp > 0) {
        GKE_HIP(p, timed(p, GKE_K_RANKK, [&] {
            return split ? gke::launch_rankk_bf16x3(p->stream, p->d, p->tab, s16, p->pending,
                                                    accumulate, p->acc)
                         : gke::launch_rankk_f64(p->stream, p->d, p->tab, s64, p->pending,
                                                 accumulate, p->acc);
        }));
    }
    if (p->d.npair > p->d.npair_tiles) {
        GKE_HIP(p, timed(p, GKE_K_RANKK_REM, [&] {
            return split ? gke::launch_rankk_rem_bf16x3(p->stream, p->d, p->tab, s16, p->pending,
                                                        accumulate, p->acc)
                         : gke::launch_rankk_rem_f64(p->stream, p->d, p->tab, s64, p->pending,
                                                     accumulate, p->acc);
        }));
    }
    if (p->general)  // eps needs the band pairs of every plane, not only the slab's
        GKE_HIP(p, timed(p, GKE_K_SMALL, [&] {
            return gke::launch_band(p->stream, p->d, p->spec, p->pending, accumulate, p->band);
        }));
    ++p->chunks_done;
    p->pending = 0;
    return GKE_OK;
}

// ---------------------------------------------------------------------------
// Checkpoint of the accumulation state: a header, the one-point sums and
// moment partials ([sums1, inter) of the workspace), the cross-spectral
// accumulators and, in the general modes, the band accumulators.

constexpr char kStateMagic[8] = {'G', 'K', 'E', 'S', 'T', 'A', 'T', '1'};
struct StateHeader {
    char magic[8];
    int32_t nx, ny, nz, prec, dtype, mirror, domain, slab_rows, cur_slab, second_scan,
        means_from_host, pad;
    uint64_t cfg;                                  // hash of y, Lx, Lz, nu and the undersampling
    int64_t n1, n2, chunks_done;
    uint64_t small_bytes, acc_bytes, band_bytes;   // the three sections that follow
};

uint64_t fnv1a(uint64_t h, const void *data, size_t n)
{
    const unsigned char *b = static_cast<const unsigned char *>(data);
    for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
    return h;
}

StateHeader state_header(gke_plan_t p)
{
    StateHeader h{};
    std::memcpy(h.magic, kStateMagic, 8);
    const gke::Dims &d = p->d;
    h.nx = d.nx;
    h.ny = d.ny;
    h.nz = d.nz;
    h.prec = d.prec;
    h.dtype = p->dtype;
    h.mirror = p->mirror;
    h.domain = p->domain;
    h.slab_rows = p->slab_rows;
    h.cur_slab = p->general ? p->cur_slab : 0;
    h.second_scan = p->second_scan ? 1 : 0;
    h.means_from_host = p->means_from_host ? 1 : 0;
    uint64_t c = 1469598103934665603ull;
    c = fnv1a(c, p->y.data(), sizeof(double) * p->y.size());
    c = fnv1a(c, &d.lx, sizeof(double));
    c = fnv1a(c, &d.lz, sizeof(double));
    c = fnv1a(c, &d.nu, sizeof(double));
    c = fnv1a(c, p->us, sizeof(p->us));
    h.cfg = c;
    h.n1 = p->n1;
    h.n2 = p->n2;
    h.chunks_done = p->chunks_done;
    h.small_bytes = (uint64_t)((char *)p->inter - (char *)p->sums1);
    h.acc_bytes = (uint64_t)sizeof(cx<double>) * gke::NSPEC * d.nk * d.pstr;
    h.band_bytes = p->general ? (uint64_t)sizeof(double) * d.nk * 5 * d.ny : 0;
    return h;
}

size_t state_bytes(const StateHeader &h)
{
    return sizeof(StateHeader) + h.small_bytes + h.acc_bytes + h.band_bytes;
}

}  // namespace

extern "C" {

gke_status gke_plan(int Nx, int Ny, int Nz, const double *y, double Lx, double Lz, double nu,
                    gke_plan_t *out)
{
    if (!out) return fail(nullptr, GKE_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!y) return fail(nullptr, GKE_ERR_ARG, "y is NULL");
    if (Nx < 4 || Nz < 4 || Nx % 2 || Nz % 2)
        return fail(nullptr, GKE_ERR_ARG, "Nx and Nz must be even and >= 4");
    if (!factors_235(Nx) || !factors_235(Nz))
        return fail(nullptr, GKE_ERR_ARG, "Nx and Nz must factor into 2, 3 and 5");
    if (Nx > 4096 || Nz > 4096) return fail(nullptr, GKE_ERR_UNSUPPORTED, "Nx, Nz > 4096");
    if (Ny < 5 || Ny > 4096) return fail(nullptr, GKE_ERR_ARG, "Ny must be in [5, 4096]");
    if (!(Lx > 0) || !(Lz > 0) || !(nu > 0))
        return fail(nullptr, GKE_ERR_ARG, "Lx, Lz and nu must be positive");
    for (int j = 1; j < Ny; ++j)
        if (!(y[j] > y[j - 1])) return fail(nullptr, GKE_ERR_ARG, "y must be strictly increasing");
    gke_plan_t p = new (std::nothrow) gke_plan_s();
    if (!p) return fail(nullptr, GKE_ERR_OOM, "host allocation failed");
    p->y.assign(y, y + Ny);
    gke::Dims &d = p->d;
    d.nx = Nx;
    d.ny = Ny;
    d.nz = Nz;
    d.nkx = Nx / 2 + 1;
    d.nk = d.nkx * Nz;
    d.ntile = Ny / 16;
    d.ntp = d.ntile * (d.ntile + 1) / 2;
    d.npair_tiles = 256 * d.ntp;
    // tile entries (diagonal tiles hold both orientations) + remainder pairs
    d.npair = d.npair_tiles + Ny * (Ny + 1) / 2 - (16 * d.ntile) * (16 * d.ntile + 1) / 2;
    d.pstr = round8(d.npair);
    d.lx = Lx;
    d.lz = Lz;
    d.nu = nu;
    // block shapes of the LDS transforms (complex FP64 elements, one buffer)
    // batch * stride <= cap bounds both the LDS bytes (plus the twiddle table)
    // and the per-thread work of the register-staged passes
    const size_t cap = std::min<size_t>(gke::LDS_BUDGET / 16 - std::max(Nx, Nz), gke::FFT_CAP);
    const size_t sx = gke::fft_stride(Nx), sz = gke::fft_stride(Nz);
    if (sx * 5 > cap || sz > cap) {
        delete p;
        return fail(nullptr, GKE_ERR_UNSUPPORTED, "transform length too large for one block");
    }
    // the smaller block shape of the kx finalize when its cap still holds
    // eight transforms; the x pass always takes the larger one (four z rows
    // per block at re200, measured faster than two in 256-thread blocks)
    const size_t cap_small = std::min<size_t>(cap, gke::SMALL_CAP);
    d.kxblk = cap_small / sx >= 8 ? gke::SMALL_BLOCK : gke::FFT_BLOCK;
    const size_t capkx = d.kxblk == gke::SMALL_BLOCK ? cap_small : cap;
    // x pass: 5 complex rows per z row (ten real fields), zb | Nz
    d.zb = 16;
    while (d.zb > 1 && (Nz % d.zb || (size_t)5 * d.zb * sx > cap)) d.zb >>= 1;
    d.nzb = Nz / d.zb;
    set_zpass_shape(d);
    // finalize: pairs per kz block, complex transforms (2 pairs each) per kx block
    // (kz pass: multiples of 8 pairs where possible, 128-byte runs of acc and
    // mid; 16 pairs let three blocks share a compute unit, measured faster
    // than 24 at re200)
    d.pbz = (int)std::min<size_t>(16, cap / sz);
    d.pbz &= d.pbz >= 8 ? ~7 : ~1;   // even: the R blocks split it in halves
    // (kx pass: at most 8 transforms, five blocks per compute unit at re200,
    // measured faster than ten)
    d.ntx = (int)std::min<size_t>(8, capkx / sx);
    // limits of the autotuned shapes: the LDS caps above
    p->max_kzpairs = (int)std::min<size_t>(16, cap / sz) & ~1;
    p->max_kxtrans = (int)std::min<size_t>(gke::MAX_NTX, capkx / sx);
    p->max_zplanes = 64;
    // 32-bit element offsets within one wavenumber row of acc (kz pass)
    if (d.zb < 1 || d.jb < 1 || d.pbz < 2 || d.ntx < 1 || (size_t)Nz * d.pstr >= ((size_t)1 << 31)) {
        delete p;
        return fail(nullptr, GKE_ERR_UNSUPPORTED, "grid too large for the LDS transforms");
    }
    d.chunk = p->chunk;

    p->h_twx = twiddles(radix_plan(Nx));
    p->h_twz = twiddles(radix_plan(Nz));
    for (const auto &c : p->h_twx) p->h_twx32.push_back(cx<float>{(float)c.x, (float)c.y});
    for (const auto &c : p->h_twz) p->h_twz32.push_back(cx<float>{(float)c.x, (float)c.y});
    p->h_w5.assign(5 * (size_t)Ny, 0.0);
    p->h_j0.assign(Ny, 0);
    for (int j = 0; j < Ny; ++j) {
        const int s = std::min(std::max(j - 2, 0), Ny - 5);
        p->h_j0[j] = s;
        fornberg_d1(y[j], y + s, 5, &p->h_w5[5 * (size_t)j]);
    }
    p->h_w2.assign(5 * (size_t)Ny, 0.0);
    for (int j = 0; j < Ny; ++j)
        fornberg_d2(y[j], y + p->h_j0[j], 5, &p->h_w2[5 * (size_t)j]);
    // pair table: tile pairs (a <= b) element by element, then the pairs of
    // the remainder planes j2 >= 16 ntile with j1 <= j2
    for (int a = 0; a < d.ntile; ++a)
        for (int b = a; b < d.ntile; ++b) {
            p->h_ta.push_back(a);
            p->h_tb.push_back(b);
            for (int i = 0; i < 16; ++i)
                for (int k = 0; k < 16; ++k)
                    p->h_pairs.push_back((16 * a + i) | (16 * b + k) << 12 | (a < b ? 1 : 0) << 24);
        }
    p->h_sb = gke::group_tile_pairs(p->h_ta, p->h_tb, d.ntp, true);
    d.nsb = (int)p->h_sb.size() / 12;
    if (p->h_ta.empty()) {
        p->h_ta.push_back(0);
        p->h_tb.push_back(0);
    }
    for (int j2 = 16 * d.ntile; j2 < Ny; ++j2)
        for (int j1 = 0; j1 <= j2; ++j1)
            p->h_pairs.push_back(j1 | j2 << 12 | (j1 < j2 ? 1 : 0) << 24);
    if ((int)p->h_pairs.size() != d.npair) {
        delete p;
        return fail(nullptr, GKE_ERR_UNSUPPORTED, "internal pair count mismatch");
    }
    // compact index of every plane pair, either order
    p->h_pidx.assign((size_t)Ny * Ny, -1);
    for (int P = 0; P < d.npair; ++P) {
        const int j1 = gke::pair_j1(p->h_pairs[P]), j2 = gke::pair_j2(p->h_pairs[P]);
        if (p->h_pidx[(size_t)j1 * Ny + j2] < 0) p->h_pidx[(size_t)j1 * Ny + j2] = P;
        if (p->h_pidx[(size_t)j2 * Ny + j1] < 0) p->h_pidx[(size_t)j2 * Ny + j1] = P;
    }
    for (int v : p->h_pidx)
        if (v < 0) {
            delete p;
            return fail(nullptr, GKE_ERR_UNSUPPORTED, "internal pair table incomplete");
        }
    for (int i = 0; i < std::max(16 * d.ntile, 1); ++i) p->h_rowplane.push_back(i);
    p->tab.px = radix_plan(Nx);
    p->tab.pz = radix_plan(Nz);
    *out = p;
    return GKE_OK;
}

gke_status gke_set_option(gke_plan_t p, int key, int64_t value)
{
    if (!p) return fail(nullptr, GKE_ERR_ARG, "plan is NULL");
    if (key == GKE_OPT_TIMING) {
        if (value != 0 && value != 1) return fail(p, GKE_ERR_ARG, "timing must be 0 or 1");
        p->timing = value != 0;
        return GKE_OK;
    }
    if (p->ws) return fail(p, GKE_ERR_STATE, "options are fixed once the workspace is set");
    switch (key) {
    case GKE_OPT_DTYPE:
        if (value != GKE_DTYPE_F64 && value != GKE_DTYPE_F32)
            return fail(p, GKE_ERR_ARG, "dtype must be GKE_DTYPE_F64 or GKE_DTYPE_F32");
        p->dtype = (int)value;
        return GKE_OK;
    case GKE_OPT_PRECISION:
        if (value != GKE_PREC_FP64 && value != GKE_PREC_BF16X3)
            return fail(p, GKE_ERR_ARG, "unknown precision");
        p->prec = (int)value;
        p->d.prec = value == GKE_PREC_BF16X3 ? gke::PREC_BF16X3 : gke::PREC_FP64;
        return GKE_OK;
    case GKE_OPT_CHUNK:
        if (value != 0 && (value < 2 || value > 4096 || value % 2))
            return fail(p, GKE_ERR_ARG, "chunk must be 0 or even and in [2, 4096]");
        p->chunk = (int)value;
        p->d.chunk = (int)value;
        return GKE_OK;
    case GKE_OPT_PAIR_BATCH:
        if (value < 0 || value > 1000000) return fail(p, GKE_ERR_ARG, "bad pair batch");
        p->pair_batch = (int)value;
        return GKE_OK;
    case GKE_OPT_MIRROR: {
        if (value != 0 && value != 1) return fail(p, GKE_ERR_ARG, "mirror must be 0 or 1");
        if (value == 1) {
            const int ny = p->d.ny;
            const double span = p->y[ny - 1] - p->y[0], c = p->y[0] + p->y[ny - 1];
            for (int j = 0; j < ny; ++j)
                if (std::fabs(p->y[ny - 1 - j] - (c - p->y[j])) > 1e-13 * span)
                    return fail(p, GKE_ERR_ARG, "mirror needs a y grid symmetric about its centre");
        }
        p->mirror = (int)value;
        return GKE_OK;
    }
    case GKE_OPT_DOMAIN:
        if (value != GKE_DOMAIN_ALLPAIRS_HALFRX && value != GKE_DOMAIN_Y1LEY2_FULLR &&
            value != GKE_DOMAIN_FUNDAMENTAL_FULLR)
            return fail(p, GKE_ERR_ARG, "unknown output domain");
        p->domain = (int)value;
        return GKE_OK;
    case GKE_OPT_SLAB:
        if (value < 0 || value > 4096) return fail(p, GKE_ERR_ARG, "slab rows must be in [0, 4096]");
        p->slab_rows = (int)value;
        return GKE_OK;
    case GKE_OPT_RESIDUAL:
        if (value != 0 && value != 1) return fail(p, GKE_ERR_ARG, "residual must be 0 or 1");
        p->residual = (int)value;
        return GKE_OK;
    case GKE_OPT_HOST_STAGING:
        if (value < 0 || value > 2) return fail(p, GKE_ERR_ARG, "host staging must be 0, 1 or 2");
        p->host_stage = (int)value;
        return GKE_OK;
    case GKE_OPT_STEP1:
        if (value != 0 && value != 1) return fail(p, GKE_ERR_ARG, "step1 must be 0 or 1");
        p->step1 = (int)value;
        return GKE_OK;
    case GKE_OPT_TUNE_ZPLANES:
        if (value < 0 || value > p->max_zplanes)
            return fail(p, GKE_ERR_ARG, "z-pass planes per block out of range");
        p->tune_zplanes = (int)value;
        return GKE_OK;
    case GKE_OPT_TUNE_KZPAIRS:
        if (value < 0 || value > p->max_kzpairs || (value & 1))
            return fail(p, GKE_ERR_ARG, "kz-finalize pairs per block must be even and within the "
                                        "block's LDS (" + std::to_string(p->max_kzpairs) + ")");
        p->tune_kzpairs = (int)value;
        return GKE_OK;
    case GKE_OPT_TUNE_KXTRANS:
        if (value < 0 || value > p->max_kxtrans)
            return fail(p, GKE_ERR_ARG, "kx-finalize transforms per block out of range (max " +
                                            std::to_string(p->max_kxtrans) + ")");
        p->tune_kxtrans = (int)value;
        return GKE_OK;
    default:
        return fail(p, GKE_ERR_ARG, "unknown option key");
    }
}

// Fix the output mode and the automatic chunk from the options (before sizing
// the workspace).  Chunk 0: the most snapshots per cross-spectral batch whose
// spectra fit kAutoChunkBytes (every batch re-reads and re-writes the
// accumulators, so fewer, larger batches move fewer bytes), in [8, 512].
// (96 GiB: a third of the 288 GB of HBM; at re200 the split path then takes
// 512 snapshots in one batch, measured 7 ms per step faster than two)
constexpr size_t kAutoChunkBytes = (size_t)96 << 30;
gke_status prepare_mode(gke_plan_t p)
{
    // autotuned block shapes (0 keeps the built-in rule)
    p->d.zplanes = p->tune_zplanes;
    if (p->tune_kzpairs > 0) p->d.pbz = p->tune_kzpairs;
    if (p->tune_kxtrans > 0) p->d.ntx = p->tune_kxtrans;
    set_zpass_shape(p->d);
    if (p->chunk == 0) {
        const size_t esz = p->d.prec == gke::PREC_BF16X3 ? 8 : 16;
        const size_t per = esz * (size_t)p->d.nk * gke::NFIELD * p->d.nys;
        size_t c = kAutoChunkBytes / per;
        c = std::max<size_t>(8, std::min<size_t>(512, c)) & ~(size_t)1;
        p->d.chunk = (int)c;
    }
    p->d.nqs = (p->d.chunk + 3) / 4;
    // 32-bit element offsets within the spectra of one kx (z pass, rank-k)
    if ((size_t)p->d.nz * gke::NFIELD * p->d.chunk * p->d.nys >= ((size_t)1 << 31))
        return fail(p, GKE_ERR_UNSUPPORTED, "chunk too large for this grid");
    // the record z pass holds the four snapshots of a quad in one block
    if (p->d.prec == gke::PREC_BF16X3 &&
        (size_t)4 * gke::fft_stride(p->d.nz) > (size_t)gke::FFT_CAP)
        return fail(p, GKE_ERR_UNSUPPORTED, "Nz too long for the split-path z pass");
    if (p->domain == GKE_DOMAIN_FUNDAMENTAL_FULLR && !p->mirror)
        return fail(p, GKE_ERR_ARG, "the fundamental domain needs GKE_OPT_MIRROR = 1");
    p->general = p->mirror || p->domain != GKE_DOMAIN_ALLPAIRS_HALFRX || p->slab_rows > 0;
    if (p->general) build_slabs(p);
    else p->slabs.clear();
    build_samples(p);
    return GKE_OK;
}

gke_status gke_get_option(gke_plan_t p, int key, int64_t *value)
{
    if (!p || !value) return fail(p, GKE_ERR_ARG, "NULL argument");
    switch (key) {
    case GKE_OPT_DTYPE: *value = p->dtype; return GKE_OK;
    case GKE_OPT_PRECISION: *value = p->prec; return GKE_OK;
    case GKE_OPT_CHUNK: *value = p->d.chunk; return GKE_OK;
    case GKE_OPT_PAIR_BATCH: *value = p->pair_batch; return GKE_OK;
    case GKE_OPT_TIMING: *value = p->timing ? 1 : 0; return GKE_OK;
    case GKE_OPT_MIRROR: *value = p->mirror; return GKE_OK;
    case GKE_OPT_DOMAIN: *value = p->domain; return GKE_OK;
    case GKE_OPT_SLAB: *value = p->slab_rows; return GKE_OK;
    case GKE_OPT_RESIDUAL: *value = p->residual; return GKE_OK;
    case GKE_OPT_HOST_STAGING: *value = p->host_stage; return GKE_OK;
    case GKE_OPT_STEP1: *value = p->step1; return GKE_OK;
    case GKE_OPT_TUNE_ZPLANES: *value = p->d.jb; return GKE_OK;
    case GKE_OPT_TUNE_KZPAIRS: *value = p->d.pbz; return GKE_OK;
    case GKE_OPT_TUNE_KXTRANS: *value = p->d.ntx; return GKE_OK;
    default: return fail(p, GKE_ERR_ARG, "unknown option key");
    }
}

gke_status gke_workspace_size(gke_plan_t p, size_t *bytes)
{
    if (!p || !bytes) return fail(p, GKE_ERR_ARG, "NULL argument");
    if (!p->ws) {
        gke_status s = prepare_mode(p);
        if (s != GKE_OK) return s;
    }
    *bytes = layout(p, nullptr);
    return GKE_OK;
}

}  // extern "C"

namespace {

// Carve a device buffer of `bytes` (256-byte aligned, at least the layout's
// size, options already fixed by prepare_mode) into the plan's workspace:
// upload the tables and clear the sums, profiles and moment partials.
gke_status attach_workspace(gke_plan_t p, void *dev, size_t bytes)
{
    p->ws = (char *)dev;
    p->ws_bytes = bytes;
    layout(p, p->ws);
    const gke::Dims &d = p->d;
    hipStream_t st = p->stream;
    GKE_HIP(p, hipMemcpyAsync(p->twx, p->h_twx.data(), sizeof(cx<double>) * d.nx, hipMemcpyHostToDevice, st));
    GKE_HIP(p, hipMemcpyAsync(p->twz, p->h_twz.data(), sizeof(cx<double>) * d.nz, hipMemcpyHostToDevice, st));
    GKE_HIP(p, hipMemcpyAsync(p->twx32, p->h_twx32.data(), sizeof(cx<float>) * d.nx, hipMemcpyHostToDevice, st));
    GKE_HIP(p, hipMemcpyAsync(p->twz32, p->h_twz32.data(), sizeof(cx<float>) * d.nz, hipMemcpyHostToDevice, st));
    GKE_HIP(p, hipMemcpyAsync(p->w5, p->h_w5.data(), sizeof(double) * 5 * d.ny, hipMemcpyHostToDevice, st));
    GKE_HIP(p, hipMemcpyAsync(p->w2, p->h_w2.data(), sizeof(double) * 5 * d.ny, hipMemcpyHostToDevice, st));
    GKE_HIP(p, hipMemcpyAsync(p->j0, p->h_j0.data(), sizeof(int) * d.ny, hipMemcpyHostToDevice, st));
    if (!p->general) {  // all-pairs tables (a slab uploads its own)
        GKE_HIP(p, hipMemcpyAsync(p->ta, p->h_ta.data(), sizeof(int) * p->h_ta.size(), hipMemcpyHostToDevice, st));
        GKE_HIP(p, hipMemcpyAsync(p->tb, p->h_tb.data(), sizeof(int) * p->h_tb.size(), hipMemcpyHostToDevice, st));
        if (!p->h_sb.empty())
            GKE_HIP(p, hipMemcpyAsync(p->sblk, p->h_sb.data(), sizeof(int) * p->h_sb.size(), hipMemcpyHostToDevice, st));
        GKE_HIP(p, hipMemcpyAsync(p->pairs, p->h_pairs.data(), sizeof(int) * d.npair, hipMemcpyHostToDevice, st));
        GKE_HIP(p, hipMemcpyAsync(p->rowplane, p->h_rowplane.data(), sizeof(int) * p->h_rowplane.size(), hipMemcpyHostToDevice, st));
    }
    GKE_HIP(p, hipMemcpyAsync(p->pidx, p->h_pidx.data(), sizeof(int) * d.ny * d.ny, hipMemcpyHostToDevice, st));
    GKE_HIP(p, hipMemcpyAsync(p->rzk, p->h_rzk.data(), sizeof(int) * p->h_rzk.size(), hipMemcpyHostToDevice, st));
    GKE_HIP(p, hipMemcpyAsync(p->rzinv, p->h_rzinv.data(), sizeof(int) * d.nz, hipMemcpyHostToDevice, st));
    GKE_HIP(p, hipMemcpyAsync(p->rxk, p->h_rxk.data(), sizeof(int) * p->h_rxk.size(), hipMemcpyHostToDevice, st));
    if (p->host_stage > 0 && !p->copy_stream) {
        GKE_HIP(p, hipStreamCreateWithFlags(&p->copy_stream, hipStreamNonBlocking));
        for (int b = 0; b < 2; ++b) {
            GKE_HIP(p, hipEventCreateWithFlags(&p->ev_ready[b], hipEventDisableTiming));
            GKE_HIP(p, hipEventCreateWithFlags(&p->ev_copied[b], hipEventDisableTiming));
        }
    }
    // sums, profiles and moment partials start at zero
    GKE_HIP(p, gke::launch_zero(st, p->sums1, (char *)p->inter - (char *)p->sums1));
    GKE_HIP(p, hipStreamSynchronize(st));
    p->tab.twx = p->twx;
    p->tab.twz = p->twz;
    p->tab.twx32 = p->twx32;
    p->tab.twz32 = p->twz32;
    p->tab.w5 = p->w5;
    p->tab.w2 = p->w2;
    p->tab.j0 = p->j0;
    p->tab.tile_a = p->ta;
    p->tab.tile_b = p->tb;
    p->tab.sblk = p->sblk;
    p->tab.pairs = p->pairs;
    p->tab.pidx = p->pidx;
    p->tab.rowplane = p->rowplane;
    p->tab.rowidx = p->rowidx;
    p->tab.rzk = p->rzk;
    p->tab.rzinv = p->rzinv;
    p->tab.rxk = p->rxk;
    if (p->general) return select_slab(p, 0);
    return GKE_OK;
}

// The library-owned workspace of gke_set_static_workspace: one copy per GPU,
// held until the process ends.  Host code never uses the array's name as an
// address; it takes the per-device address from hipGetSymbolAddress.
__device__ __align__(256) unsigned char scratch[GKE_STATIC_WORKSPACE_BYTES];

std::mutex g_scratch_mu;
std::vector<void *> g_scratch_ptr;   // [device] address of `scratch` on that device

// Address of `scratch` on the current device (looked up once per device).
gke_status static_scratch(gke_plan_t p, void **out)
{
    int dev = -1;
    GKE_HIP(p, hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (dev < 0) return fail(p, GKE_ERR_HIP, "no current device");
    if ((size_t)dev >= g_scratch_ptr.size()) g_scratch_ptr.resize(dev + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        void *a = nullptr;
        GKE_HIP(p, hipGetSymbolAddress(&a, HIP_SYMBOL(scratch)));
        if (!a || ((uintptr_t)a & 255)) return fail(p, GKE_ERR_HIP, "static workspace address");
        g_scratch_ptr[dev] = a;
    }
    *out = g_scratch_ptr[dev];
    return GKE_OK;
}

}  // namespace

extern "C" {

gke_status gke_set_workspace(gke_plan_t p, void *dev, size_t bytes)
{
    if (!p) return fail(nullptr, GKE_ERR_ARG, "plan is NULL");
    if (p->ws) return fail(p, GKE_ERR_STATE, "workspace already set");
    if (!dev || ((uintptr_t)dev & 255)) return fail(p, GKE_ERR_ARG, "workspace NULL or not 256-byte aligned");
    {
        gke_status s = prepare_mode(p);
        if (s != GKE_OK) return s;
    }
    const size_t need = layout(p, nullptr);
    if (bytes < need)
        return fail(p, GKE_ERR_OOM, "workspace too small: need " + std::to_string(need) + " bytes");
    return attach_workspace(p, dev, bytes);
}

gke_status gke_set_static_workspace(gke_plan_t p)
{
    if (!p) return fail(nullptr, GKE_ERR_ARG, "plan is NULL");
    if (p->ws) return fail(p, GKE_ERR_STATE, "workspace already set");
    {
        gke_status s = prepare_mode(p);
        if (s != GKE_OK) return s;
    }
    if (p->host_stage > 0)
        return fail(p, GKE_ERR_UNSUPPORTED, "host staging (a copy stream of its own) needs a "
                                            "caller workspace");
    const size_t need = layout(p, nullptr);
    if (need > (size_t)GKE_STATIC_WORKSPACE_BYTES)
        return fail(p, GKE_ERR_OOM, "the plan needs " + std::to_string(need) +
                                        " workspace bytes; the static workspace holds " +
                                        std::to_string((size_t)GKE_STATIC_WORKSPACE_BYTES));
    void *dev = nullptr;
    {
        gke_status s = static_scratch(p, &dev);
        if (s != GKE_OK) return s;
    }
    return attach_workspace(p, dev, (size_t)GKE_STATIC_WORKSPACE_BYTES);
}

gke_status gke_set_undersampling(gke_plan_t p, int dir, int t1, int t2, int s1, int s2)
{
    if (!p) return fail(nullptr, GKE_ERR_ARG, "plan is NULL");
    if (p->ws) return fail(p, GKE_ERR_STATE, "undersampling is fixed once the workspace is set");
    if (dir != 0 && dir != 1) return fail(p, GKE_ERR_ARG, "dir must be 0 (rx) or 1 (rz)");
    if (t1 < 0 || t2 < t1 || s1 < 1 || s2 < 1)
        return fail(p, GKE_ERR_ARG, "need 0 <= t1 <= t2 and steps >= 1");
    const int u[4] = {t1, t2, s1, s2};
    for (int k = 0; k < 4; ++k) p->us[dir][k] = u[k];
    return GKE_OK;
}

gke_status gke_sample_indices(gke_plan_t p, int dir, int *count, int *idx)
{
    if (!p || !count) return fail(p, GKE_ERR_ARG, "NULL argument");
    if (dir != 0 && dir != 1) return fail(p, GKE_ERR_ARG, "dir must be 0 (rx) or 1 (rz)");
    if (!p->ws) {   // the lists follow the options in effect
        gke_status s = prepare_mode(p);
        if (s != GKE_OK) return s;
    }
    const std::vector<int> &v = dir == 0 ? p->h_rxk : p->h_rzk;
    *count = (int)v.size();
    if (idx) std::copy(v.begin(), v.end(), idx);
    return GKE_OK;
}

gke_status gke_set_stream(gke_plan_t p, void *stream)
{
    if (!p) return fail(nullptr, GKE_ERR_ARG, "plan is NULL");
    p->stream = (hipStream_t)stream;
    return GKE_OK;
}

gke_status gke_accumulate(gke_plan_t p, const void *u, const void *v, const void *w,
                          const void *pr)
{
    if (!p) return fail(nullptr, GKE_ERR_ARG, "plan is NULL");
    if (!u || !v || !w || !pr) return fail(p, GKE_ERR_ARG, "field pointer is NULL");
    if (!p->ws) return fail(p, GKE_ERR_STATE, "no workspace");
    const int f32 = p->dtype == GKE_DTYPE_F32;
    if (!p->second_scan) {
        GKE_HIP(p, timed(p, GKE_K_PLANE_SUMS, [&] {
            // split path: also the wall-normal gradient energy (first scan)
            return gke::launch_plane_sums(p->stream, p->d, p->tab, f32,
                                          p->d.prec == gke::PREC_BF16X3 ? 1 : 0, u, v, w, pr,
                                          p->sums1);
        }));
        ++p->n1;
        return GKE_OK;
    }
    const bool split = p->d.prec == gke::PREC_BF16X3;
    // split path: snapshot i of a quad in x-transformed buffer i
    void *xdst = split ? (void *)((char *)p->inter + (p->pending & 3) * inter_bytes(p->d))
                       : p->inter;
    // the gradient energy by the x pass's stencil only when the first scan
    // did not sum it (means given by the caller)
    const int gy = split && p->means_from_host ? 1 : 0;
    GKE_HIP(p, timed(p, GKE_K_FLUCT_XFFT, [&] {
        return gke::launch_fluct_xfft(p->stream, p->d, p->tab, f32, gy, u, v, w, pr, p->prof,
                                      xdst, p->momp);
    }));
    if (!split)
        GKE_HIP(p, timed(p, GKE_K_ZFFT_PACK, [&] {
            return gke::launch_zfft_pack(p->stream, p->d, p->tab, p->inter, p->pending, p->spec);
        }));
    ++p->pending;
    ++p->n2;
    if (split && (p->pending & 3) == 0) {
        const gke_status s = zfft_quad(p, (p->pending >> 2) - 1, 4);
        if (s != GKE_OK) return s;
    }
    if (p->pending == p->d.chunk) return launch_flush(p);
    return GKE_OK;
}

gke_status gke_accumulate_batch(gke_plan_t p, int n, const void *const *u,
                                const void *const *v, const void *const *w,
                                const void *const *pr)
{
    constexpr size_t kMaxGraphs = 4;
    if (!p) return fail(nullptr, GKE_ERR_ARG, "plan is NULL");
    if (n <= 0 || !u || !v || !w || !pr) return fail(p, GKE_ERR_ARG, "bad batch");
    if (!p->ws) return fail(p, GKE_ERR_STATE, "no workspace");
    for (int i = 0; i < n; ++i)
        if (!u[i] || !v[i] || !w[i] || !pr[i]) return fail(p, GKE_ERR_ARG, "field pointer is NULL");
    if (p->timing) {   // per-launch events: run the launches one by one
        for (int i = 0; i < n; ++i) {
            const gke_status s = gke_accumulate(p, u[i], v[i], w[i], pr[i]);
            if (s != GKE_OK) return s;
        }
        return GKE_OK;
    }
    std::vector<const void *> ptrs;
    ptrs.reserve(4 * (size_t)n);
    for (int i = 0; i < n; ++i) {
        ptrs.push_back(u[i]);
        ptrs.push_back(v[i]);
        ptrs.push_back(w[i]);
        ptrs.push_back(pr[i]);
    }
    const bool acc0 = p->chunks_done > 0;
    gke_plan_s::BatchGraph *g = nullptr;
    for (auto &e : p->graphs)
        if (e.exec && e.n == n && e.second == p->second_scan && e.pending0 == p->pending &&
            e.acc0 == acc0 && e.ptrs == ptrs) {
            g = &e;
            break;
        }
    if (g) {   // replay: advance the host state as the captured calls did
        if (g->second) {
            p->n2 += n;
            p->pending = g->pending1;
            p->chunks_done += g->dchunks;
        } else {
            p->n1 += n;
        }
    } else {
        // capture the launches of the n calls on a stream of the library's own
        // (the plan's stream may be the legacy default stream, which cannot be
        // captured), then launch the graph on the plan's stream
        if (!p->capture_stream)
            GKE_HIP(p, hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking));
        const int pending0 = p->pending;
        const long long chunks0 = p->chunks_done;
        const bool second = p->second_scan;
        hipStream_t user = p->stream;
        p->stream = p->capture_stream;
        GKE_HIP(p, hipStreamBeginCapture(p->capture_stream, hipStreamCaptureModeThreadLocal));
        gke_status st = GKE_OK;
        for (int i = 0; i < n && st == GKE_OK; ++i) st = gke_accumulate(p, u[i], v[i], w[i], pr[i]);
        hipGraph_t graph = nullptr;
        const hipError_t ec = hipStreamEndCapture(p->capture_stream, &graph);
        p->stream = user;
        if (st != GKE_OK || ec != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            if (st != GKE_OK) return st;
            return fail(p, GKE_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ec));
        }
        // a new entry, or the least recently used one updated in place
        if (p->graphs.size() < kMaxGraphs) {
            p->graphs.emplace_back();
            g = &p->graphs.back();
        } else {
            g = &p->graphs[0];
            for (auto &e : p->graphs)
                if (e.used < g->used) g = &e;
        }
        bool updated = false;
        if (g->exec) {
            hipGraphNode_t bad = nullptr;
            hipGraphExecUpdateResult res;
            updated = hipGraphExecUpdate(g->exec, graph, &bad, &res) == hipSuccess &&
                      res == hipGraphExecUpdateSuccess;
            if (!updated) {
                (void)hipGetLastError();
                (void)hipGraphExecDestroy(g->exec);
                g->exec = nullptr;
            }
        }
        hipError_t ei = hipSuccess;
        if (!updated) ei = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) {
            g->exec = nullptr;
            return fail(p, GKE_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
        }
        g->ptrs = ptrs;
        g->n = n;
        g->second = second;
        g->pending0 = pending0;
        g->acc0 = chunks0 > 0;
        g->pending1 = p->pending;
        g->dchunks = p->chunks_done - chunks0;
    }
    g->used = ++p->graph_clock;
    GKE_HIP(p, hipGraphLaunch(g->exec, p->stream));
    return GKE_OK;
}

gke_status gke_reconstruct(gke_plan_t p, const void *vhat, const void *ohat,
                           const double *mean_u, const double *mean_w, double *u, double *v,
                           double *w, double *pr)
{
    if (!p) return fail(nullptr, GKE_ERR_ARG, "plan is NULL");
    if (!vhat || !ohat || !mean_u || !mean_w || !u || !v || !w || !pr)
        return fail(p, GKE_ERR_ARG, "pointer is NULL");
    if (((uintptr_t)vhat | (uintptr_t)ohat) % 16)
        return fail(p, GKE_ERR_ARG, "vhat and ohat must be 16-byte aligned");
    if (!p->ws) return fail(p, GKE_ERR_STATE, "no workspace");
    if (!p->step1) return fail(p, GKE_ERR_STATE, "gke_reconstruct needs GKE_OPT_STEP1 = 1 "
                                                 "before the workspace");
    GKE_HIP(p, timed(p, GKE_K_STEP1, [&] {
        return gke::launch_step1(p->stream, p->d, p->tab, (const cx<double> *)vhat,
                                 (const cx<double> *)ohat, mean_u, mean_w, p->s1vel, p->s1prod,
                                 p->s1ph, p->s1u, p->s1b, u, v, w, pr);
    }));
    return GKE_OK;
}

gke_status gke_begin_stats(gke_plan_t p)
{
    if (!p) return fail(nullptr, GKE_ERR_ARG, "plan is NULL");
    if (!p->ws) return fail(p, GKE_ERR_STATE, "no workspace");
    if (p->second_scan) return fail(p, GKE_ERR_STATE, "second scan already started");
    if (p->n1 == 0) return fail(p, GKE_ERR_STATE, "no first-scan snapshot");
    GKE_HIP(p, timed(p, GKE_K_SMALL, [&] {
        return gke::launch_means(p->stream, p->d, p->tab, p->sums1, (double)p->n1, p->prof,
                                 p->d.prec == gke::PREC_BF16X3 ? p->gy1 : nullptr);
    }));
    GKE_HIP(p, hipStreamSynchronize(p->stream));
    p->second_scan = true;
    return GKE_OK;
}

gke_status gke_set_means(gke_plan_t p, const double *U, const double *V, const double *W,
                         const double *P)
{
    if (!p) return fail(nullptr, GKE_ERR_ARG, "plan is NULL");
    if (!U || !V || !W || !P) return fail(p, GKE_ERR_ARG, "mean pointer is NULL");
    if (!p->ws) return fail(p, GKE_ERR_STATE, "no workspace");
    if (p->second_scan) return fail(p, GKE_ERR_STATE, "second scan already started");
    const int ny = p->d.ny;
    const double *src[4] = {U, V, W, P};
    for (int f = 0; f < 4; ++f)
        GKE_HIP(p, hipMemcpyAsync(p->prof + f * ny, src[f], sizeof(double) * ny,
                                  hipMemcpyHostToDevice, p->stream));
    GKE_HIP(p, gke::launch_shear(p->stream, p->d, p->tab, p->prof));
    GKE_HIP(p, hipStreamSynchronize(p->stream));
    p->second_scan = true;
    p->means_from_host = true;
    return GKE_OK;
}

gke_status gke_finalize(gke_plan_t p, const gke_terms *out)
{
    if (!p) return fail(nullptr, GKE_ERR_ARG, "plan is NULL");
    if (!out) return fail(p, GKE_ERR_ARG, "out is NULL");
    if (!p->ws) return fail(p, GKE_ERR_STATE, "no workspace");
    if (!p->second_scan || p->n2 == 0) return fail(p, GKE_ERR_STATE, "no second-scan snapshot");
    if (!p->means_from_host && p->n1 != p->n2)
        return fail(p, GKE_ERR_STATE, "the two scans saw different snapshot counts");
    if (out->dtype != GKE_OUT_F64 && out->dtype != GKE_OUT_F32)
        return fail(p, GKE_ERR_ARG, "output dtype must be GKE_OUT_F64 or GKE_OUT_F32");
    const bool host = out->on_device == 0;
    if (host && p->host_stage == 0)
        return fail(p, GKE_ERR_STATE, "host outputs need GKE_OPT_HOST_STAGING before the workspace");
    if (!p->general && (out->t[GKE_T_PHIY_V] || out->t[GKE_T_PHI_V]) && !out->t[GKE_T_DU2])
        return fail(p, GKE_ERR_ARG, "the Y-derivative terms need the <du^2> output buffer");
    if (out->residual) {
        if (p->general)
            return fail(p, GKE_ERR_UNSUPPORTED, "the residual is written in the all-pairs mode only");
        if (!p->residual)
            return fail(p, GKE_ERR_STATE, "the residual needs GKE_OPT_RESIDUAL = 1 before the workspace");
        for (int k : {GKE_T_DU2, GKE_T_PHIY_T, GKE_T_PHIY_V, GKE_T_PHI_T, GKE_T_PHI_P, GKE_T_PHI_V,
                      GKE_T_XI_P1, GKE_T_XI_P2})
            if (!out->t[k])
                return fail(p, GKE_ERR_ARG, "the residual needs the maps T1, T5, T6, T9-T13");
    }
    gke_status s = launch_flush(p);
    if (s != GKE_OK) return s;
    const gke::Dims &d = p->d;
    hipStream_t st = p->stream;
    const int f32 = out->dtype == GKE_OUT_F32 ? 1 : 0;
    const size_t esz = f32 ? sizeof(float) : sizeof(double);
    // maps of this call: the pairs of the slab (general modes) or all pairs
    const size_t npairs = p->general ? p->slabs[p->cur_slab].opairs.size() : (size_t)d.ny * d.ny;
    const size_t map_bytes = esz * npairs * (size_t)d.nqo * d.npo, t14_bytes = esz * npairs;
    // device destinations: the caller's maps, or a staging buffer whose
    // previous copies to the host have finished
    void *dst[15];
    int b = 0;
    if (host) {
        b = p->stage_next;
        p->stage_next = (b + 1) % p->host_stage;
        if (p->stage_used[b]) GKE_HIP(p, hipStreamWaitEvent(st, p->ev_copied[b], 0));
        char *base = p->stage + b * p->stage_bytes;
        for (int i = 0; i < 15; ++i) {
            const void *want = i < 14 ? out->t[i] : out->residual;
            dst[i] = want ? base + i * p->stage_slot : nullptr;
        }
    } else {
        for (int i = 0; i < 14; ++i) dst[i] = out->t[i];
        dst[14] = out->residual;
    }
    void *resid = dst[14];
    const double inv = 1.0 / (double)p->n2;
    GKE_HIP(p, timed(p, GKE_K_SMALL, [&] {
        return p->general ? gke::launch_r0_band(st, d, p->band, inv, p->r0, p->gxz)
                          : gke::launch_r0(st, d, p->tab, p->acc, inv, p->r0, p->gxz);
    }));
    GKE_HIP(p, timed(p, GKE_K_SMALL, [&] {
        const int gy_mode = d.prec != gke::PREC_BF16X3 ? 0 : p->means_from_host ? 2 : 1;
        return gke::launch_profiles(st, d, p->tab, p->momp, p->r0, p->gxz, p->gy1, gy_mode,
                                    (double)p->n2, p->prof);
    }));
    const int pbt = (p->pair_batch > 0 && p->pair_batch < d.npair) ? p->pair_batch : d.npair;
    if (p->general) {
        // every transformed term of the slab's rows into the full-plane buffer,
        // then mirror average, domain, T6 / T11 / T14 into the maps
        static const int kslot[14] = {0, 1, 2, 3, 4, -1, 5, 6, 7, 8, -1, 9, 10, -1};
        void *mfp[14];
        for (int i = 0; i < 14; ++i) mfp[i] = kslot[i] >= 0 ? p->mf + kslot[i] * p->mstride : nullptr;
        for (int q0 = 0; q0 < d.npair; q0 += pbt) {
            const int q1 = std::min(d.npair, q0 + pbt);
            GKE_HIP(p, timed(p, GKE_K_FIN_KZ, [&] {
                return gke::launch_fin_kz(st, d, p->tab, p->acc, q0, q1, inv, p->mid);
            }));
            GKE_HIP(p, timed(p, GKE_K_FIN_KX, [&] {
                return gke::launch_fin_kx(st, d, p->tab, p->mid, q0, q1, p->prof, mfp, 0, 1,
                                          nullptr);
            }));
        }
        GKE_HIP(p, timed(p, GKE_K_FD, [&] {
            return gke::launch_slab_out(st, d, p->tab, p->mf, p->mstride, p->opairs, (int)npairs,
                                        p->prof, p->mirror, dst, f32);
        }));
    } else {
        for (int q0 = 0; q0 < d.npair; q0 += pbt) {
            const int q1 = std::min(d.npair, q0 + pbt);
            GKE_HIP(p, timed(p, GKE_K_FIN_KZ, [&] {
                return gke::launch_fin_kz(st, d, p->tab, p->acc, q0, q1, inv, p->mid);
            }));
            if (resid)
                GKE_HIP(p, timed(p, GKE_K_RESID, [&] {
                    return gke::launch_fin_kz_h(st, d, p->tab, p->acc, q0, q1, inv, p->prof,
                                                p->mid);
                }));
            GKE_HIP(p, timed(p, GKE_K_FIN_KX, [&] {
                return gke::launch_fin_kx(st, d, p->tab, p->mid, q0, q1, p->prof, dst, f32, 0,
                                          resid);
            }));
        }
        if (dst[GKE_T_PHIY_V] || dst[GKE_T_PHI_V])
            GKE_HIP(p, timed(p, GKE_K_FD, [&] {
                return gke::launch_fd_terms(st, d, p->tab, dst[GKE_T_DU2], dst[GKE_T_PHIY_V],
                                            dst[GKE_T_PHI_V], f32);
            }));
        if (resid)
            GKE_HIP(p, timed(p, GKE_K_RESID, [&] {
                return gke::launch_resid(st, d, p->tab, dst, f32, p->prof, resid);
            }));
        if (dst[GKE_T_XI_D])
            GKE_HIP(p, timed(p, GKE_K_SMALL, [&] {
                return gke::launch_t14(st, d, p->prof, dst[GKE_T_XI_D], f32);
            }));
    }
    if (host) {
        // the copies run on the library's stream once the maps are written;
        // the next finalize into this buffer waits for them
        GKE_HIP(p, hipEventRecord(p->ev_ready[b], st));
        GKE_HIP(p, hipStreamWaitEvent(p->copy_stream, p->ev_ready[b], 0));
        for (int i = 0; i < 15; ++i) {
            void *h = i < 14 ? out->t[i] : out->residual;
            if (!h) continue;
            GKE_HIP(p, hipMemcpyAsync(h, dst[i], i == GKE_T_XI_D ? t14_bytes : map_bytes,
                                      hipMemcpyDeviceToHost, p->copy_stream));
        }
        GKE_HIP(p, hipEventRecord(p->ev_copied[b], p->copy_stream));
        p->stage_used[b] = true;
    }
    if (p->slab_fn) {   // after the copies (host) or the kernels (device outputs)
        {
            gke_status s = notify_slab(p, host ? p->copy_stream : st);
            if (s != GKE_OK) return s;
        }
    }
    GKE_HIP(p, hipStreamSynchronize(st));
    return GKE_OK;
}

gke_status gke_set_slab_callback(gke_plan_t p, gke_slab_fn fn, void *user)
{
    if (!p) return fail(nullptr, GKE_ERR_ARG, "plan is NULL");
    p->slab_fn = fn;
    p->slab_user = fn ? user : nullptr;
    return GKE_OK;
}

gke_status gke_wait_outputs(gke_plan_t p)
{
    if (!p) return fail(nullptr, GKE_ERR_ARG, "plan is NULL");
    if (p->copy_stream) GKE_HIP(p, hipStreamSynchronize(p->copy_stream));
    return GKE_OK;
}

gke_status gke_slab_count(gke_plan_t p, int *count)
{
    if (!p || !count) return fail(p, GKE_ERR_ARG, "NULL argument");
    if (!p->ws) return fail(p, GKE_ERR_STATE, "no workspace");
    *count = p->general ? (int)p->slabs.size() : 1;
    return GKE_OK;
}

gke_status gke_slab_pairs(gke_plan_t p, int slab, int *count, int *pairs)
{
    if (!p || !count) return fail(p, GKE_ERR_ARG, "NULL argument");
    if (!p->ws) return fail(p, GKE_ERR_STATE, "no workspace");
    const int ns = p->general ? (int)p->slabs.size() : 1;
    if (slab < 0 || slab >= ns) return fail(p, GKE_ERR_ARG, "slab out of range");
    const int ny = p->d.ny;
    if (!p->general) {
        *count = ny * ny;
        if (pairs)
            for (int n = 0; n < ny * ny; ++n) {
                pairs[2 * n] = n / ny;
                pairs[2 * n + 1] = n % ny;
            }
        return GKE_OK;
    }
    const SlabTables &t = p->slabs[slab];
    *count = (int)t.opairs.size();
    if (pairs)
        for (size_t n = 0; n < t.opairs.size(); ++n) {
            pairs[2 * n] = t.opairs[n] & 0xffff;
            pairs[2 * n + 1] = t.opairs[n] >> 16;
        }
    return GKE_OK;
}

gke_status gke_begin_slab(gke_plan_t p, int slab)
{
    if (!p) return fail(nullptr, GKE_ERR_ARG, "plan is NULL");
    if (!p->ws) return fail(p, GKE_ERR_STATE, "no workspace");
    const int ns = p->general ? (int)p->slabs.size() : 1;
    if (slab < 0 || slab >= ns) return fail(p, GKE_ERR_ARG, "slab out of range");
    if (!p->second_scan) return fail(p, GKE_ERR_STATE, "the means are not known yet");
    // forget the second scan of the previous slab: moments restart, the
    // accumulators are overwritten by the first chunk
    GKE_HIP(p, gke::launch_zero(p->stream, p->momp, sizeof(double) * p->d.ny * gke::NMOMP * p->d.nzb));
    p->n2 = 0;
    p->pending = 0;
    p->chunks_done = 0;
    if (p->general) return select_slab(p, slab);
    GKE_HIP(p, hipStreamSynchronize(p->stream));
    return GKE_OK;
}

gke_status gke_state_size(gke_plan_t p, size_t *bytes)
{
    if (!p || !bytes) return fail(p, GKE_ERR_ARG, "NULL argument");
    if (!p->ws) return fail(p, GKE_ERR_STATE, "no workspace");
    *bytes = state_bytes(state_header(p));
    return GKE_OK;
}

gke_status gke_save_state(gke_plan_t p, void *host, size_t bytes)
{
    if (!p || !host) return fail(p, GKE_ERR_ARG, "NULL argument");
    if (!p->ws) return fail(p, GKE_ERR_STATE, "no workspace");
    {   // the snapshots of the current chunk go into the accumulators first
        gke_status s = launch_flush(p);
        if (s != GKE_OK) return s;
    }
    const StateHeader h = state_header(p);
    if (bytes < state_bytes(h))
        return fail(p, GKE_ERR_ARG, "state buffer too small: need " +
                                        std::to_string(state_bytes(h)) + " bytes");
    char *o = static_cast<char *>(host);
    std::memcpy(o, &h, sizeof(h));
    o += sizeof(h);
    hipStream_t st = p->stream;
    GKE_HIP(p, hipMemcpyAsync(o, p->sums1, h.small_bytes, hipMemcpyDeviceToHost, st));
    o += h.small_bytes;
    if (h.acc_bytes)
        GKE_HIP(p, hipMemcpyAsync(o, p->acc, h.acc_bytes, hipMemcpyDeviceToHost, st));
    o += h.acc_bytes;
    if (h.band_bytes)
        GKE_HIP(p, hipMemcpyAsync(o, p->band, h.band_bytes, hipMemcpyDeviceToHost, st));
    GKE_HIP(p, hipStreamSynchronize(st));
    return GKE_OK;
}

gke_status gke_load_state(gke_plan_t p, const void *host, size_t bytes)
{
    if (!p || !host) return fail(p, GKE_ERR_ARG, "NULL argument");
    if (!p->ws) return fail(p, GKE_ERR_STATE, "no workspace");
    if (bytes < sizeof(StateHeader)) return fail(p, GKE_ERR_ARG, "state buffer too small");
    StateHeader h;
    std::memcpy(&h, host, sizeof(h));
    if (std::memcmp(h.magic, kStateMagic, 8) != 0)
        return fail(p, GKE_ERR_ARG, "not a saved state of this library");
    if (p->general && (h.cur_slab < 0 || h.cur_slab >= (int)p->slabs.size()))
        return fail(p, GKE_ERR_ARG, "saved slab out of range for this plan");
    // the slab decides the pair extents of the accumulators
    if (p->general && p->cur_slab != h.cur_slab) {
        gke_status s = select_slab(p, h.cur_slab);
        if (s != GKE_OK) return s;
    }
    StateHeader mine = state_header(p);
    mine.cur_slab = h.cur_slab;
    if (h.nx != mine.nx || h.ny != mine.ny || h.nz != mine.nz || h.prec != mine.prec ||
        h.dtype != mine.dtype || h.mirror != mine.mirror || h.domain != mine.domain ||
        h.slab_rows != mine.slab_rows || h.cfg != mine.cfg ||
        h.small_bytes != mine.small_bytes || h.acc_bytes != mine.acc_bytes ||
        h.band_bytes != mine.band_bytes)
        return fail(p, GKE_ERR_ARG, "the saved state belongs to a plan of another shape or "
                                    "options");
    if (bytes < state_bytes(h)) return fail(p, GKE_ERR_ARG, "state buffer truncated");
    const char *o = static_cast<const char *>(host) + sizeof(h);
    hipStream_t st = p->stream;
    GKE_HIP(p, hipMemcpyAsync(p->sums1, o, h.small_bytes, hipMemcpyHostToDevice, st));
    o += h.small_bytes;
    if (h.acc_bytes)
        GKE_HIP(p, hipMemcpyAsync(p->acc, o, h.acc_bytes, hipMemcpyHostToDevice, st));
    o += h.acc_bytes;
    if (h.band_bytes)
        GKE_HIP(p, hipMemcpyAsync(p->band, o, h.band_bytes, hipMemcpyHostToDevice, st));
    GKE_HIP(p, hipStreamSynchronize(st));
    p->n1 = h.n1;
    p->n2 = h.n2;
    p->chunks_done = h.chunks_done;
    p->pending = 0;
    p->second_scan = h.second_scan != 0;
    p->means_from_host = h.means_from_host != 0;
    return GKE_OK;
}

gke_status gke_get_profiles(gke_plan_t p, double *out)
{
    if (!p || !out) return fail(p, GKE_ERR_ARG, "NULL argument");
    if (!p->ws) return fail(p, GKE_ERR_STATE, "no workspace");
    GKE_HIP(p, hipStreamSynchronize(p->stream));
    GKE_HIP(p, hipMemcpy(out, p->prof, sizeof(double) * gke::NPROF * p->d.ny, hipMemcpyDeviceToHost));
    return GKE_OK;
}

gke_status gke_reset(gke_plan_t p)
{
    if (!p) return fail(nullptr, GKE_ERR_ARG, "plan is NULL");
    if (!p->ws) return fail(p, GKE_ERR_STATE, "no workspace");
    // sums, profiles and moment partials are contiguous in the workspace;
    // the cross-spectral accumulators are overwritten by the first chunk
    GKE_HIP(p, gke::launch_zero(p->stream, p->sums1, (char *)p->inter - (char *)p->sums1));
    p->n1 = p->n2 = 0;
    p->pending = 0;
    p->chunks_done = 0;
    p->second_scan = false;
    p->means_from_host = false;
    if (p->general && p->cur_slab != 0) return select_slab(p, 0);
    return GKE_OK;
}

gke_status gke_timings(gke_plan_t p, double *total_ms, int64_t *launches, int reset)
{
    if (!p) return fail(nullptr, GKE_ERR_ARG, "plan is NULL");
    GKE_HIP(p, hipStreamSynchronize(p->stream));
    GKE_HIP(p, collect_timings(p));
    for (int k = 0; k < GKE_NKERNELS; ++k) {
        if (total_ms) total_ms[k] = p->t_ms[k];
        if (launches) launches[k] = p->t_n[k];
        if (reset) {
            p->t_ms[k] = 0.0;
            p->t_n[k] = 0;
        }
    }
    return GKE_OK;
}

void gke_destroy(gke_plan_t p)
{
    if (!p) return;
    if (p->ws) (void)hipStreamSynchronize(p->stream);
    for (auto &e : p->graphs)
        if (e.exec) (void)hipGraphExecDestroy(e.exec);
    if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
    if (p->copy_stream) {
        (void)hipStreamSynchronize(p->copy_stream);
        for (int b = 0; b < 2; ++b) {
            (void)hipEventDestroy(p->ev_ready[b]);
            (void)hipEventDestroy(p->ev_copied[b]);
        }
        (void)hipStreamDestroy(p->copy_stream);
    }
    for (hipEvent_t e : p->ev_pool) (void)hipEventDestroy(e);
    delete p;
}

const char *gke_last_error(gke_plan_t p)
{
    return p ? p->err.c_str() : g_plan_error.c_str();
}

const char *gke_version(void) { return "gke-mi355x 0.1 (gfx950)"; }

}  // extern "C"
