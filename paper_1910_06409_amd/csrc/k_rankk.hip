// k_rankk.hip -- cross-spectral accumulation over snapshots, FP64.
//
// Every GKE term is a linear combination of two-point correlations
// (Section "Products instead of correlations", eq. expansion and its analogues
// for the triple terms), and every correlation is the inverse transform of a
// cross-spectrum conj(A^(k;Y1)) B^(k;Y2) averaged over snapshots (Parseval).
// Averaging commutes with the inverse transform, so the spectra are summed
// over snapshots first and transformed once at the end (the same linearity the
// paper uses to defer derivatives, Section "General structure of the program").
//
// Per wavenumber k this is a complex rank-K update over the snapshots with the
// wall-normal planes as rows and columns.  The spectra hold the fluctuations
// and Q_ij = 2 u'_i u'_j + delta_ij q (q = u'_i u'_i = (Q_xx + Q_yy + Q_zz)/5);
// the eight term spectra needed per ordered pair (Y1, Y2) are built from nine
// accumulators c0..c8 of products conj(L(Y1)) R(Y2) (27 complex products per
// pair and snapshot):
//   c0 = sum_i (u_i, u_i)                          -> R^      (scale energy)
//   c1 = sum_i (Q_ix, u_i) - (u_i, Q_ix)           -> <du^2 du>  spectrum
//   c2 = sum_i (Q_iz, u_i) - (u_i, Q_iz)           -> <du^2 dw>  spectrum
//   c3 = sum_i (Q_iy, u_i),  c4 = sum_i (u_i, Q_iy)
//   c5 = (v, q) + (q, v),    c6 = (p, v) + (v, p)
//   c7 = (u, v),             c8 = (v, u)
//   <du^2 dv>: c3 - c4;  <v* du^2>: 2 c5 - c3 - c4;  <dp dv>: c6;
//   <du dv>: c7 + c8;    <du v*>: c8 - c7     (r-dependent parts)
// Only unordered pairs are computed; the reverse orientation follows from the
// r-inversion symmetry (Section "Exploiting symmetries") at finalize.
//
// The planes split into full 16-plane tiles, handled on the matrix cores by
// tile pairs, and the remaining Ny mod 16 planes, whose pairs go to a small
// FP64 vector kernel.  A tile pair (a, b) takes its 16 rows (planes Y1) from
// the row-plane table at 16 a .. 16 a + 15 and its 16 columns (planes Y2) from
// 16 b .. 16 b + 15: for all pairs the row table is the identity and a <= b;
// for a subset of rows (a slab of Y1 planes) it lists those planes.
// Accumulators are indexed by a compact pair index P: tile pair tp covers
// P = 256 tp + 16 (row offset) + (column offset), the remainder pairs follow in
// the order of the host-built pair table.
//
// MFMA mapping (v_mfma_f64_16x16x4f64, K = four snapshots s0 .. s0+3):
//   A (lane l): L[Y1 = row plane 16a + l%16][s0 + l/16],
//   B (lane l): R[Y2 = 16b + l%16][s0 + l/16],
//   D (lane l, register v): element (row l/16 + 4v, Y2 = 16b + l%16)
//   (checked on the device: the f64 form strides the rows by 4 across registers).
// Each complex product conj(L) R = (Lr - i Li)(Rr + i Ri) takes three real
// products (the three-multiplication form of a complex product):
//   K1 = (Lr - Li) Rr,  K2 = Lr (Ri - Rr),  K3 = -Li (Rr + Ri),
//   Re = K1 - K3,  Im = K1 + K2,
// so 27 complex products cost 81 MFMAs per four snapshots instead of 108.
// The three real accumulators per complex accumulator do not fit one wave, so
// a tile pair takes three waves, each with three complex accumulators and
// loading only the fields they need: wave 0 holds c3 c4 c5 (8 products),
// wave 1 c1 c7 c8 (8 products), wave 2 c0 c2 c6 (11 products); every term
// spectrum is formed from one wave's accumulators.
#include "rankk_common.h"

namespace gke {

typedef double d4 __attribute__((ext_vector_type(4)));

// Loads of four snapshots (one per lane group) of the fields a wave uses.
// Addresses split into a wave-uniform part (wavenumber, field, snapshot group:
// scalar registers) and a 32-bit lane offset (plane, snapshot within the
// group).  Branch-free: a snapshot past the end reloads the last valid one and
// its left operand is zeroed (a zero left value cancels every product of that
// snapshot), so the loads stay in flight.
struct Loader {
    const char *kb;
    size_t fbytes;
    unsigned loff, roff, sbytes;
    __device__ __forceinline__ cx<double> get(int f, unsigned off, int s0, unsigned so) const
    {
        // the 32-bit lane offset is formed first, so that the load takes the
        // uniform base from scalar registers
        const char *base = kb + (size_t)s0 * sbytes + f * fbytes;
        return *reinterpret_cast<const cx<double> *>(base + (off + so));
    }
};

// acc[3c + 0..2] += K1, K2, K3 of sg conj(l) r  (sg = -1 when neg, folded into
// A); the right-hand forms Rr, Ri - Rr, Rr + Ri are formed here, so that only
// the complex values stay live between products
__device__ __forceinline__ void mac3(d4 *acc, int c, cx<double> l, cx<double> r, bool neg)
{
    const double a1 = neg ? l.y - l.x : l.x - l.y;
    const double a2 = neg ? -l.x : l.x;
    const double a3 = neg ? l.y : -l.y;
    acc[3 * c + 0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, r.x, acc[3 * c + 0], 0, 0, 0);
    acc[3 * c + 1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a2, r.y - r.x, acc[3 * c + 1], 0, 0, 0);
    acc[3 * c + 2] = __builtin_amdgcn_mfma_f64_16x16x4f64(a3, r.x + r.y, acc[3 * c + 2], 0, 0, 0);
}

// fields of each wave, left and right
constexpr int W0F[8] = {F_U, F_V, F_W, F_QXX, F_QYY, F_QZZ, F_QXY, F_QYZ};   // c3 c4 c5
constexpr int W1F[6] = {F_U, F_V, F_W, F_QXX, F_QXY, F_QXZ};                 // c1 c7 c8
constexpr int W2F[7] = {F_U, F_V, F_W, F_P, F_QXZ, F_QYZ, F_QZZ};            // c0 c2 c6

template <int N>
__device__ __forceinline__ void load_fields(cx<double> *L, cx<double> *R, const int (&fl)[N],
                                            const Loader &ld, int s0, unsigned so, bool ok)
{
#pragma unroll
    for (int i = 0; i < N; ++i) {
        L[i] = ld.get(fl[i], ld.loff, s0, so);
        R[i] = ld.get(fl[i], ld.roff, s0, so);
    }
    if (!ok) {
#pragma unroll
        for (int i = 0; i < N; ++i) L[i] = cx<double>{0.0, 0.0};
    }
}

// wave 0: acc slots 0 1 2 = c3 c4 c5; L, R in W0F order
__device__ __forceinline__ void step_w0(d4 *acc, const cx<double> *L, const cx<double> *R)
{
    enum { u, v, w, xx, yy, zz, xy, yz };
    const cx<double> lq = cx<double>{0.2 * (L[xx].x + L[yy].x + L[zz].x),
                                     0.2 * (L[xx].y + L[yy].y + L[zz].y)};
    const cx<double> rq = cx<double>{0.2 * (R[xx].x + R[yy].x + R[zz].x),
                                     0.2 * (R[xx].y + R[yy].y + R[zz].y)};
    mac3(acc, 0, L[xy], R[u], false);   // c3
    mac3(acc, 1, L[u], R[xy], false);   // c4
    mac3(acc, 2, lq, R[v], false);      // c5
    mac3(acc, 0, L[yy], R[v], false);   // c3
    mac3(acc, 1, L[v], R[yy], false);   // c4
    mac3(acc, 2, L[v], rq, false);      // c5
    mac3(acc, 0, L[yz], R[w], false);   // c3
    mac3(acc, 1, L[w], R[yz], false);   // c4
}

// wave 1: acc slots 0 1 2 = c1 c7 c8; L, R in W1F order
__device__ __forceinline__ void step_w1(d4 *acc, const cx<double> *L, const cx<double> *R)
{
    enum { u, v, w, xx, xy, xz };
    mac3(acc, 0, L[xx], R[u], false);
    mac3(acc, 1, L[u], R[v], false);    // c7
    mac3(acc, 2, L[v], R[u], false);    // c8
    mac3(acc, 0, L[xy], R[v], false);
    mac3(acc, 0, L[xz], R[w], false);
    mac3(acc, 0, L[u], R[xx], true);
    mac3(acc, 0, L[v], R[xy], true);
    mac3(acc, 0, L[w], R[xz], true);
}

// wave 2: acc slots 0 1 2 = c0 c2 c6; L, R in W2F order
__device__ __forceinline__ void step_w2(d4 *acc, const cx<double> *L, const cx<double> *R)
{
    enum { u, v, w, p, xz, yz, zz };
    mac3(acc, 0, L[u], R[u], false);    // c0
    mac3(acc, 1, L[xz], R[u], false);   // c2
    mac3(acc, 2, L[p], R[v], false);    // c6
    mac3(acc, 0, L[v], R[v], false);
    mac3(acc, 1, L[yz], R[v], false);
    mac3(acc, 2, L[v], R[p], false);
    mac3(acc, 0, L[w], R[w], false);
    mac3(acc, 1, L[zz], R[w], false);
    mac3(acc, 1, L[u], R[xz], true);
    mac3(acc, 1, L[v], R[yz], true);
    mac3(acc, 1, L[w], R[zz], true);
}

// register prefetch depth in groups of four snapshots (0: none)
#ifndef GKE_RANKK_PF
#define GKE_RANKK_PF 0
#endif

// ZERO: zero the left operand of a snapshot past the end at once (false when
// the loads are a prefetch: the caller zeroes at use, so that no register of a
// load in flight is written)
template <int W, int N, bool ZERO = true>
__device__ __forceinline__ void load_kind(cx<double> *L, cx<double> *R, const Loader &ld, int s0,
                                          int kq, int nsnap)
{
    const bool ok = s0 + kq < nsnap;
    const unsigned so = (unsigned)((ok ? kq : nsnap - 1 - s0)) * ld.sbytes;
    if (W == 0) load_fields(L, R, W0F, ld, s0, so, ok || !ZERO);
    else if (W == 1) load_fields(L, R, W1F, ld, s0, so, ok || !ZERO);
    else load_fields(L, R, W2F, ld, s0, so, ok || !ZERO);
}

template <int W>
__device__ __forceinline__ void step_kind(d4 *ac, const cx<double> *L, const cx<double> *R)
{
    if (W == 0) step_w0(ac, L, R);
    else if (W == 1) step_w1(ac, L, R);
    else step_w2(ac, L, R);
}

// all snapshots, four at a time, for wave kind W
template <int W>
__device__ __forceinline__ void snapshot_loop(d4 *ac, const Loader &ld, int nsnap, int kq)
{
    constexpr int N = W == 0 ? 8 : W == 1 ? 6 : 7;
#if GKE_RANKK_PF
    constexpr int PF = GKE_RANKK_PF;   // groups of four snapshots loaded ahead
    cx<double> Lp[PF][N], Rp[PF][N];
#pragma unroll
    for (int q = 0; q < PF; ++q)
        load_kind<W, N, false>(Lp[q], Rp[q], ld, 4 * q < nsnap ? 4 * q : 0, kq, nsnap);
    for (int s0 = 0; s0 < nsnap; s0 += 4) {
        cx<double> L[N], R[N];
#pragma unroll
        for (int i = 0; i < N; ++i) {
            L[i] = Lp[0][i];
            R[i] = Rp[0][i];
        }
#pragma unroll
        for (int q = 0; q + 1 < PF; ++q)
#pragma unroll
            for (int i = 0; i < N; ++i) {
                Lp[q][i] = Lp[q + 1][i];
                Rp[q][i] = Rp[q + 1][i];
            }
        const int sn = s0 + 4 * PF;
        load_kind<W, N, false>(Lp[PF - 1], Rp[PF - 1], ld, sn < nsnap ? sn : s0, kq, nsnap);
        __builtin_amdgcn_sched_barrier(0);
        if (s0 + kq >= nsnap) {   // past the end: a zero left operand
#pragma unroll
            for (int i = 0; i < N; ++i) L[i] = cx<double>{0.0, 0.0};
        }
        step_kind<W>(ac, L, R);
        __builtin_amdgcn_sched_barrier(0);
    }
#else
    for (int s0 = 0; s0 < nsnap; s0 += 4) {
        cx<double> L[N], R[N];
        load_kind<W, N>(L, R, ld, s0, kq, nsnap);
        step_kind<W>(ac, L, R);
    }
#endif
}

// minimum waves per SIMD (register budget)
#ifndef GKE_RANKK_MINW
#define GKE_RANKK_MINW 3
#endif

// acc layout: [NSPEC][nk][P] complex.  One block (three waves) per (k, tile pair).
__global__ __launch_bounds__(192, GKE_RANKK_MINW) void k_rankk_f64(
    const cx<double> *__restrict__ spec, Dims d, const int *__restrict__ tile_a,
    const int *__restrict__ tile_b, const int *__restrict__ t_rowplane, int nsnap,
    int accumulate, int total, cx<double> *__restrict__ acc)
{
    // XCD-aware order: workgroup i runs on XCD i % 8; give every XCD a
    // contiguous range of (k, tile pair) so the tiles of one wavenumber share
    // that XCD's L2.
    const int G = gridDim.x;
    const int bid = blockIdx.x;
    const int L = (bid & 7) * (G >> 3) + (bid >> 3);
    if (L >= total) return;
    const int k = L / d.ntp;
    const int tp = L - k * d.ntp;
    const int ta = tile_a[tp], tb = tile_b[tp];

    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int row = lane & 15, kq = lane >> 4;
    const size_t fstride = (size_t)d.chunk * d.nys;  // complex elements per field
    Loader ld;
    ld.kb = reinterpret_cast<const char *>(spec + (size_t)k * NFIELD * fstride);
    ld.fbytes = fstride * sizeof(cx<double>);
    ld.sbytes = (unsigned)d.nys * sizeof(cx<double>);
    ld.loff = (unsigned)t_rowplane[ta * 16 + row] * sizeof(cx<double>);
    ld.roff = (unsigned)(tb * 16 + row) * sizeof(cx<double>);

    d4 ac[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) ac[c] = d4{0.0, 0.0, 0.0, 0.0};

    // one loop per wave kind, so that each keeps only its own loop invariants
    if (wv == 0) snapshot_loop<0>(ac, ld, nsnap, kq);
    else if (wv == 1) snapshot_loop<1>(ac, ld, nsnap, kq);
    else snapshot_loop<2>(ac, ld, nsnap, kq);

    const size_t sp_stride = (size_t)d.nk * d.pstr;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const size_t o = (size_t)k * d.pstr + (size_t)tp * 256 + (kq + 4 * v) * 16 + row;
        // Re = K1 - K3, Im = K1 + K2 of each accumulator of this wave
        double cr[9], ci[9];
#pragma unroll
        for (int c = 0; c < 9; ++c) cr[c] = ci[c] = 0.0;
        auto put = [&](int slot, int c) {
            cr[c] = ac[3 * slot][v] - ac[3 * slot + 2][v];
            ci[c] = ac[3 * slot][v] + ac[3 * slot + 1][v];
        };
        if (wv == 0) {
            put(0, 3);
            put(1, 4);
            put(2, 5);
        } else if (wv == 1) {
            put(0, 1);
            put(1, 7);
            put(2, 8);
        } else {
            put(0, 0);
            put(1, 2);
            put(2, 6);
        }
        store_spectra_part(acc, sp_stride, o, cr, ci, accumulate, wv);
    }
}

hipError_t launch_rankk_f64(hipStream_t st, const Dims &d, const Tables &t,
                            const cx<double> *spec, int nsnap, int accumulate,
                            cx<double> *acc)
{
    if (d.ntp > 0) {
        const long long total = (long long)d.nk * d.ntp;
        if (total >= (1LL << 31) - 8) return hipErrorInvalidValue;
        const int G = (int)((total + 7) / 8 * 8);
        hipLaunchKernelGGL(k_rankk_f64, dim3(G), dim3(192), 0, st, spec, d, t.tile_a, t.tile_b,
                           t.rowplane, nsnap, accumulate, (int)total, acc);
    }
    return hipGetLastError();
}

hipError_t launch_rankk_rem_f64(hipStream_t st, const Dims &d, const Tables &t,
                                const cx<double> *spec, int nsnap, int accumulate,
                                cx<double> *acc)
{
    return launch_rankk_rem(st, d, t, spec, nsnap, accumulate, acc);
}

}  // namespace gke
