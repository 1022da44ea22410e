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
// MFMA mapping (v_mfma_f64_16x16x4f64, one wave per 16x16 output tile):
//   K index = (snapshot pair s0, s0+1) x (real, imaginary part);
//   A (lane l): Re/Im of L[Y1 = row plane 16a + l%16][s0 + (l/16)/2], picked by (l/16)%2;
//   B (lane l): for the real output (Rr, Ri), for the imaginary output
//               (Ri, -Rr) of R[Y2 = 16b + l%16][s0 + (l/16)/2];
//   so sum_k A B = Re/Im of conj(L) R.
//   D (lane l, register v): element (row l/16 + 4v, Y2 = 16b + l%16)
//   (checked on the device: the f64 form strides the rows by 4 across registers).
#include "rankk_common.h"

namespace gke {

typedef double d4 __attribute__((ext_vector_type(4)));

#define GKE_MFMA2(c, a, br, bi)                                                   \
    do {                                                                         \
        ar[c] = __builtin_amdgcn_mfma_f64_16x16x4f64((a), (br), ar[c], 0, 0, 0); \
        ai[c] = __builtin_amdgcn_mfma_f64_16x16x4f64((a), (bi), ai[c], 0, 0, 0); \
    } while (0)

struct Operands {
    double L[NFIELD];
    cx<double> R[NFIELD];
};

// Loads of one snapshot pair.  Addresses split into a wave-uniform part
// (wavenumber, field, snapshot pair: scalar registers) and a 32-bit lane
// offset (plane, snapshot within the pair, real/imaginary part).
// Branch-free: a pair past the end reloads the last valid snapshot; the caller
// zeroes the left operand of such a slot when it uses it (a zero left value
// cancels every product of that snapshot), so the loads stay in flight.
__device__ __forceinline__ void load_operands(Operands &op, const char *kb, size_t fbytes,
                                              unsigned loff, unsigned roff, unsigned sbytes,
                                              int s0, int soff, int nsnap)
{
    const int s = s0 + soff < nsnap ? s0 + soff : nsnap - 1;
    const unsigned so = (unsigned)(s - s0) * sbytes;
    const char *base = kb + (size_t)s0 * sbytes;
#pragma unroll
    for (int f = 0; f < NFIELD; ++f) {
        const char *bf = base + f * fbytes;
        const unsigned lo = loff + so, ro = roff + so;
        op.L[f] = *reinterpret_cast<const double *>(bf + lo);
        op.R[f] = *reinterpret_cast<const cx<double> *>(bf + ro);
    }
}

// The products of one snapshot pair into the nine accumulators.
__device__ __forceinline__ void rankk_f64_step(d4 *ar, d4 *ai, const Operands &cur, bool ok,
                                               int ri)
{
    // left operand (planes Y1): fluctuations and Q_ij; zero past the end
    double Lc[NFIELD];
#pragma unroll
    for (int f = 0; f < NFIELD; ++f) Lc[f] = ok ? cur.L[f] : 0.0;
    const double lu = Lc[F_U], lv = Lc[F_V], lw = Lc[F_W], lp = Lc[F_P];
    const double lQxx = Lc[F_QXX], lQyy = Lc[F_QYY], lQzz = Lc[F_QZZ];
    const double lQxy = Lc[F_QXY], lQxz = Lc[F_QXZ], lQyz = Lc[F_QYZ];
    const double lq = 0.2 * (lQxx + lQyy + lQzz);
    const double nu_ = -lu, nv = -lv, nw = -lw;
    // right operand (planes Y2): real-output and imaginary-output forms
    double br[NFIELD], bi[NFIELD];
#pragma unroll
    for (int f = 0; f < NFIELD; ++f) {
        br[f] = ri ? cur.R[f].y : cur.R[f].x;
        bi[f] = ri ? -cur.R[f].x : cur.R[f].y;
    }
    const double rQxxr = br[F_QXX], rQxxi = bi[F_QXX];
    const double rQyyr = br[F_QYY], rQyyi = bi[F_QYY];
    const double rQzzr = br[F_QZZ], rQzzi = bi[F_QZZ];
    const double rQxyr = br[F_QXY], rQxyi = bi[F_QXY];
    const double rQxzr = br[F_QXZ], rQxzi = bi[F_QXZ];
    const double rQyzr = br[F_QYZ], rQyzi = bi[F_QYZ];
    const double rqr = 0.2 * (rQxxr + rQyyr + rQzzr);
    const double rqi = 0.2 * (rQxxi + rQyyi + rQzzi);
    const double ur = br[F_U], ui = bi[F_U], vr = br[F_V], vi = bi[F_V];
    const double wr = br[F_W], wi = bi[F_W], pr = br[F_P], pi = bi[F_P];

    // 27 products, ordered so that successive ones feed different accumulators
    GKE_MFMA2(0, lu, ur, ui);
    GKE_MFMA2(1, lQxx, ur, ui);
    GKE_MFMA2(2, lQxz, ur, ui);
    GKE_MFMA2(3, lQxy, ur, ui);
    GKE_MFMA2(8, lv, ur, ui);
    GKE_MFMA2(4, lu, rQxyr, rQxyi);
    GKE_MFMA2(1, nu_, rQxxr, rQxxi);
    GKE_MFMA2(2, nu_, rQxzr, rQxzi);
    GKE_MFMA2(5, lv, rqr, rqi);
    GKE_MFMA2(0, lv, vr, vi);
    GKE_MFMA2(1, lQxy, vr, vi);
    GKE_MFMA2(2, lQyz, vr, vi);
    GKE_MFMA2(3, lQyy, vr, vi);
    GKE_MFMA2(6, lp, vr, vi);
    GKE_MFMA2(7, lu, vr, vi);
    GKE_MFMA2(4, lv, rQyyr, rQyyi);
    GKE_MFMA2(5, lq, vr, vi);
    GKE_MFMA2(1, nv, rQxyr, rQxyi);
    GKE_MFMA2(2, nv, rQyzr, rQyzi);
    GKE_MFMA2(6, lv, pr, pi);
    GKE_MFMA2(0, lw, wr, wi);
    GKE_MFMA2(1, lQxz, wr, wi);
    GKE_MFMA2(2, lQzz, wr, wi);
    GKE_MFMA2(3, lQyz, wr, wi);
    GKE_MFMA2(4, lw, rQyzr, rQyzi);
    GKE_MFMA2(1, nw, rQxzr, rQxzi);
    GKE_MFMA2(2, nw, rQzzr, rQzzi);
}

// Register prefetch of the next snapshot pair (1) or none (0), and the
// minimum waves per SIMD.  Without the prefetch the kernel fits 2 waves per
// SIMD (220 VGPRs), and each wave's MFMA chain covers the other's loads; this
// measured about 1.35x faster than one wave with a prefetch.
#ifndef GKE_RANKK_PF
#define GKE_RANKK_PF 0
#endif
#ifndef GKE_RANKK_MINW
#define GKE_RANKK_MINW 2
#endif

// acc layout: [NSPEC][nk][P] complex.
__global__ __launch_bounds__(64, GKE_RANKK_MINW) void k_rankk_f64(
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

    const int lane = threadIdx.x;
    const int row = lane & 15, kq = lane >> 4, soff = kq >> 1, ri = kq & 1;
    const size_t fstride = (size_t)d.chunk * d.ny;  // complex elements per field
    const char *kb = reinterpret_cast<const char *>(spec + (size_t)k * NFIELD * fstride);
    const size_t fbytes = fstride * sizeof(cx<double>);
    const unsigned sbytes = (unsigned)d.ny * sizeof(cx<double>);
    const unsigned loff =
        (unsigned)t_rowplane[ta * 16 + row] * sizeof(cx<double>) + ri * sizeof(double);
    const unsigned roff = (unsigned)(tb * 16 + row) * sizeof(cx<double>);

    d4 ar[9], ai[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) {
        ar[c] = d4{0.0, 0.0, 0.0, 0.0};
        ai[c] = d4{0.0, 0.0, 0.0, 0.0};
    }

#if GKE_RANKK_PF
    Operands cur;
    load_operands(cur, kb, fbytes, loff, roff, sbytes, 0, soff, nsnap);
    for (int s0 = 0; s0 < nsnap; s0 += 2) {
        // prefetch the next snapshot pair while this one is multiplied
        Operands nxt;
        load_operands(nxt, kb, fbytes, loff, roff, sbytes, s0 + 2 < nsnap ? s0 + 2 : s0, soff,
                      nsnap);
        // keep the scheduler from pulling the consumers of these loads into
        // this iteration: they are waited for only at the next one
        __builtin_amdgcn_sched_barrier(0);
        rankk_f64_step(ar, ai, cur, s0 + soff < nsnap, ri);
        __builtin_amdgcn_sched_barrier(0);
        cur = nxt;
    }
#else
    for (int s0 = 0; s0 < nsnap; s0 += 2) {
        Operands cur;
        load_operands(cur, kb, fbytes, loff, roff, sbytes, s0, soff, nsnap);
        rankk_f64_step(ar, ai, cur, s0 + soff < nsnap, ri);
    }
#endif

    const size_t sp_stride = (size_t)d.nk * d.pstr;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const size_t o = (size_t)k * d.pstr + (size_t)tp * 256 + (kq + 4 * v) * 16 + row;
        double cr[9], ci[9];
#pragma unroll
        for (int c = 0; c < 9; ++c) {
            cr[c] = ar[c][v];
            ci[c] = ai[c][v];
        }
        store_spectra(acc, sp_stride, o, cr, ci, accumulate);
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
        hipLaunchKernelGGL(k_rankk_f64, dim3(G), dim3(64), 0, st, spec, d, t.tile_a, t.tile_b,
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
