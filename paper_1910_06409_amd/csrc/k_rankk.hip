// k_rankk.hip -- cross-spectral accumulation over snapshots, FP64 MFMA.
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
// wall-normal planes as rows and columns.  With q = u'_i u'_i and
// Q_ij = 2 u'_i u'_j + delta_ij q, the eight term spectra needed per ordered
// pair (Y1, Y2) are built from nine accumulators c0..c8 of products
// conj(L(Y1)) R(Y2) (27 complex products per pair and snapshot):
//   c0 = sum_i (u_i, u_i)                          -> R^      (scale energy)
//   c1 = sum_i (Q_ix, u_i) - (u_i, Q_ix)           -> <du^2 du>  spectrum
//   c2 = sum_i (Q_iz, u_i) - (u_i, Q_iz)           -> <du^2 dw>  spectrum
//   c3 = sum_i (Q_iy, u_i),  c4 = sum_i (u_i, Q_iy)
//   c5 = (v, q) + (q, v),    c6 = (p, v) + (v, p)
//   c7 = (u, v),             c8 = (v, u)
//   <du^2 dv>: c3 - c4;  <v* du^2>: 2 c5 - c3 - c4;  <dp dv>: c6;
//   <du dv>: c7 + c8;    <du v*>: c8 - c7     (r-dependent parts)
// Only tile pairs (a <= b) of 16x16 planes are computed; the pairs below the
// diagonal follow from the r-inversion symmetry (Section "Exploiting
// symmetries") at finalize.
//
// MFMA mapping (v_mfma_f64_16x16x4f64, one wave per 16x16 output tile):
//   K index = (snapshot pair s0, s0+1) x (real, imaginary part);
//   A (lane l): Re/Im of L[Y1 = 16a + l%16][s0 + (l/16)/2], picked by (l/16)%2;
//   B (lane l): for the real output (Rr, Ri), for the imaginary output
//               (Ri, -Rr) of R[Y2 = 16b + l%16][s0 + (l/16)/2];
//   so sum_k A B = Re/Im of conj(L) R.
//   D (lane l, register v): element (Y1 = 16a + l/16 + 4v, Y2 = 16b + l%16)
//   (checked on the device: the f64 form strides the rows by 4 across registers).
#include "gke_internal.h"

namespace gke {

typedef double d4 __attribute__((ext_vector_type(4)));

#define GKE_MFMA2(acc_r, acc_i, a, br, bi)                                       \
    do {                                                                         \
        acc_r = __builtin_amdgcn_mfma_f64_16x16x4f64((a), (br), acc_r, 0, 0, 0); \
        acc_i = __builtin_amdgcn_mfma_f64_16x16x4f64((a), (bi), acc_i, 0, 0, 0); \
    } while (0)

// acc layout: [NSPEC][nk][ntp * 256] complex, element index within a tile
// pair = (Y1 offset) * 16 + (Y2 offset).
__global__ __launch_bounds__(64) void k_rankk_f64(const cx<double> *__restrict__ spec, Dims d,
                                                  const int *__restrict__ tile_a,
                                                  const int *__restrict__ tile_b, int nsnap,
                                                  int accumulate, int total,
                                                  cx<double> *__restrict__ acc)
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
    const size_t fstride = (size_t)d.chunk * d.nyp;  // complex elements per field
    const cx<double> *kb = spec + (size_t)k * NFIELD * fstride;
    const double *lbase = reinterpret_cast<const double *>(kb + ta * 16 + row) + ri;
    const cx<double> *rbase = kb + tb * 16 + row;

    d4 ar[9], ai[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) {
        ar[c] = d4{0.0, 0.0, 0.0, 0.0};
        ai[c] = d4{0.0, 0.0, 0.0, 0.0};
    }

    for (int s0 = 0; s0 < nsnap; s0 += 2) {
        const int s = s0 + soff;
        const bool ok = s < nsnap;
        double Lf[NFIELD];
        cx<double> Rf[NFIELD];
#pragma unroll
        for (int f = 0; f < NFIELD; ++f) {
            const size_t o = f * fstride + (size_t)s * d.nyp;
            Lf[f] = ok ? lbase[2 * o] : 0.0;
            Rf[f] = ok ? rbase[o] : cx<double>{0.0, 0.0};
        }
        // left operand (planes Y1): fluctuations and Q_ij
        const double lu = Lf[F_U], lv = Lf[F_V], lw = Lf[F_W], lp = Lf[F_P];
        const double lq = Lf[F_UU] + Lf[F_VV] + Lf[F_WW];
        const double lQxx = 2.0 * Lf[F_UU] + lq, lQyy = 2.0 * Lf[F_VV] + lq;
        const double lQzz = 2.0 * Lf[F_WW] + lq;
        const double lQxy = 2.0 * Lf[F_UV], lQxz = 2.0 * Lf[F_UW], lQyz = 2.0 * Lf[F_VW];
        // right operand (planes Y2): real-output and imaginary-output forms
        double br[NFIELD], bi[NFIELD];
#pragma unroll
        for (int f = 0; f < NFIELD; ++f) {
            br[f] = ri ? Rf[f].y : Rf[f].x;
            bi[f] = ri ? -Rf[f].x : Rf[f].y;
        }
        const double rqr = br[F_UU] + br[F_VV] + br[F_WW];
        const double rqi = bi[F_UU] + bi[F_VV] + bi[F_WW];
        const double rQxxr = 2.0 * br[F_UU] + rqr, rQxxi = 2.0 * bi[F_UU] + rqi;
        const double rQyyr = 2.0 * br[F_VV] + rqr, rQyyi = 2.0 * bi[F_VV] + rqi;
        const double rQzzr = 2.0 * br[F_WW] + rqr, rQzzi = 2.0 * bi[F_WW] + rqi;
        const double rQxyr = 2.0 * br[F_UV], rQxyi = 2.0 * bi[F_UV];
        const double rQxzr = 2.0 * br[F_UW], rQxzi = 2.0 * bi[F_UW];
        const double rQyzr = 2.0 * br[F_VW], rQyzi = 2.0 * bi[F_VW];
        const double ur = br[F_U], ui = bi[F_U], vr = br[F_V], vi = bi[F_V];
        const double wr = br[F_W], wi = bi[F_W], pr = br[F_P], pi = bi[F_P];

        // c0: scale energy
        GKE_MFMA2(ar[0], ai[0], lu, ur, ui);
        GKE_MFMA2(ar[0], ai[0], lv, vr, vi);
        GKE_MFMA2(ar[0], ai[0], lw, wr, wi);
        // c1: flux x
        GKE_MFMA2(ar[1], ai[1], lQxx, ur, ui);
        GKE_MFMA2(ar[1], ai[1], lQxy, vr, vi);
        GKE_MFMA2(ar[1], ai[1], lQxz, wr, wi);
        GKE_MFMA2(ar[1], ai[1], -lu, rQxxr, rQxxi);
        GKE_MFMA2(ar[1], ai[1], -lv, rQxyr, rQxyi);
        GKE_MFMA2(ar[1], ai[1], -lw, rQxzr, rQxzi);
        // c2: flux z
        GKE_MFMA2(ar[2], ai[2], lQxz, ur, ui);
        GKE_MFMA2(ar[2], ai[2], lQyz, vr, vi);
        GKE_MFMA2(ar[2], ai[2], lQzz, wr, wi);
        GKE_MFMA2(ar[2], ai[2], -lu, rQxzr, rQxzi);
        GKE_MFMA2(ar[2], ai[2], -lv, rQyzr, rQyzi);
        GKE_MFMA2(ar[2], ai[2], -lw, rQzzr, rQzzi);
        // c3, c4: y-flux halves
        GKE_MFMA2(ar[3], ai[3], lQxy, ur, ui);
        GKE_MFMA2(ar[3], ai[3], lQyy, vr, vi);
        GKE_MFMA2(ar[3], ai[3], lQyz, wr, wi);
        GKE_MFMA2(ar[4], ai[4], lu, rQxyr, rQxyi);
        GKE_MFMA2(ar[4], ai[4], lv, rQyyr, rQyyi);
        GKE_MFMA2(ar[4], ai[4], lw, rQyzr, rQyzi);
        // c5: (v, q) + (q, v)
        GKE_MFMA2(ar[5], ai[5], lv, rqr, rqi);
        GKE_MFMA2(ar[5], ai[5], lq, vr, vi);
        // c6: (p, v) + (v, p)
        GKE_MFMA2(ar[6], ai[6], lp, vr, vi);
        GKE_MFMA2(ar[6], ai[6], lv, pr, pi);
        // c7, c8
        GKE_MFMA2(ar[7], ai[7], lu, vr, vi);
        GKE_MFMA2(ar[8], ai[8], lv, ur, ui);
    }

    // term spectra: R FX FY FZ PHI PP UVS UVA
    const size_t ptot = (size_t)d.ntp * 256;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const size_t el = (size_t)tp * 256 + (kq + 4 * v) * 16 + row;
        double sr[NSPEC], si[NSPEC];
        sr[S_R] = ar[0][v];
        si[S_R] = ai[0][v];
        sr[S_FX] = ar[1][v];
        si[S_FX] = ai[1][v];
        sr[S_FY] = ar[3][v] - ar[4][v];
        si[S_FY] = ai[3][v] - ai[4][v];
        sr[S_FZ] = ar[2][v];
        si[S_FZ] = ai[2][v];
        sr[S_PHI] = 2.0 * ar[5][v] - ar[3][v] - ar[4][v];
        si[S_PHI] = 2.0 * ai[5][v] - ai[3][v] - ai[4][v];
        sr[S_PP] = ar[6][v];
        si[S_PP] = ai[6][v];
        sr[S_UVS] = ar[7][v] + ar[8][v];
        si[S_UVS] = ai[7][v] + ai[8][v];
        sr[S_UVA] = ar[8][v] - ar[7][v];
        si[S_UVA] = ai[8][v] - ai[7][v];
#pragma unroll
        for (int sp = 0; sp < NSPEC; ++sp) {
            cx<double> *dst = acc + ((size_t)sp * d.nk + k) * ptot + el;
            cx<double> val = cx<double>{sr[sp], si[sp]};
            if (accumulate) {
                const cx<double> old = *dst;
                val.x += old.x;
                val.y += old.y;
            }
            *dst = val;
        }
    }
}

hipError_t launch_rankk_f64(hipStream_t st, const Dims &d, const Tables &t,
                            const cx<double> *spec, int nsnap, int accumulate,
                            cx<double> *acc)
{
    const long long total = (long long)d.nk * d.ntp;
    if (total >= (1LL << 31) - 8) return hipErrorInvalidValue;
    const int G = (int)((total + 7) / 8 * 8);
    hipLaunchKernelGGL(k_rankk_f64, dim3(G), dim3(64), 0, st, spec, d, t.tile_a, t.tile_b, nsnap,
                       accumulate, (int)total, acc);
    return hipGetLastError();
}

}  // namespace gke
