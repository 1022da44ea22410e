// rankk_common.h -- pieces shared by the FP64 and the split-BF16 forms of the
// cross-spectral update: the epilogue that forms the eight term spectra from
// the nine product accumulators, and the FP64 vector kernel for the pairs that
// involve the last Ny mod 16 planes.
#pragma once
#include "gke_internal.h"

namespace gke {

// Store the eight term spectra of one element from the nine accumulators
// (part < 0: all of them; part 0: S_FY S_PHI from c3 c4 c5; part 1: S_FX
// S_UVS S_UVA from c1 c7 c8; part 2: S_R S_FZ S_PP from c0 c2 c6).
__device__ __forceinline__ void store_spectra_part(cx<double> *acc, size_t sp_stride, size_t o,
                                                   const double *cr, const double *ci,
                                                   int accumulate, int part)
{
    double sr[NSPEC], si[NSPEC];
    sr[S_R] = cr[0];
    si[S_R] = ci[0];
    sr[S_FX] = cr[1];
    si[S_FX] = ci[1];
    sr[S_FY] = cr[3] - cr[4];
    si[S_FY] = ci[3] - ci[4];
    sr[S_FZ] = cr[2];
    si[S_FZ] = ci[2];
    sr[S_PHI] = 2.0 * cr[5] - cr[3] - cr[4];
    si[S_PHI] = 2.0 * ci[5] - ci[3] - ci[4];
    sr[S_PP] = cr[6];
    si[S_PP] = ci[6];
    sr[S_UVS] = cr[7] + cr[8];
    si[S_UVS] = ci[7] + ci[8];
    sr[S_UVA] = cr[8] - cr[7];
    si[S_UVA] = ci[8] - ci[7];
#pragma unroll
    for (int sp = 0; sp < NSPEC; ++sp) {
        const int owner = (sp == S_FY || sp == S_PHI) ? 0
                          : (sp == S_FX || sp == S_UVS || sp == S_UVA) ? 1 : 2;
        if (part >= 0 && owner != part) continue;
        cx<double> *dst = acc + sp * sp_stride + o;
        cx<double> val = cx<double>{sr[sp], si[sp]};
        if (accumulate) {
            const cx<double> old = *dst;
            val.x += old.x;
            val.y += old.y;
        }
        *dst = val;
    }
}

__device__ __forceinline__ void store_spectra(cx<double> *acc, size_t sp_stride, size_t o,
                                              const double *cr, const double *ci,
                                              int accumulate)
{
    store_spectra_part(acc, sp_stride, o, cr, ci, accumulate, -1);
}

// Pairs that involve the last Ny mod 16 planes: one thread per (k, pair), FP64
// vector arithmetic on the stored values (for split spectra: hi + lo).
// pairs[i] = j1 | j2 << 12 for compact index P = npair_tiles + i.
__device__ __forceinline__ cx<double> spec_value(const cx<double> *s, size_t i) { return s[i]; }
__device__ __forceinline__ cx<double> spec_value(const bf16x4 *s, size_t i)
{
    const bf16x4 v = s[i];
    const double rh = __uint_as_float(v.hi << 16), rl = __uint_as_float(v.lo << 16);
    const double ih = __uint_as_float(v.hi & 0xffff0000u), il = __uint_as_float(v.lo & 0xffff0000u);
    return cx<double>{rh + rl, ih + il};
}

// One thread per (k, pair).  FLAT: threads packed across wavenumbers with the
// pair fastest, so that no wave is left mostly empty when nrem is small (129
// pairs at Ny = 129), measured faster for the split spectra; otherwise blocks
// of one wavenumber (blockIdx.y), measured faster for FP64.
// The loads of snapshot s + 1 are issued before the products of snapshot s.
template <typename S, bool FLAT>
__global__ __launch_bounds__(64, 2) void k_rankk_rem(const S *__restrict__ spec, Dims d,
                                                     const int *__restrict__ pairs, int nrem,
                                                     int nsnap, int accumulate,
                                                     cx<double> *__restrict__ acc)
{
    int k, i;
    if (FLAT) {
        const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
        if (t >= (long long)nrem * d.nk) return;
        k = (int)(t / nrem);
        i = (int)(t - (long long)k * nrem);
    } else {
        i = blockIdx.x * blockDim.x + threadIdx.x;
        k = blockIdx.y;
        if (i >= nrem) return;
    }
    const int code = pairs[d.npair_tiles + i];
    const int j1 = pair_j1(code), j2 = pair_j2(code);
    const int fstride = d.chunk * d.nys;   // offsets within one wavenumber stay below 2^31
    const S *kb = spec + (size_t)k * NFIELD * fstride;
    double cr[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, ci[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    S An[NFIELD], Bn[NFIELD];
#pragma unroll
    for (int f = 0; f < NFIELD; ++f) {
        An[f] = kb[f * fstride + j1];
        Bn[f] = kb[f * fstride + j2];
    }
    for (int s = 0; s < nsnap; ++s) {
        cx<double> A[NFIELD], B[NFIELD];
#pragma unroll
        for (int f = 0; f < NFIELD; ++f) {
            A[f] = spec_value(An, f);
            B[f] = spec_value(Bn, f);
        }
        const int sn = (s + 1 < nsnap ? s + 1 : s) * d.nys;
#pragma unroll
        for (int f = 0; f < NFIELD; ++f) {
            An[f] = kb[f * fstride + sn + j1];
            Bn[f] = kb[f * fstride + sn + j2];
        }
        const cx<double> qa = cx<double>{0.2 * (A[F_QXX].x + A[F_QYY].x + A[F_QZZ].x),
                                         0.2 * (A[F_QXX].y + A[F_QYY].y + A[F_QZZ].y)};
        const cx<double> qb = cx<double>{0.2 * (B[F_QXX].x + B[F_QYY].x + B[F_QZZ].x),
                                         0.2 * (B[F_QXX].y + B[F_QYY].y + B[F_QZZ].y)};
        // conj(a) b accumulated into channel c with sign sg
        auto mac = [&](int c, cx<double> a, cx<double> b, double sg) {
            cr[c] += sg * (a.x * b.x + a.y * b.y);
            ci[c] += sg * (a.x * b.y - a.y * b.x);
        };
        const cx<double> ua = A[F_U], va = A[F_V], wa = A[F_W], pa = A[F_P];
        const cx<double> ub = B[F_U], vb = B[F_V], wb = B[F_W], pb = B[F_P];
        mac(0, ua, ub, 1.0); mac(0, va, vb, 1.0); mac(0, wa, wb, 1.0);
        mac(1, A[F_QXX], ub, 1.0); mac(1, A[F_QXY], vb, 1.0); mac(1, A[F_QXZ], wb, 1.0);
        mac(1, ua, B[F_QXX], -1.0); mac(1, va, B[F_QXY], -1.0); mac(1, wa, B[F_QXZ], -1.0);
        mac(2, A[F_QXZ], ub, 1.0); mac(2, A[F_QYZ], vb, 1.0); mac(2, A[F_QZZ], wb, 1.0);
        mac(2, ua, B[F_QXZ], -1.0); mac(2, va, B[F_QYZ], -1.0); mac(2, wa, B[F_QZZ], -1.0);
        mac(3, A[F_QXY], ub, 1.0); mac(3, A[F_QYY], vb, 1.0); mac(3, A[F_QYZ], wb, 1.0);
        mac(4, ua, B[F_QXY], 1.0); mac(4, va, B[F_QYY], 1.0); mac(4, wa, B[F_QYZ], 1.0);
        mac(5, va, qb, 1.0); mac(5, qa, vb, 1.0);
        mac(6, pa, vb, 1.0); mac(6, va, pb, 1.0);
        mac(7, ua, vb, 1.0);
        mac(8, va, ub, 1.0);
    }
    store_spectra(acc, (size_t)d.nk * d.pstr, (size_t)k * d.pstr + d.npair_tiles + i, cr, ci,
                  accumulate);
}

template <typename S>
hipError_t launch_rankk_rem(hipStream_t st, const Dims &d, const Tables &t, const S *spec,
                            int nsnap, int accumulate, cx<double> *acc)
{
    const int nrem = d.npair - d.npair_tiles;
    if (nrem <= 0) return hipSuccess;
    constexpr bool flat = sizeof(S) == sizeof(bf16x4);
    if (flat) {
        const long long nthr = (long long)nrem * d.nk;
        if (nthr >= (1LL << 37)) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_rankk_rem<S, true>), dim3((unsigned)((nthr + 63) / 64)), dim3(64), 0,
                           st, spec, d, t.pairs, nrem, nsnap, accumulate, acc);
    } else {
        hipLaunchKernelGGL((k_rankk_rem<S, false>), dim3((nrem + 63) / 64, d.nk), dim3(64), 0, st,
                           spec, d, t.pairs, nrem, nsnap, accumulate, acc);
    }
    return hipGetLastError();
}

}  // namespace gke
