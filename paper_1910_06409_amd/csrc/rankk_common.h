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

// The 27 products conj(A) B of one pair and snapshot into the nine channels
// (A: plane Y1, B: plane Y2, fields in the order of the spectra), formed in
// type V and summed in FP64.
template <typename V>
__device__ __forceinline__ void rem_macs(double *cr, double *ci, const cx<V> *A, const cx<V> *B)
{
    const V fifth = V(0.2);
    const cx<V> qa = cx<V>{fifth * (A[F_QXX].x + A[F_QYY].x + A[F_QZZ].x),
                           fifth * (A[F_QXX].y + A[F_QYY].y + A[F_QZZ].y)};
    const cx<V> qb = cx<V>{fifth * (B[F_QXX].x + B[F_QYY].x + B[F_QZZ].x),
                           fifth * (B[F_QXX].y + B[F_QYY].y + B[F_QZZ].y)};
    // conj(a) b accumulated into channel c with sign sg
    auto mac = [&](int c, cx<V> a, cx<V> b, double sg) {
        cr[c] += sg * (double)(a.x * b.x + a.y * b.y);
        ci[c] += sg * (double)(a.x * b.y - a.y * b.x);
    };
    const cx<V> ua = A[F_U], va = A[F_V], wa = A[F_W], pa = A[F_P];
    const cx<V> ub = B[F_U], vb = B[F_V], wb = B[F_W], pb = B[F_P];
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
    const S *kb = spec_base(spec, d, k);
    double cr[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, ci[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if constexpr (sizeof(S) == sizeof(SplitRec)) {
        // one snapshot quad per step: 16-byte loads of both planes' records
        // (the h and l halves of a wave's records cover whole lines), then the
        // four snapshots with hi + lo as FP32 (exact: two 8-bit significands
        // 2^-8 apart) and FP32 products (error 2^-24, far below the split
        // form's 2^-16), summed in FP64
        const int nq = (nsnap + 3) >> 2;
        for (int q = 0; q < nq; ++q) {
            typedef unsigned int u4v __attribute__((ext_vector_type(4)));
            u4v ah[NFIELD], al[NFIELD], bh[NFIELD], bl[NFIELD];
#pragma unroll
            for (int f = 0; f < NFIELD; ++f) {
                const int rq = (f * d.nqs + q) * d.nys;
                const SplitRec *ra = kb + rq + j1, *rb = kb + rq + j2;
                ah[f] = *reinterpret_cast<const u4v *>(ra->h);
                al[f] = *reinterpret_cast<const u4v *>(ra->l);
                bh[f] = *reinterpret_cast<const u4v *>(rb->h);
                bl[f] = *reinterpret_cast<const u4v *>(rb->l);
            }
            auto val = [](unsigned int h, unsigned int l) {
                return cx<float>{__uint_as_float(h << 16) + __uint_as_float(l << 16),
                                 __uint_as_float(h & 0xffff0000u) + __uint_as_float(l & 0xffff0000u)};
            };
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                if (4 * q + t < nsnap) {
                    cx<float> A[NFIELD], B[NFIELD];
#pragma unroll
                    for (int f = 0; f < NFIELD; ++f) {
                        A[f] = val(ah[f][t], al[f][t]);
                        B[f] = val(bh[f][t], bl[f][t]);
                    }
                    rem_macs(cr, ci, A, B);
                }
            }
        }
    } else {
        typedef typename RawOf<S>::type Raw;
        Raw An[NFIELD], Bn[NFIELD];
#pragma unroll
        for (int f = 0; f < NFIELD; ++f) {
            An[f] = raw_at(kb, d, f, 0, j1);
            Bn[f] = raw_at(kb, d, f, 0, j2);
        }
        for (int s = 0; s < nsnap; ++s) {
            cx<double> A[NFIELD], B[NFIELD];
#pragma unroll
            for (int f = 0; f < NFIELD; ++f) {
                A[f] = value_of(An[f]);
                B[f] = value_of(Bn[f]);
            }
            const int sn = s + 1 < nsnap ? s + 1 : s;
#pragma unroll
            for (int f = 0; f < NFIELD; ++f) {
                An[f] = raw_at(kb, d, f, sn, j1);
                Bn[f] = raw_at(kb, d, f, sn, j2);
            }
            rem_macs(cr, ci, A, B);
        }
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
    constexpr bool flat = sizeof(S) == sizeof(SplitRec);
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
