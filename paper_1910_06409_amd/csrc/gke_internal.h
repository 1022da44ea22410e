// gke_internal.h -- shapes and kernel launchers shared by the library's own
// sources (never by the CPU oracle).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <type_traits>

#include "fft_lds.h"

namespace gke {

// fields carried in the spectra, in this order: the fluctuations and six
// combinations of the in-plane products formed in physical space (Section
// "Products instead of correlations"): Q_ij = 2 u'_i u'_j + delta_ij q with
// q = u'_i u'_i.  q itself is (Q_xx + Q_yy + Q_zz) / 5.
enum { F_U = 0, F_V, F_W, F_P, F_QXX, F_QYY, F_QZZ, F_QXY, F_QXZ, F_QYZ, NFIELD };

// precision of the cross-spectral update (GKE_PREC_*)
enum { PREC_FP64 = 0, PREC_BF16X3 = 1 };

// one complex spectral value split for the three-term BF16 products, as BF16
// bit patterns with hi = RN(x), lo = RN(x - hi) for x = re, im; the two high
// parts share one dword and the two low parts the other
struct bf16x4 {
    unsigned int hi;  // re_hi | im_hi << 16
    unsigned int lo;  // re_lo | im_lo << 16
};
// The split spectra hold the values of four consecutive snapshots of one
// plane as one 32-byte record: the four hi dwords, then the four lo dwords
// (snapshot 4 q + i at dword i), so that one 16-byte load is a whole operand
// of the matrix-core update (k_rankk_bf16.hip).  Record (k, f, q, j) sits at
// ((k NFIELD + f) nqs + q) nys + j.
struct SplitRec {
    unsigned int h[4];
    unsigned int l[4];
};

// term spectra accumulated per unordered pair tile (see k_rankk.hip)
enum { S_R = 0, S_FX, S_FY, S_FZ, S_PHI, S_PP, S_UVS, S_UVA, NSPEC };

// r-space maps produced by the inverse transforms in finalize; M_H, the
// spectral divergence of the homogeneous scale fluxes (the r_x and r_z part
// of the budget residual), only when the residual is requested
enum { M_R = 0, M_DRX, M_DRZ, M_FX, M_FY, M_FZ, M_PHI, M_PP, M_UVS, M_UVA, NMAP, M_H = NMAP };
// planes of the finalize intermediate (kz-transformed spectra): every map but
// M_DRX, which the kx pass forms from the M_R plane (i alpha is constant along kz);
// M_H takes plane NMID after them
constexpr int NMID = NMAP - 1;
__host__ __device__ inline int mid_plane(int m) { return m == M_DRX ? M_R : m > M_DRX ? m - 1 : m; }

// terms kept as full-plane maps per slab in the general output modes:
// T1-T5, T7-T10, T12, T13 (T6, T11 and T14 are formed from them at output)
constexpr int NSTORED = 11;

// profile rows (same order as the public GKE_P_* rows)
enum { P_U = 0, P_V, P_W, P_P, P_S, P_Q, P_UV, P_PV, P_TX, P_TY, P_TZ, P_EPS, NPROF };

// physical-space moment partials per (plane, z block): q uv pv qu qv qw and,
// on the split-BF16 path, the wall-normal gradient energy gy
enum { MP_Q = 0, MP_UV, MP_PV, MP_QU, MP_QV, MP_QW, MP_GY, NMOMP };

// pass-1 plane sums are split over this many blocks per plane
constexpr int NSPLIT = 32;

// LDS transforms: at most FFT_CAP complex elements per block and FFT_BLOCK
// threads per block.  4096 FP64 elements (64 KiB) and 512 threads let two
// blocks share a compute unit (160 KiB LDS, 128 VGPRs at 4 waves per SIMD),
// so that one block's global loads overlap the other's transform.
#ifndef GKE_FFT_CAP
#define GKE_FFT_CAP 4096
#endif
#ifndef GKE_FFT_BLOCK
#define GKE_FFT_BLOCK 512
#endif
#ifndef GKE_FFT_WAVES
#define GKE_FFT_WAVES 4
#endif
constexpr int FFT_CAP = GKE_FFT_CAP;
constexpr int MAX_NTX = 16;   // complex transforms (two pairs each) per kx-pass block
constexpr int FFT_BLOCK = GKE_FFT_BLOCK;
// launch bounds of the transform kernels: FFT_BLOCK threads, at least
// GKE_FFT_WAVES waves per SIMD (so that several blocks share a compute unit)
#define GKE_FFT_BOUNDS __launch_bounds__(GKE_FFT_BLOCK, GKE_FFT_WAVES)
constexpr size_t LDS_BUDGET = 156 * 1024;
// The x pass and the kx finalize also come in a smaller shape, 256 threads and
// 2048 elements per block (four blocks per compute unit), used when the grid
// still gives each block at least two z rows (x pass) or eight transforms (kx
// finalize); measured faster for both at the re200 size.
constexpr int SMALL_BLOCK = 256, SMALL_CAP = 2048;
template <int BLOCK>
constexpr int cap_of() { return BLOCK == SMALL_BLOCK ? SMALL_CAP : FFT_CAP; }

// Transform lengths whose plans are compiled in (the x and z lengths of the
// channel grids the library is tuned for, 192 x 160 and 512 x 384): f is
// called with std::integral_constant<int, n> for those, with
// std::integral_constant<int, 0> (the run-time plan) for any other n.
template <typename F>
inline void with_fft_len(int n, F &&f)
{
    switch (n) {
    case 160: f(std::integral_constant<int, 160>{}); break;
    case 192: f(std::integral_constant<int, 192>{}); break;
    case 384: f(std::integral_constant<int, 384>{}); break;
    case 512: f(std::integral_constant<int, 512>{}); break;
    default: f(std::integral_constant<int, 0>{}); break;
    }
}

struct Dims {
    int nx, ny, nz;
    int nkx;          // nx/2 + 1
    int nk;           // nkx * nz
    int ntile;        // full 16-plane tiles: ny / 16
    int ntp;          // ntile (ntile + 1) / 2 unordered tile pairs
    int npair_tiles;  // 256 ntp pairs handled on the matrix cores
    int nsb;          // groups of four tile pairs (split-BF16 rank-k workgroups)
    int npair;        // all unordered pairs (tile pairs + remainder pairs)
    int pstr;         // pair stride of the accumulators: npair rounded up to 8 (128-byte rows)
    int kxblk;        // threads of a kx-finalize block (SMALL_BLOCK or FFT_BLOCK)
    int zpblk;        // threads of a z-pass block (SMALL_BLOCK or FFT_BLOCK)
    int zb, nzb;      // z rows per block in the x pass, number of blocks
    int zg, nzg;      // z rows per group of the x-transformed layout (a multiple of zb)
    int jb, njb;      // planes per block in the z pass, number of blocks
    int pbz;          // pairs per block in the finalize kz pass
    int ntx;          // complex transforms (two pairs each) per block in the kx pass
    int chunk;        // snapshot slots in the spectra buffer
    int nys;          // planes per snapshot row of the spectra: ny rounded up so that
                      // every 16-plane tile of a row starts on a 128-byte line
    int nqs;          // split path: snapshot quads per chunk, (chunk + 3) / 4
    int prec;         // PREC_FP64 or PREC_BF16X3
    int zplanes;      // an autotuned bound on the planes of a z-pass block (0: none)
    int nqo, npo;     // rows (rz) and columns (rx) of an output map: the separations kept
                      // by the rx/rz undersampling (Nz and Nx/2 + 1 or Nx without it)
    double lx, lz, nu;
};

// Stored value of (field f, snapshot s, plane j) of one wavenumber (kb: its
// first element), as loaded (raw_at) and as an FP64 complex (value_of).
__device__ __forceinline__ const cx<double> *spec_base(const cx<double> *s, const Dims &d, int k)
{
    return s + (size_t)k * NFIELD * d.chunk * d.nys;
}
__device__ __forceinline__ const SplitRec *spec_base(const SplitRec *s, const Dims &d, int k)
{
    return s + (size_t)k * NFIELD * d.nqs * d.nys;
}
__device__ __forceinline__ cx<double> raw_at(const cx<double> *kb, const Dims &d, int f, int s,
                                             int j)
{
    return kb[(f * d.chunk + s) * d.nys + j];   // below 2^31 within a wavenumber (host)
}
__device__ __forceinline__ bf16x4 raw_at(const SplitRec *kb, const Dims &d, int f, int s, int j)
{
    const unsigned int *r = kb[(f * d.nqs + (s >> 2)) * d.nys + j].h;
    return bf16x4{r[s & 3], r[4 + (s & 3)]};
}
__device__ __forceinline__ cx<double> value_of(cx<double> v) { return v; }
__device__ __forceinline__ cx<double> value_of(bf16x4 v)
{
    const double rh = __uint_as_float(v.hi << 16), rl = __uint_as_float(v.lo << 16);
    const double ih = __uint_as_float(v.hi & 0xffff0000u), il = __uint_as_float(v.lo & 0xffff0000u);
    return cx<double>{rh + rl, ih + il};
}
template <typename S>
struct RawOf {
    typedef cx<double> type;
};
template <>
struct RawOf<SplitRec> {
    typedef bf16x4 type;
};

// pair table entry: j1 | j2 << 12 | mirror << 24 (mirror: also write (j2, j1))
__host__ __device__ inline int pair_j1(int code) { return code & 4095; }
__host__ __device__ inline int pair_j2(int code) { return (code >> 12) & 4095; }
__host__ __device__ inline int pair_mirror(int code) { return (code >> 24) & 1; }

struct Tables {
    const cx<double> *twx;   // exp(-2 pi i m/nx)
    const cx<double> *twz;   // exp(-2 pi i m/nz)
    const cx<float> *twx32;  // the same rounded to FP32
    const cx<float> *twz32;
    const double *w5;        // [ny][5] five-point weights
    const double *w2;        // [ny][5] five-point second-derivative weights (same windows)
    const int *j0;           // [ny] first stencil node
    const int *tile_a;       // [ntp] tile-pair row tiles (index into rowplane / 16)
    const int *tile_b;       // [ntp] tile-pair column tiles (planes 16 b .. 16 b + 15)
    const int *sblk;         // [12 nsb] groups of four tile pairs (split rank-k): four tile
                             // slots, the pair of each wave, each wave's operand slots
    const int *rowplane;     // [16 * row tiles] plane of each row of the row tiles
    const int *rowidx;       // [ny] row of plane Y1 in the full-plane map buffer, or -1
    const int *pairs;        // [npair] pair table
    const int *pidx;         // [ny][ny] compact pair index of (Y1, Y2), either order
    const int *rzk;          // [nqo] rz index of each output row (kept separations)
    const int *rzinv;        // [nz] output row of rz index q, -1 if not kept
    const int *rxk;          // [npo] rx index of each output column
    FftPlanDev px, pz;
};

// twiddle table of the x (which = 0) or z (which = 1) transforms in type T
template <typename T>
__device__ __forceinline__ const cx<T> *tw_of(const Tables &t, int which);
template <>
__device__ __forceinline__ const cx<double> *tw_of<double>(const Tables &t, int which)
{
    return which ? t.twz : t.twx;
}
template <>
__device__ __forceinline__ const cx<float> *tw_of<float>(const Tables &t, int which)
{
    return which ? t.twz32 : t.twx32;
}

// Sums each of eight values over the 64 lanes of a wave in a fixed order: on
// return, every lane of the group of eight lanes g = lane / 8 holds the sum of
// v[g].  Each step halves the values a lane keeps and sends the other half to
// its partner (lanes 32, 16, 8 apart), then the last three steps finish the
// sum within the group: 10 exchanges instead of 8 x 6.
__device__ __forceinline__ double wave_sum8(const double (&v)[8])
{
    const int lane = threadIdx.x & 63;
    double a[4], b[2];
    const bool h5 = lane & 32, h4 = lane & 16, h3 = lane & 8;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const double keep = h5 ? v[4 + i] : v[i], send = h5 ? v[i] : v[4 + i];
        a[i] = keep + __shfl_xor(send, 32, 64);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const double keep = h4 ? a[2 + i] : a[i], send = h4 ? a[i] : a[2 + i];
        b[i] = keep + __shfl_xor(send, 16, 64);
    }
    double c = (h3 ? b[1] : b[0]) + __shfl_xor(h3 ? b[0] : b[1], 8, 64);
    c += __shfl_xor(c, 4, 64);
    c += __shfl_xor(c, 2, 64);
    c += __shfl_xor(c, 1, 64);
    return c;
}

// pass 1: plane sums of u~ v~ w~ p~ added into sums[f][ny][NSPLIT], f < 4;
// with gy, also the plane sums of (D u~)^2 + (D v~)^2 + (D w~)^2 (D: the
// five-point wall-normal weights) into sums[4][ny][NSPLIT]
hipError_t launch_plane_sums(hipStream_t st, const Dims &d, const Tables &t, int f32, int gy,
                             const void *u, const void *v, const void *w, const void *p,
                             double *sums);
// means = sums / count, S = D U (profile rows U V W P S); with gy1 != NULL
// also gy1[j] = <(D u')^2 + (D v')^2 + (D w')^2> = <(D u~)^2 + ...> - (D U)^2
// - (D V)^2 - (D W)^2 (D commutes with the average)
hipError_t launch_means(hipStream_t st, const Dims &d, const Tables &t, const double *sums,
                        double count, double *prof, double *gy1);
// S = D U only (means already in prof)
hipError_t launch_shear(hipStream_t st, const Dims &d, const Tables &t, double *prof);
// plane averages of u'_i(Y1) u'_i(Y2) for |Y1 - Y2| <= 4 (r0[Y1][Y2 - Y1]) and
// of |grad_xz u'|^2 (gxz[Y]) from the scale-energy spectrum accumulators
hipError_t launch_r0(hipStream_t st, const Dims &d, const Tables &t, const cx<double> *acc,
                     double inv_count, double *r0, double *gxz);
// reduce moment partials into the remaining profile rows; eps from gxz and
// the wall-normal part: gy_mode 0 from r0 (Parseval, FP64 spectra), 1 from
// gy1 (first scan), 2 from the moment partials (the x pass's stencil)
hipError_t launch_profiles(hipStream_t st, const Dims &d, const Tables &t, const double *momp,
                           const double *r0, const double *gxz, const double *gy1, int gy_mode,
                           double count, double *prof);

// pass 2, per snapshot: fluctuations, products, x transforms, moments;
// with gy (split path only) also the plane sums of (D u')^2 + (D v')^2 +
// (D w')^2 from the five-plane stencil of the fluctuations.
// inter holds cx<double> (FP64 path) or cx<float> (split-BF16 path).
hipError_t launch_fluct_xfft(hipStream_t st, const Dims &d, const Tables &t, int f32, int gy,
                             const void *u, const void *v, const void *w, const void *p,
                             const double *prof, void *inter, double *momp);
// z transforms and packing into the spectra slot (FP64 path: cx<double>)
hipError_t launch_zfft_pack(hipStream_t st, const Dims &d, const Tables &t, const void *inter,
                            int slot, void *spec);
// split path: z transforms of ng <= 4 snapshots (x-transformed rows in inter,
// one buffer of inter_stride elements each) into the records of quad q
// (missing snapshots of a partial quad written as zero)
hipError_t launch_zfft_rec(hipStream_t st, const Dims &d, const Tables &t, const void *inter,
                           size_t inter_stride, int q, int ng, SplitRec *spec);
// cross-spectral rank-k update over the snapshots of one chunk, pairs of full
// plane tiles (FP64 MFMA)
hipError_t launch_rankk_f64(hipStream_t st, const Dims &d, const Tables &t,
                            const cx<double> *spec, int nsnap, int accumulate,
                            cx<double> *acc);
// the same with split-BF16 three-term MFMA products and FP32 accumulation
hipError_t launch_rankk_bf16x3(hipStream_t st, const Dims &d, const Tables &t,
                               const SplitRec *spec, int nsnap, int accumulate,
                               cx<double> *acc);
// the pairs that involve the last Ny mod 16 planes (FP64 vector arithmetic)
hipError_t launch_rankk_rem_f64(hipStream_t st, const Dims &d, const Tables &t,
                                const cx<double> *spec, int nsnap, int accumulate,
                                cx<double> *acc);
hipError_t launch_rankk_rem_bf16x3(hipStream_t st, const Dims &d, const Tables &t,
                                   const SplitRec *spec, int nsnap, int accumulate,
                                   cx<double> *acc);
// finalize: inverse transform along kz of the term spectra of the pairs
// [p0, p1) of the compact pair index, scaled by 1/count
hipError_t launch_fin_kz(hipStream_t st, const Dims &d, const Tables &t,
                         const cx<double> *acc, int p0, int p1, double inv_count,
                         cx<double> *mid);
// residual: the spectral divergence of the homogeneous fluxes,
//   H^ = i alpha FX^ + i beta FZ^ - 2 (U(Y2) - U(Y1)) i alpha R^ - 4 nu (alpha^2 + beta^2) R^,
// of the pairs [p0, p1), scaled by 1/count, inverse-transformed along kz into
// mid plane NMID (the kx pass then transforms it as map M_H)
hipError_t launch_fin_kz_h(hipStream_t st, const Dims &d, const Tables &t,
                           const cx<double> *acc, int p0, int p1, double inv_count,
                           const double *prof, cx<double> *mid);
// Output maps below are FP64, or FP32 with f32 = 1 (assembled in FP64, rounded
// once when stored).
// finalize: inverse real transform along kx, FP64 assembly.  full = 0: both
// orientations into the all-pairs half-plane maps out[t][Y1][Y2][rz][rx <= Nx/2];
// full = 1: orientation (Y1, Y2) of the pair code only, every rx, into
// out[t][rowidx[Y1]][Y2][rz][rx < Nx]
hipError_t launch_fin_kx(hipStream_t st, const Dims &d, const Tables &t,
                         const cx<double> *mid, int p0, int p1, const double *prof,
                         void *const *out, int f32, int full, void *resid);
// residual, Y part: resid += (d/dY2 - d/dY1)(T5 + T6)/2 + (d/dY1 + d/dY2)(T9 + T10 + T11)
// - (T12 + T13 + T14), five-point derivatives along Y1 and Y2 of the maps
// out[t][Y1][Y2][rz][rx <= Nx/2]; resid holds the homogeneous part on entry
hipError_t launch_resid(hipStream_t st, const Dims &d, const Tables &t, void *const *out,
                        int f32, const double *prof, void *resid);
// general output modes: mirror average, output domain, T6/T11/T14, from the
// full-plane map buffer of the slab rows (see k_final.hip)
hipError_t launch_slab_out(hipStream_t st, const Dims &d, const Tables &t, const double *mf,
                           size_t mstride, const int *opairs, int nopairs, const double *prof,
                           int mirror, void *const *out, int f32);
// band accumulators for eps in the general modes: band[a][Y][k] += sum over the
// chunk of sum_i Re conj(u_i^(k; Y)) u_i^(k; Y + a), a = 0..4
hipError_t launch_band(hipStream_t st, const Dims &d, const void *spec, int nsnap,
                       int accumulate, double *band);
// r0, gxz (as launch_r0) from the band accumulators
hipError_t launch_r0_band(hipStream_t st, const Dims &d, const double *band, double inv_count,
                          double *r0, double *gxz);
// Step 3: T6 and T11 from T1 along Y1 and Y2
hipError_t launch_fd_terms(hipStream_t st, const Dims &d, const Tables &t, const void *t1,
                           void *t6, void *t11, int f32);
// Step 1 upstream (k_step1.hip): from v^ and omega_y^ ([Ny][Nz][Nkx] complex)
// and the plane-mean u, w ([Ny]) the physical u, v, w and p ([Ny][Nz][Nx]);
// vel [3], prod [6], ph: spectral buffers of [Ny][Nz][Nkx]; su [Ny][9][nk],
// sb [Ny][nk]: the pivot rows of the pressure elimination
hipError_t launch_step1(hipStream_t st, const Dims &d, const Tables &t, const cx<double> *vh,
                        const cx<double> *oh, const double *mean_u, const double *mean_w,
                        cx<double> *vel, cx<double> *prod, cx<double> *ph, double *su,
                        cx<double> *sb, double *u, double *v, double *w, double *p);
// zero `bytes` bytes at p (8-byte aligned, a multiple of 8) with a fill kernel
hipError_t launch_zero(hipStream_t st, void *p, size_t bytes);
// T14 = -2 (eps(Y1) + eps(Y2))
hipError_t launch_t14(hipStream_t st, const Dims &d, const double *prof, void *t14, int f32);

}  // namespace gke
