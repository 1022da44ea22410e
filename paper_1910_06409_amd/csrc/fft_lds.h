// fft_lds.h -- batched mixed-radix (2, 3, 4, 5, 8) Stockham FFT in LDS.
//
// Used for the in-plane transforms of the method (Section "Products instead of
// correlations": correlations in x and z through the Parseval identity).
// A batch of `batch` transforms of length n lives in one LDS buffer with
// element (b, i) at buf[b * bs + fft_pad(i)]; every pass reads the inputs of all
// its butterflies into registers, then, after a barrier, writes the outputs in
// place, so the result ends in natural order in the same buffer.  Twiddles
// come from a table built on the host in FP64, one block per pass after the
// first (the first multiplies by none), laid out [j - 1][k]: entry
// (j - 1) p + k = exp(-2 pi i j k / (p R)) for the pass of radix R after
// radices of product p, so that the lanes of a wave, which take consecutive k,
// read consecutive entries; n - R_first entries in all.  The inverse direction
// conjugates them.
//   sign = -1: X[k] = sum_j x[j] exp(-2 pi i jk/n)      (forward)
//   sign = +1: x[j] = sum_k X[k] exp(+2 pi i jk/n)      (inverse, unscaled)
#pragma once
#include <hip/hip_runtime.h>

namespace gke {

// aligned to its size, so that an LDS or global access of one value is a
// single 16-byte (FP64) or 8-byte (FP32) access, not two halves
template <typename T>
struct alignas(2 * sizeof(T)) cx {
    T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return cx<T>{a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return cx<T>{a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b)
{
    return cx<T>{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return cx<T>{a.x * s, a.y * s}; }
template <typename T>
__device__ __forceinline__ cx<T> cconj(cx<T> a) { return cx<T>{a.x, -a.y}; }
// multiply by (sign * i)
template <typename T>
__device__ __forceinline__ cx<T> cmul_si(cx<T> a, int sign)
{
    return sign > 0 ? cx<T>{-a.y, a.x} : cx<T>{a.y, -a.x};
}

struct FftPlanDev {
    int n;
    int npass;
    int radix[16];   // powers of two first (the host's radix_plan)
    int swz;         // 1: the first pass's outputs sit at swz8(i) (see below)
};

// LDS layout of a batch of transforms of length n: element i of transform b
// sits at b * fft_stride(n) + pad(i).  One padding slot per 32 elements and an
// odd stride keep the strided accesses of the passes on distinct banks.
__host__ __device__ __forceinline__ int fft_pad(int i) { return i + (i >> 5); }
__host__ __device__ __forceinline__ int fft_stride(int n)
{
    const int s = n + (n >> 5) + 1;
    return s | 1;
}

// LDS banks (measured on gfx950): a 16-byte access takes 8 lanes per cycle on
// a write and 16 on a read, and is free of conflicts when those lanes fall
// on distinct 16-byte slots modulo 8 (writes) or 16 (reads); 8-byte accesses
// take 16 and 32 lanes.  The first pass of radix R writes R consecutive
// outputs per lane, i.e. a lane stride of R, an R-way conflict for R = 2, 4,
// 8 on 16-byte elements.  Its outputs therefore sit at swz8(i): the low three
// index bits XORed with the next three, a permutation within every aligned
// run of 8 elements, which puts the stride-R writes of 8 lanes on 8 distinct
// slots and keeps a read of 16 consecutive elements (aligned to 8) on 16.
__host__ __device__ __forceinline__ int swz8(int i) { return i ^ ((i >> 3) & 7); }

// a / d and a % d for 0 <= a < 2^24 through a float reciprocal, corrected
__device__ __forceinline__ int div_small(int a, int d, float inv_d)
{
    int q = (int)((float)a * inv_d);
    const int r = a - q * d;
    q += (r >= d) ? 1 : 0;
    q -= (r < 0) ? 1 : 0;
    return q;
}

// e = hi * n + lo for e = start, start + step, start + 2 step, ... with one
// division at the start and none per step (step < n or any step >= 0).
struct Walk2 {
    int hi, lo, dhi, dlo, n;
    __device__ __forceinline__ Walk2(int start, int step, int n_) : n(n_)
    {
        hi = start / n;
        lo = start - hi * n;
        dhi = step / n;
        dlo = step - dhi * n;
    }
    __device__ __forceinline__ void next()
    {
        hi += dhi;
        lo += dlo;
        if (lo >= n) {
            lo -= n;
            ++hi;
        }
    }
};

template <int R, typename T>
struct Dft;

template <typename T>
struct Dft<2, T> {
    __device__ __forceinline__ static void run(cx<T> *v, int)
    {
        cx<T> a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};

template <typename T>
struct Dft<3, T> {
    __device__ __forceinline__ static void run(cx<T> *v, int sign)
    {
        // w = exp(sign 2 pi i/3) = -1/2 + sign i sqrt(3)/2
        const T h = T(0.86602540378443864676372317075294);  // sqrt(3)/2
        cx<T> a = v[0], b = v[1], c = v[2];
        cx<T> t1 = cadd(b, c);
        cx<T> t2 = cscale(cmul_si(csub(b, c), sign), h);
        cx<T> m = csub(a, cscale(t1, T(0.5)));
        v[0] = cadd(a, t1);
        v[1] = cadd(m, t2);
        v[2] = csub(m, t2);
    }
};

template <typename T>
struct Dft<4, T> {
    __device__ __forceinline__ static void run(cx<T> *v, int sign)
    {
        cx<T> a = v[0], b = v[1], c = v[2], d = v[3];
        cx<T> s0 = cadd(a, c), d0 = csub(a, c);
        cx<T> s1 = cadd(b, d), d1 = cmul_si(csub(b, d), sign);
        v[0] = cadd(s0, s1);
        v[1] = cadd(d0, d1);
        v[2] = csub(s0, s1);
        v[3] = csub(d0, d1);
    }
};

template <typename T>
struct Dft<5, T> {
    __device__ __forceinline__ static void run(cx<T> *v, int sign)
    {
        const T c1 = T(0.30901699437494742410229341718282);   // cos(2pi/5)
        const T c2 = T(-0.80901699437494742410229341718282);  // cos(4pi/5)
        const T s1 = T(0.95105651629515357211643933337938);   // sin(2pi/5)
        const T s2 = T(0.58778525229247312916870595463907);   // sin(4pi/5)
        cx<T> a = v[0];
        cx<T> be = cadd(v[1], v[4]), bm = csub(v[1], v[4]);
        cx<T> cd = cadd(v[2], v[3]), cm = csub(v[2], v[3]);
        cx<T> r1 = cadd(a, cadd(cscale(be, c1), cscale(cd, c2)));
        cx<T> r2 = cadd(a, cadd(cscale(be, c2), cscale(cd, c1)));
        cx<T> i1 = cmul_si(cadd(cscale(bm, s1), cscale(cm, s2)), sign);
        cx<T> i2 = cmul_si(csub(cscale(bm, s2), cscale(cm, s1)), sign);
        v[0] = cadd(a, cadd(be, cd));
        v[1] = cadd(r1, i1);
        v[4] = csub(r1, i1);
        v[2] = cadd(r2, i2);
        v[3] = csub(r2, i2);
    }
};

template <typename T>
struct Dft<8, T> {
    __device__ __forceinline__ static void run(cx<T> *v, int sign)
    {
        // two radix-4 transforms on the even and odd samples, then radix-2
        cx<T> e[4] = {v[0], v[2], v[4], v[6]};
        cx<T> o[4] = {v[1], v[3], v[5], v[7]};
        Dft<4, T>::run(e, sign);
        Dft<4, T>::run(o, sign);
        const T r = T(0.70710678118654752440084436210485);
        // w8^k, k = 0..3, with w8 = exp(sign 2 pi i/8)
        cx<T> w1 = cx<T>{r, T(sign) * r};
        cx<T> w3 = cx<T>{-r, T(sign) * r};
        cx<T> t0 = o[0];
        cx<T> t1 = cmul(o[1], w1);
        cx<T> t2 = cmul_si(o[2], sign);
        cx<T> t3 = cmul(o[3], w3);
        v[0] = cadd(e[0], t0);
        v[4] = csub(e[0], t0);
        v[1] = cadd(e[1], t1);
        v[5] = csub(e[1], t1);
        v[2] = cadd(e[2], t2);
        v[6] = csub(e[2], t2);
        v[3] = cadd(e[3], t3);
        v[7] = csub(e[3], t3);
    }
};

// One in-place Stockham pass of radix R (p = product of the radices already
// applied): every thread first reads the inputs of its butterflies into
// registers, then, after a barrier, writes the outputs.  CAP bounds batch * n
// and BLOCK the block size, so a thread holds at most ceil(CAP / (R * BLOCK))
// butterflies of radix R.  Element i of transform b lives at b * bs +
// fft_pad(i), or at b * bs + fft_pad(swz8(i)) where sin (inputs) or sout
// (outputs) is set.  tw: this pass's twiddle block (p > 1).
template <int R, typename T, int CAP, int BLOCK>
__device__ __forceinline__ void stockham_pass_ip(cx<T> *buf, int n, int p, int batch, int bs,
                                                 const cx<T> *tw, int sign, bool sin, bool sout)
{
    constexpr int MAXIT = (CAP / R + BLOCK - 1) / BLOCK;
    // the pass is selected at run time from the plan's radices: an empty asm
    // keeps the compiler from hoisting this radix's index set-up out of the
    // pass loop, where it would be computed for every radix of the switch
    int nn = n;
    asm volatile("" : "+s"(nn));
    const int m = nn / R;
    const int total = batch * m;
    const float inv_m = 1.0f / (float)m, inv_p = 1.0f / (float)p;
    cx<T> v[MAXIT][R];
    int out0[MAXIT];
#pragma unroll
    for (int q = 0; q < MAXIT; ++q) {
        const int it = threadIdx.x + q * BLOCK;
        out0[q] = -1;
        if (it < total) {
            const int b = div_small(it, m, inv_m);
            const int i = it - b * m;
            const int k = i - p * div_small(i, p, inv_p);
            const cx<T> *s = buf + b * bs;
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const int e = i + j * m;
                v[q][j] = s[fft_pad(sin ? swz8(e) : e)];
            }
            if (p > 1) {
#pragma unroll
                for (int j = 1; j < R; ++j) {
                    cx<T> w = tw[(j - 1) * p + k];
                    if (sign > 0) w.y = -w.y;
                    v[q][j] = cmul(v[q][j], w);
                }
            }
            Dft<R, T>::run(v[q], sign);
            out0[q] = (b << 16) | ((i - k) * R + k);   // transform, first output
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < MAXIT; ++q) {
        if (out0[q] >= 0) {
            const int o = out0[q] & 0xffff;
            cx<T> *d = buf + (out0[q] >> 16) * bs;
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const int e = o + j * p;
                d[fft_pad(sout ? swz8(e) : e)] = v[q][j];
            }
        }
    }
    __syncthreads();
}

// Copy of a twiddle table of n entries into LDS, in two steps so that the
// caller can issue it among its other loads: load() reads two entries per
// thread, unconditionally (a thread past the end reads the last entry),
// store() writes them to LDS (a thread past the end writes the last entry onto
// itself); entries beyond 2 * BLOCK are copied by a loop in store().  No branch
// holds a load and its wait.
template <typename T, int BLOCK>
struct TwiddleCopy {
    cx<T> v[2];
    __device__ __forceinline__ void load(const cx<T> *src, int n)
    {
#pragma unroll
        for (int q = 0; q < 2; ++q) v[q] = src[min((int)threadIdx.x + q * BLOCK, n - 1)];
    }
    __device__ __forceinline__ void store(cx<T> *dst, const cx<T> *src, int n) const
    {
#pragma unroll
        for (int q = 0; q < 2; ++q) dst[min((int)threadIdx.x + q * BLOCK, n - 1)] = v[q];
        for (int i = threadIdx.x + 2 * BLOCK; i < n; i += BLOCK) dst[i] = src[i];
    }
};

// Batched in-place transform: batch transforms of length pl.n, element i of
// transform b at buf[b * bs + fft_pad(i)] (bs >= fft_stride(n),
// batch * pl.n <= CAP, blockDim.x == BLOCK).  Ends with a barrier.
template <typename T, int CAP, int BLOCK>
__device__ void lds_fft_ip(cx<T> *buf, int batch, int bs, const FftPlanDev &pl,
                           const cx<T> *tw, int sign)
{
    int p = 1, toff = 0;
    for (int ps = 0; ps < pl.npass; ++ps) {
        const int R = pl.radix[ps];
        const cx<T> *twp = tw + toff;
        const bool sin = ps == 1 && pl.swz, sout = ps == 0 && pl.swz;
        switch (R) {
        case 2: stockham_pass_ip<2, T, CAP, BLOCK>(buf, pl.n, p, batch, bs, twp, sign, sin, sout); break;
        case 3: stockham_pass_ip<3, T, CAP, BLOCK>(buf, pl.n, p, batch, bs, twp, sign, sin, sout); break;
        case 4: stockham_pass_ip<4, T, CAP, BLOCK>(buf, pl.n, p, batch, bs, twp, sign, sin, sout); break;
        case 5: stockham_pass_ip<5, T, CAP, BLOCK>(buf, pl.n, p, batch, bs, twp, sign, sin, sout); break;
        default: stockham_pass_ip<8, T, CAP, BLOCK>(buf, pl.n, p, batch, bs, twp, sign, sin, sout); break;
        }
        if (p > 1) toff += p * (R - 1);
        p *= R;
    }
}

// ---------------------------------------------------------------------------
// The same transform with the length a compile-time constant N: the plan
// (radix_order below, the host's rule), the pass extents and the butterfly
// index arithmetic fold into constants (divisions by the pass extents become
// multiplications), and the direction is a constant too.  Used for the
// lengths of the workloads the library is tuned for; any other length takes
// lds_fft_ip.

// the radix plan of length n, as the host's radix_plan: 8s, 4s, a 2, 5s, 3s
constexpr int cplan_npass(int n)
{
    int k = 0, m = n, e2 = 0;
    while (m % 2 == 0) { ++e2; m /= 2; }
    while (e2 >= 3 && e2 != 4) { ++k; e2 -= 3; }
    while (e2 >= 2) { ++k; e2 -= 2; }
    if (e2 == 1) ++k;
    while (m % 5 == 0) { ++k; m /= 5; }
    while (m % 3 == 0) { ++k; m /= 3; }
    return k;
}
constexpr int cplan_radix(int n, int ps)
{
    int r[16] = {}, k = 0, m = n, e2 = 0;
    while (m % 2 == 0) { ++e2; m /= 2; }
    while (e2 >= 3 && e2 != 4) { r[k++] = 8; e2 -= 3; }
    while (e2 >= 2) { r[k++] = 4; e2 -= 2; }
    if (e2 == 1) r[k++] = 2;
    while (m % 5 == 0) { r[k++] = 5; m /= 5; }
    while (m % 3 == 0) { r[k++] = 3; m /= 3; }
    return r[ps];
}
constexpr bool cplan_swz(int n)
{
    return cplan_npass(n) > 1 && n % 8 == 0 && cplan_radix(n, 0) % 2 == 0;
}

template <int R, typename T, int N, int P, int CAP, int BLOCK, int SIGN, bool SIN, bool SOUT>
__device__ __forceinline__ void stockham_pass_n(cx<T> *buf, int batch, int bs, const cx<T> *tw)
{
    constexpr int M = N / R;
    constexpr int MAXIT = (CAP / R + BLOCK - 1) / BLOCK;
    const int total = batch * M;
    cx<T> v[MAXIT][R];
    int ob[MAXIT];   // (transform << 16) | first output, or -1
#pragma unroll
    for (int q = 0; q < MAXIT; ++q) {
        const int it = threadIdx.x + q * BLOCK;
        ob[q] = -1;
        if (it < total) {
            const int b = it / M;
            const int i = it - b * M;
            const int k = i % P;
            const cx<T> *s = buf + b * bs;
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const int e = i + j * M;
                v[q][j] = s[fft_pad(SIN ? swz8(e) : e)];
            }
            if (P > 1) {
#pragma unroll
                for (int j = 1; j < R; ++j) {
                    cx<T> w = tw[(j - 1) * P + k];
                    if (SIGN > 0) w.y = -w.y;
                    v[q][j] = cmul(v[q][j], w);
                }
            }
            Dft<R, T>::run(v[q], SIGN);
            ob[q] = (b << 16) | ((i - k) * R + k);   // transform, first output
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < MAXIT; ++q) {
        if (ob[q] >= 0) {
            const int o = ob[q] & 0xffff;
            cx<T> *d = buf + (ob[q] >> 16) * bs;
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const int e = o + j * P;
                d[fft_pad(SOUT ? swz8(e) : e)] = v[q][j];
            }
        }
    }
    __syncthreads();
}

template <typename T, int N, int CAP, int BLOCK, int SIGN, int PS, int P, int TOFF>
__device__ __forceinline__ void lds_fft_n_from(cx<T> *buf, int batch, int bs, const cx<T> *tw)
{
    if constexpr (PS < cplan_npass(N)) {
        constexpr int R = cplan_radix(N, PS);
        constexpr bool SW = cplan_swz(N);
        stockham_pass_n<R, T, N, P, CAP, BLOCK, SIGN, PS == 1 && SW, PS == 0 && SW>(buf, batch, bs,
                                                                                   tw + TOFF);
        lds_fft_n_from<T, N, CAP, BLOCK, SIGN, PS + 1, P * R, (P > 1 ? TOFF + P * (R - 1) : TOFF)>(
            buf, batch, bs, tw);
    }
}

// Batched in-place transform of length N (a constant), otherwise as
// lds_fft_ip with the plan of N.  Ends with a barrier.
template <typename T, int N, int CAP, int BLOCK, int SIGN>
__device__ __forceinline__ void lds_fft_n(cx<T> *buf, int batch, int bs, const cx<T> *tw)
{
    static_assert(N > 1 && N < 65536 && cplan_npass(N) <= 16, "transform length");
    lds_fft_n_from<T, N, CAP, BLOCK, SIGN, 0, 1, 0>(buf, batch, bs, tw);
}

// lds_fft_n when NF > 0, else lds_fft_ip with the run-time plan
template <typename T, int NF, int CAP, int BLOCK, int SIGN>
__device__ __forceinline__ void lds_fft(cx<T> *buf, int batch, int bs, const FftPlanDev &pl,
                                        const cx<T> *tw)
{
    if constexpr (NF > 0) lds_fft_n<T, NF, CAP, BLOCK, SIGN>(buf, batch, bs, tw);
    else lds_fft_ip<T, CAP, BLOCK>(buf, batch, bs, pl, tw, SIGN);
}

}  // namespace gke
