// match.hip -- the rotational-matching head around the inverse transform:
// SO(3) coefficients of the correlation of two functions on the sphere, the
// vector-Jacobian product of that map, and the argmax of the real part of the
// correlation grid.  (Matching by correlation over rotations is the
// application that motivates fast SO(3) transforms in Sect. 1.)
//
// Layouts: a function on the sphere is B^2 complex coefficients, (l, m) at
// l^2 + m + l; SO(3) coefficients use the plan layout
// l(4l^2-1)/3 + (M+l)(2l+1) + (M'+l).  Every kernel is HBM-bound: one pass
// over its output (coefficients), or over its input (the grid, argmax).
#include "soft_internal.h"

namespace soft {
namespace {

template <typename C>
__device__ __forceinline__ C cmul_conj(C a, C b) {  // a * conj(b)
    C r;
    r.x = a.x * b.x + a.y * b.y;
    r.y = a.y * b.x - a.x * b.y;
    return r;
}

__device__ __forceinline__ long long deg_offset(long long l) { return l * (4 * l * l - 1) / 3; }

// Degree of spherical-harmonic entry q: the l with l^2 <= q < (l+1)^2.
__device__ __forceinline__ int sh_degree(int q) {
    int l = (int)sqrt((double)q);
    if ((l + 1) * (l + 1) <= q) ++l;
    if (l * l > q) --l;
    return l;
}

// f°(l, M, M') = a(l, M) conj(b(l, M')); block (l', f) writes the
// (2l+1)^2 contiguous coefficients of degree l = B-1-l' of pair f (largest
// degrees first): a(l, .) and b(l, .) are staged in LDS (2l+1 <= 1023
// values each), then each wave writes whole rows M, its lanes on
// neighbouring M', so every store is part of a contiguous run.
template <typename C>
__global__ __launch_bounds__(256) void k_corr_coeffs(int B, const C *__restrict__ a, const C *__restrict__ b,
                                                     C *__restrict__ out) {
    __shared__ C sa[1024], sb[1024];
    const int l = B - 1 - (int)blockIdx.x, f = blockIdx.y;
    const int w = 2 * l + 1;
    const C *al = a + (long long)f * B * B + (long long)l * l;
    const C *bl = b + (long long)f * B * B + (long long)l * l;
    C *o = out + (long long)f * deg_offset(B) + deg_offset(l);
    for (int t = threadIdx.x; t < w; t += 256) {
        sa[t] = al[t];
        sb[t] = bl[t];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int row = wave; row < w; row += 4) {
        const C x = sa[row];
        C *orow = o + (long long)row * w;
        for (int c = lane; c < w; c += 64) orow[c] = cmul_conj(x, sb[c]);
    }
}

// Vector-Jacobian product, gradient of a: ga(l, M) = sum_M' g(l, M, M') b(l, M').
// One wave per (function, l, M) row; lanes stride over M' and reduce.
template <typename C>
__global__ __launch_bounds__(256) void k_corr_vjp_a(int B, int n, const C *__restrict__ b, const C *__restrict__ g,
                                                    C *__restrict__ ga) {
    const long long rows = (long long)n * B * B;
    const long long rw = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (rw >= rows) return;
    const long long f = rw / ((long long)B * B);
    const int q = (int)(rw - f * B * B);
    const int l = sh_degree(q);
    const int w = 2 * l + 1, row = q - l * l;
    const C *grow = g + f * deg_offset(B) + deg_offset(l) + (long long)row * w;
    const C *bl = b + f * (long long)B * B + (long long)l * l;
    double sr = 0.0, si = 0.0;
    for (int c = lane; c < w; c += 64) {
        const C x = grow[c], y = bl[c];
        sr += (double)x.x * y.x - (double)x.y * y.y;
        si += (double)x.x * y.y + (double)x.y * y.x;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        sr += __shfl_xor(sr, o);
        si += __shfl_xor(si, o);
    }
    if (lane == 0) {
        C r;
        r.x = (decltype(r.x))sr;
        r.y = (decltype(r.y))si;
        ga[rw] = r;
    }
}

// Gradient of b: gb(l, M') = sum_M conj(g(l, M, M')) a(l, M); one thread per
// (function, l, M') column (neighbouring threads read neighbouring M').
template <typename C>
__global__ __launch_bounds__(256) void k_corr_vjp_b(int B, int n, const C *__restrict__ a, const C *__restrict__ g,
                                                    C *__restrict__ gb) {
    const long long cols = (long long)n * B * B;
    const long long cl = (long long)blockIdx.x * 256 + threadIdx.x;
    if (cl >= cols) return;
    const long long f = cl / ((long long)B * B);
    const int q = (int)(cl - f * B * B);
    const int l = sh_degree(q);
    const int w = 2 * l + 1, col = q - l * l;
    const C *gl = g + f * deg_offset(B) + deg_offset(l) + col;
    const C *al = a + f * (long long)B * B + (long long)l * l;
    double sr = 0.0, si = 0.0;
    for (int r = 0; r < w; ++r) {
        const C x = gl[(long long)r * w], y = al[r];
        sr += (double)x.x * y.x + (double)x.y * y.y;  // conj(x) * y
        si += (double)x.x * y.y - (double)x.y * y.x;
    }
    C r;
    r.x = (decltype(r.x))sr;
    r.y = (decltype(r.y))si;
    gb[cl] = r;
}

__device__ ArgBest block_best(ArgBest b) {
    __shared__ double sv[4];
    __shared__ long long si[4];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        ArgBest q;
        q.v = __shfl_xor(b.v, o);
        q.i = __shfl_xor(b.i, o);
        b = arg_better(b, q);
    }
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sv[wave] = b.v;
        si[wave] = b.i;
    }
    __syncthreads();
    ArgBest r{sv[0], si[0]};
#pragma unroll
    for (int w = 1; w < 4; ++w) r = arg_better(r, ArgBest{sv[w], si[w]});
    return r;
}

// Stage 1: block (c, f) scans chunk c of grid f (elements [c*chunk,
// (c+1)*chunk) of count) and writes its best (Re, index) to part[f*nblk + c].
template <typename C>
__global__ __launch_bounds__(256) void k_argmax_part(const C *__restrict__ x, long long count, long long chunk,
                                                     int nblk, ArgBest *__restrict__ part) {
    const int c = blockIdx.x, f = blockIdx.y;
    const long long lo = (long long)c * chunk;
    const long long hi = lo + chunk < count ? lo + chunk : count;
    const C *xf = x + (long long)f * count;
    ArgBest b{-__builtin_huge_val(), kNoIndex};
    long long i = lo + threadIdx.x;
    for (; i + 3 * 256 < hi; i += 4 * 256) {
        C v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = xf[i + u * 256];
#pragma unroll
        for (int u = 0; u < 4; ++u) b = arg_better(b, ArgBest{(double)v[u].x, i + u * 256});
    }
    for (; i < hi; i += 256) b = arg_better(b, ArgBest{(double)xf[i].x, i});
    b = block_best(b);
    if (threadIdx.x == 0) part[(long long)f * nblk + c] = b;
}

// Stage 2: one block per grid reduces its nblk partial results.
__global__ __launch_bounds__(256) void k_argmax_final(const ArgBest *__restrict__ part, int nblk,
                                                      long long *__restrict__ index) {
    const int f = blockIdx.x;
    ArgBest b{-__builtin_huge_val(), kNoIndex};
    for (int c = threadIdx.x; c < nblk; c += 256) b = arg_better(b, part[(long long)f * nblk + c]);
    b = block_best(b);
    if (threadIdx.x == 0) index[f] = b.i == kNoIndex ? -1 : b.i;
}

}  // namespace

template <typename C>
hipError_t launch_corr_coeffs(int B, int n, const C *a, const C *b, C *coeffs, hipStream_t s) {
    if (n > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_corr_coeffs<C>, dim3(B, n), dim3(256), 0, s, B, a, b, coeffs);
    return hipGetLastError();
}

template <typename C>
hipError_t launch_corr_vjp(int B, int n, const C *a, const C *b, const C *g, C *ga, C *gb, hipStream_t s) {
    const long long rows = (long long)n * B * B;
    hipLaunchKernelGGL(k_corr_vjp_a<C>, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, s, B, n, b, g, ga);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_corr_vjp_b<C>, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s, B, n, a, g, gb);
    return hipGetLastError();
}

int argmax_blocks(long long count, int n) {
    // about 4096 blocks over all grids, each scanning at least 16K elements
    long long nb = 4096 / (n > 0 ? n : 1);
    const long long by_size = (count + 16383) / 16384;
    if (nb > by_size) nb = by_size;
    if (nb < 1) nb = 1;
    return (int)nb;
}

size_t argmax_workspace_bytes(long long count, int n) {
    return sizeof(ArgBest) * (size_t)argmax_blocks(count, n) * (size_t)n;
}

template <typename C>
hipError_t launch_argmax_real(const C *x, long long count, int n, void *workspace, long long *index, hipStream_t s) {
    const int nblk = argmax_blocks(count, n);
    const long long chunk = (count + nblk - 1) / nblk;
    ArgBest *part = static_cast<ArgBest *>(workspace);
    hipLaunchKernelGGL(k_argmax_part<C>, dim3(nblk, n), dim3(256), 0, s, x, count, chunk, nblk, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_argmax_final, dim3(n), dim3(256), 0, s, part, nblk, index);
    return hipGetLastError();
}

hipError_t launch_argmax_final(const ArgBest *part, int nblk, int n, long long *index, hipStream_t s) {
    if (n < 1 || nblk < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_argmax_final, dim3(n), dim3(256), 0, s, part, nblk, index);
    return hipGetLastError();
}

#define SOFT_MATCH_INSTANTIATE(C)                                                                            \
    template hipError_t launch_corr_coeffs<C>(int, int, const C *, const C *, C *, hipStream_t);            \
    template hipError_t launch_corr_vjp<C>(int, int, const C *, const C *, const C *, C *, C *, hipStream_t); \
    template hipError_t launch_argmax_real<C>(const C *, long long, int, void *, long long *, hipStream_t);
SOFT_MATCH_INSTANTIATE(double2)
SOFT_MATCH_INSTANTIATE(float2)

}  // namespace soft
