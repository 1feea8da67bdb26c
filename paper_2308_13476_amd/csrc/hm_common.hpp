// Device-side building blocks shared by the HIP kernels: complex arithmetic,
// the padded level layout and the block geometry.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace hm {

// Interleaved complex value; 16-byte (double) or 8-byte (float) aligned so a
// node is one vector load.
template <typename T>
struct alignas(2 * sizeof(T)) cplx {
    T re, im;
};

template <typename T>
__host__ __device__ __forceinline__ cplx<T> mk(T r, T i) { return cplx<T>{r, i}; }
template <typename T>
__device__ __forceinline__ cplx<T> operator+(cplx<T> a, cplx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cplx<T> operator-(cplx<T> a, cplx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cplx<T> operator*(cplx<T> a, cplx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cplx<T> operator*(T s, cplx<T> a) { return {s * a.re, s * a.im}; }
// a + b * c
template <typename T>
__device__ __forceinline__ cplx<T> cfma(cplx<T> a, cplx<T> b, cplx<T> c) {
    return {fma(b.re, c.re, fma(-b.im, c.im, a.re)), fma(b.re, c.im, fma(b.im, c.re, a.im))};
}
template <typename T>
__device__ __forceinline__ cplx<T> conj(cplx<T> a) { return {a.re, -a.im}; }
template <typename T>
__device__ __forceinline__ T norm2(cplx<T> a) { return a.re * a.re + a.im * a.im; }
// a / b
template <typename T>
__device__ __forceinline__ cplx<T> cdiv(cplx<T> a, cplx<T> b) {
    T d = T(1) / (b.re * b.re + b.im * b.im);
    return {(a.re * b.re + a.im * b.im) * d, (a.im * b.re - a.re * b.im) * d};
}
template <typename T, typename U>
__device__ __forceinline__ cplx<T> cast(cplx<U> a) { return {T(a.re), T(a.im)}; }

// Ghost frame of every level grid: zero-valued nodes around the domain so
// that stencils of radius <= 3 and the transfer masks (radius 2) read
// without branches: kGhost rows below and above, kGhost columns on the
// right and kGhostX on the left. kGhostX = 32 and a pitch that is a multiple
// of 32 values put node (0, j) at the start of a 128-byte line for every
// element size used (4-byte k^2 to 16-byte complex128), so the 64 nodes of a
// wavefront's row segment fill whole lines instead of straddling one more.
constexpr int kGhost = 4;
constexpr int kGhostX = 32;
constexpr int kPitchAlign = 32;

// One level of the hierarchy in the padded layout: node (i, j), 0 <= i, j <= n,
// lives at (j + kGhost) * pitch + (i + kGhostX) of a plane of `plane` values.
struct Grid {
    int n;          // intervals per side
    int pitch;      // values per padded row
    long long plane;  // values per padded plane
    __host__ __device__ __forceinline__ long long at(int i, int j) const {
        return (long long)(j + kGhost) * pitch + (i + kGhostX);
    }
};

// Blocks are 64 x 4 threads (one wavefront per row of 64 nodes); a block
// covers 64 columns and 4 * rows_per_thread rows of a level.
constexpr int kBX = 64;
constexpr int kBY = 4;      // short blocks (register-heavy stencils, small grids)
constexpr int kMaxBY = 16;  // tall blocks (light kernels on large grids)

// A level kernel launches at most kMaxPartialBlocks blocks per right-hand
// side; reductions keep up to 8 partial sums per block in each of two
// regions. Consumers reduce the partials themselves up to the runtime block
// cap; above it a one-block pass pre-reduces them first.
constexpr int kMaxPartialBlocks = 8192;
constexpr long long kPartStride = (long long)kMaxPartialBlocks * 8;  // doubles per (region, right-hand side)

// Boundary weight w of a grid line position (1/2 at both ends).
template <typename T>
__device__ __forceinline__ T line_w(int i, int n) { return (i == 0 || i == n) ? T(0.5) : T(1); }

}  // namespace hm
