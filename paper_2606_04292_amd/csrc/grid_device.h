// Index and launch-shape helpers shared by the FP64 and FP32 kernels.
#pragma once

#include "rs_internal.h"
#include "soil_device.h"

namespace rs {

constexpr int kBX = 64;
constexpr int kBY = 4;

// Maximum over a work-group (NaN wins); the result is valid in thread 0.
__device__ __forceinline__ double block_max(double v)
{
    __shared__ double red[8];
    int lane = threadIdx.x + threadIdx.y * blockDim.x;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        double o = __shfl_xor(v, off);
        v = (o > v || o != o) ? o : v;
    }
    int wave = lane >> 6;
    if ((lane & 63) == 0) red[wave] = v;
    __syncthreads();
    int nw = (blockDim.x * blockDim.y + 63) >> 6;
    if (lane == 0) {
        double m = red[0];
        for (int w = 1; w < nw; ++w) m = (red[w] > m || red[w] != red[w]) ? red[w] : m;
        v = m;
    }
    return v;
}

// Work-groups are dispatched round-robin over the 8 XCDs; renumber them so that
// XCD x runs the contiguous logical range [x per, (x+1) per) and its L2 sees a
// compact slab of the grid (neighbouring rows and planes hit in L2).  The grid
// is padded to a multiple of 8; padded groups fall past the last cell.
__device__ __forceinline__ unsigned xcd_block(unsigned per)
{
    return (blockIdx.x % 8u) * per + blockIdx.x / 8u;
}

// The same, with each XCD walking its slab from the far end when reverse is
// set: a pass that follows another in the opposite direction starts on the
// lines the previous one touched last, which are still in the memory-side
// cache.
__device__ __forceinline__ unsigned xcd_block_dir(unsigned per, bool reverse)
{
    const unsigned pos = blockIdx.x / 8u;
    return (blockIdx.x % 8u) * per + (reverse ? per - 1u - pos : pos);
}

inline unsigned xcd_grid(unsigned long long blocks) { return (unsigned)((blocks + 7) / 8 * 8); }

// Packed enumeration of the cells of one colour: rows (fixed j, k) of
// H = (n0 + 1) / 2 slots, slot ih -> i = 2 ih + parity; every lane of a wave
// holds a cell (only the last slot of odd-parity rows falls outside).
struct ColourMap {
    unsigned long long total;
    unsigned H;
    FastDiv dH;
    unsigned n1;
    FastDiv dN1;
};

inline ColourMap colour_map(const Geo &g)
{
    ColourMap m;
    m.H = (unsigned)((g.n[0] + 1) / 2);
    m.dH = make_fastdiv(m.H);
    m.n1 = (unsigned)g.n[1];
    m.dN1 = make_fastdiv(m.n1);
    m.total = (unsigned long long)m.H * g.n[1] * g.n[2];
    return m;
}

// Slots of the pair kernels of a level with parity-split rows: xh per row
// (position m of the even half, with the even node after it and the odd
// node between them), rows over axes 1 and 2.
inline ColourMap pair_map(const Geo &g)
{
    ColourMap m;
    m.H = (unsigned)g.xh;
    m.dH = make_fastdiv(m.H);
    m.n1 = (unsigned)g.n[1];
    m.dN1 = make_fastdiv(m.n1);
    m.total = (unsigned long long)m.H * g.n[1] * g.n[2];
    return m;
}

// Memory position of node i within its row (see Geo::xs): i itself, or with
// the row split by parity (i >> 1) + (i & 1) xh.  Defined for i = -1 and
// i = n0 too (a row's neighbouring value, or the padding around an array).
__host__ __device__ __forceinline__ long long xpos(const Geo &g, int i)
{
    return (long long)((i >> g.xs) + (i & 1) * g.xh);
}

// Memory index of node (i, j, k) of a level.
__host__ __device__ __forceinline__ long long lin(const Geo &g, int i, int j, int k)
{
    return xpos(g, i) + (long long)j * g.stride[1] + (long long)k * g.stride[2];
}

// Index of the axis-0 neighbour i + side of node i stored at idx.
__device__ __forceinline__ long long xnb(const Geo &g, int i, long long idx, int side)
{
    return idx - xpos(g, i) + xpos(g, i + side);
}

// Visit the neighbours of node (i, j, k) along the first DIM axes in the
// order axis 0 low/high, axis 1 low/high, axis 2 low/high; fn(jdx, coef, axis,
// side) with coef = 1/(2 w h^2).
template <int DIM, typename Fn>
__device__ __forceinline__ void for_nb(const Geo &g, int i, int j, int k, long long idx, Fn &&fn)
{
#pragma unroll
    for (int l = 0; l < DIM; ++l) {
        const int cl = (l == 0) ? i : (l == 1 ? j : k);
        const double cf = ((cl == 0 || cl == g.n[l] - 1) ? 1.0 : 0.5) * g.ih2[l];
        const long long s = g.stride[l];
        if (cl > 0) fn(l == 0 ? xnb(g, i, idx, -1) : idx - s, cf, l, -1);
        if (cl < g.n[l] - 1) fn(l == 0 ? xnb(g, i, idx, 1) : idx + s, cf, l, +1);
    }
}

// Visit the existing neighbours of node c, runtime dimension (order: axis 0 low/high, axis 1,
// axis 2), calling fn(jdx, coef, axis, side) with coef = 1/(2 w h^2).
template <typename Fn>
__device__ __forceinline__ void for_each_nb(const Geo &g, const int c[3], long long idx, Fn &&fn)
{
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        if (l >= g.dim) break;
        double iw = (c[l] == 0 || c[l] == g.n[l] - 1) ? 2.0 : 1.0;
        double cf = 0.5 * iw * g.ih2[l];
        if (c[l] > 0) fn(l == 0 ? xnb(g, c[0], idx, -1) : idx - g.stride[l], cf, l, -1);
        if (c[l] < g.n[l] - 1) fn(l == 0 ? xnb(g, c[0], idx, 1) : idx + g.stride[l], cf, l, +1);
    }
}

// The 2 DIM neighbours of node (i, j, k) in the order of for_nb, as indices
// and coefficients 1/(2 w h^2).  A neighbour outside the domain gets the node
// itself as index and a zero coefficient, so every load of a stencil can be
// issued before any arithmetic (no branch per neighbour) and the zero terms
// leave the sums unchanged.  XPAD (arrays with finite padding around them, as
// in a grid workspace): the axis-0 neighbours are always the positions of
// i -/+ 1 (another value of the row, the neighbouring row's first value, or
// the padding, when outside the domain, still with a zero coefficient), so the
// loads of a row need no branch.
template <int DIM>
struct Stencil {
    long long jn[2 * DIM];
    double cf[2 * DIM];
};

template <int DIM, bool XPAD = false>
__device__ __forceinline__ Stencil<DIM> stencil(const Geo &g, int i, int j, int k, long long idx)
{
    Stencil<DIM> s;
#pragma unroll
    for (int l = 0; l < DIM; ++l) {
        const int cl = (l == 0) ? i : (l == 1 ? j : k);
        const double cf = ((cl == 0 || cl == g.n[l] - 1) ? 1.0 : 0.5) * g.ih2[l];
        const bool lo = cl > 0, hi = cl < g.n[l] - 1;
        const bool xp = XPAD && l == 0;
        const long long dn = l == 0 ? xnb(g, i, idx, -1) : idx - g.stride[l];
        const long long up = l == 0 ? xnb(g, i, idx, 1) : idx + g.stride[l];
        s.jn[2 * l] = (lo || xp) ? dn : idx;
        s.cf[2 * l] = lo ? cf : 0.0;
        s.jn[2 * l + 1] = (hi || xp) ? up : idx;
        s.cf[2 * l + 1] = hi ? cf : 0.0;
    }
    return s;
}

// Two adjacent values of an array as one access: 16-byte (8-byte for floats)
// global loads need only dword alignment, so any pair of neighbouring
// positions can be loaded together.
typedef double double2_u __attribute__((ext_vector_type(2), aligned(8)));
typedef float float2_u __attribute__((ext_vector_type(2), aligned(4)));
template <typename T> struct PairOf;
template <> struct PairOf<double> { typedef double2_u type; };
template <> struct PairOf<float> { typedef float2_u type; };

template <typename T>
__device__ __forceinline__ typename PairOf<T>::type load_pair(const T *p)
{
    return *(const typename PairOf<T>::type *)p;
}

template <typename T>
__device__ __forceinline__ void store_pair(T *p, T a, T b)
{
    typename PairOf<T>::type v;
    v.x = a;
    v.y = b;
    *(typename PairOf<T>::type *)p = v;
}

// Stencil of node (i, j, k) stored at idx on a level with parity-split rows
// (Geo::xs = 1, as in every level of a grid): the axis-0 neighbours i - 1 and
// i + 1 sit side by side in the other half of the row, at xl and xl + 1
// (xl = idx - xpos(i) + xpos(i - 1); at the ends of the row one of them is
// another value of the row, or the next row's first value, with coefficient
// 0).  Off-row neighbours as in stencil().
template <int DIM>
__device__ __forceinline__ Stencil<DIM> stencil_split(const Geo &g, int i, int j, int k,
                                                      long long idx, long long xl)
{
    Stencil<DIM> s;
    {
        const double cf = ((i == 0 || i == g.n[0] - 1) ? 1.0 : 0.5) * g.ih2[0];
        s.jn[0] = xl;
        s.cf[0] = i > 0 ? cf : 0.0;
        s.jn[1] = xl + 1;
        s.cf[1] = i < g.n[0] - 1 ? cf : 0.0;
    }
#pragma unroll
    for (int l = 1; l < DIM; ++l) {
        const int cl = l == 1 ? j : k;
        const double cf = ((cl == 0 || cl == g.n[l] - 1) ? 1.0 : 0.5) * g.ih2[l];
        const bool lo = cl > 0, hi = cl < g.n[l] - 1;
        s.jn[2 * l] = lo ? idx - g.stride[l] : idx;
        s.cf[2 * l] = lo ? cf : 0.0;
        s.jn[2 * l + 1] = hi ? idx + g.stride[l] : idx;
        s.cf[2 * l + 1] = hi ? cf : 0.0;
    }
    return s;
}

// Raw buffer access to one array of a level (arrays of < 2 GiB): 32-bit byte
// offsets from a base held in scalar registers, so a stencil's addresses cost
// one 32-bit add each; an offset outside [0, bytes) reads 0.
typedef int v2i32 __attribute__((ext_vector_type(2)));
typedef int v4i32 __attribute__((ext_vector_type(4)));
typedef double v2f64 __attribute__((ext_vector_type(2)));
typedef float v2f32 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void *p, long long bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes,
                                             0x00020000);
}

template <typename T> __device__ __forceinline__ T buf_ld(__amdgpu_buffer_rsrc_t r, int off);
template <> __device__ __forceinline__ double buf_ld<double>(__amdgpu_buffer_rsrc_t r, int off)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
template <> __device__ __forceinline__ float buf_ld<float>(__amdgpu_buffer_rsrc_t r, int off)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

// Two adjacent values at byte offset off (dword alignment suffices).
__device__ __forceinline__ v2f64 buf_ld2(__amdgpu_buffer_rsrc_t r, int off, double)
{
    return __builtin_bit_cast(v2f64, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}
__device__ __forceinline__ v2f32 buf_ld2(__amdgpu_buffer_rsrc_t r, int off, float)
{
    return __builtin_bit_cast(v2f32, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}

__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, int off, double v)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2i32, v), r, off, 0, 0);
}
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, int off, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, v), r, off, 0, 0);
}
// Two adjacent values at byte offset off (dword alignment suffices).
__device__ __forceinline__ void buf_st2(__amdgpu_buffer_rsrc_t r, int off, double a, double b)
{
    const v2f64 v = {a, b};
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(v4i32, v), r, off, 0, 0);
}

// Levels whose arrays (with their padding) stay below 2 GiB take the buffer
// paths of the sweeps.
inline bool buffer_ok(const Geo &g, size_t elem)
{
    return (unsigned long long)(g.N + 64) * elem < (1ull << 31);
}

struct NodeMap {
    unsigned n0, n1;
    FastDiv d0, d1;
    int xh;          // Geo::xh (0: lexicographic rows)
};

inline NodeMap node_map(const Geo &g)
{
    NodeMap m;
    m.n0 = (unsigned)g.n[0];
    m.n1 = (unsigned)g.n[1];
    m.d0 = make_fastdiv(m.n0);
    m.d1 = make_fastdiv(m.n1);
    m.xh = g.xh;
    return m;
}

// (i, j, k) of the node stored at index t of a level (t < 2^31): threads that
// walk t walk memory in order, whatever the row layout.
__device__ __forceinline__ void node_ijk(const NodeMap &nm, unsigned long long t, int &i, int &j,
                                         int &k)
{
    const unsigned row = udiv((unsigned)t, nm.d0);
    const int p = (int)(t - (unsigned long long)row * nm.n0);
    i = nm.xh == 0 ? p : (p < nm.xh ? 2 * p : 2 * (p - nm.xh) + 1);
    k = (int)udiv(row, nm.d1);
    j = (int)row - k * (int)nm.n1;
}

// (i, j, k) of colour slot t (false for the padding slot of a row).
__device__ __forceinline__ bool colour_ijk(const Geo &g, const ColourMap &cm,
                                           unsigned long long t, int colour, int &i, int &j,
                                           int &k)
{
    if (t >= cm.total) return false;
    const unsigned row = udiv((unsigned)t, cm.dH);
    const unsigned ih = (unsigned)(t - (unsigned long long)row * cm.H);
    k = (int)udiv(row, cm.dN1);
    j = (int)row - k * (int)cm.n1;
    i = 2 * (int)ih + ((j + k + colour) & 1);
    return i < g.n[0];
}

// Colour slots and node order of a level of the one-work-group cycle.
__device__ __forceinline__ ColourMap tail_cm(const TailLevel &T)
{
    ColourMap m;
    m.total = (unsigned long long)T.cm_total;
    m.H = T.H;
    m.dH = FastDiv{T.dH_m, T.dH_s};
    m.n1 = T.n1;
    m.dN1 = FastDiv{T.dN1_m, T.dN1_s};
    return m;
}

__device__ __forceinline__ NodeMap tail_nm(const TailLevel &T)
{
    NodeMap m;
    m.n0 = T.n0;
    m.n1 = T.nn1;
    m.d0 = FastDiv{T.d0_m, T.d0_s};
    m.d1 = FastDiv{T.d1_m, T.d1_s};
    m.xh = T.g.xh;
    return m;
}

inline dim3 node_grid(const Geo &g)
{
    return dim3((g.n[0] + kBX - 1) / kBX, (g.n[1] + kBY - 1) / kBY, g.n[2]);
}


// Call fn.template operator()<MODEL, SINK, DIM>() for the law and level.
// EXT: also the Gardner law and per-node soils (FP64 kernels only).
template <bool EXT = false, typename Fn>
inline void dispatch(const Law &law, int dim, Fn &&fn)
{
    const bool s = law.sink == kSinkFeddes;
#define RS_DIMS(M, S)                                   \
    do {                                                \
        if (dim == 1) fn.template go<M, S, 1>();        \
        else if (dim == 2) fn.template go<M, S, 2>();   \
        else fn.template go<M, S, 3>();                 \
    } while (0)
    if constexpr (EXT) {
        if (law.model == kGardner) {
            if (s) RS_DIMS(kGardner, true); else RS_DIMS(kGardner, false);
            return;
        }
        if (law.model == kMulti) {
            if (s) RS_DIMS(kMulti, true); else RS_DIMS(kMulti, false);
            return;
        }
    }
    if (law.model == kHaverkamp) {
        if (s) RS_DIMS(kHaverkamp, true); else RS_DIMS(kHaverkamp, false);
    } else if (law.model == kVgm) {
        if (s) RS_DIMS(kVgm, true); else RS_DIMS(kVgm, false);
    } else {
        if (s) RS_DIMS(kLinear, true); else RS_DIMS(kLinear, false);
    }
#undef RS_DIMS
}

}  // namespace rs
