// Device code of liblilac.so for gfx950 (CDNA4, wave64): CSR analysis and
// the layout builds, the CSR product in its four storage layouts (row-class
// tiles with the split-row finaliser, column panels, hot columns, band) and
// their grouped launches, dot products, the conjugate-gradient vector
// kernels (single and batched), PageRank relabelling, JDS and BFS.
//
// Every reduction here has a fixed shape (lane groups reduce with DPP moves
// in a fixed pattern, segmented scans run over lanes in order, workgroups
// combine their wavefronts in index order, split rows add their chunk sums
// in chunk order, carries between wavefronts are added in slot order, and a
// row sum held in LDS takes its additions from the one wavefront that owns
// the row, whose LDS operations complete in program order), so a given
// matrix, layout and plan always give bitwise identical results, whatever
// else runs on the GPU.
#include <algorithm>
#include <type_traits>

#include "lilac_internal.h"

namespace lilac {
namespace {

// Streaming loads for data read exactly once per product (vals, col_idx):
// non-temporal, so they do not push the gathered vector out of the caches.
template <typename T>
__device__ __forceinline__ T ld_stream(const T *p)
{
    return __builtin_nontemporal_load((const __attribute__((address_space(1))) T *)p);
}

// Loads and stores of device memory through a global (address space 1)
// pointer.  Pointers read from a descriptor table (grouped launches) are
// otherwise generic to the compiler, which then emits flat instructions;
// those also count against the LDS wait counter and so stall LDS work.
template <typename T>
__device__ __forceinline__ T gld(const T *p)
{
    return *(const __attribute__((address_space(1))) T *)p;
}

template <typename T>
__device__ __forceinline__ void gst(T *p, T v)
{
    *(__attribute__((address_space(1))) T *)p = v;
}

// Set bits of a wavefront mask in the lanes below this one.
__device__ __forceinline__ int32_t lanes_below(uint64_t m)
{
    return (int32_t)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                              __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ int32_t wave_sum_i32(int32_t v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

// Cross-lane move of a double with a DPP pattern (two 32-bit halves); a
// lane with no source lane gets 0 (bound_ctrl), so no old value has to be
// set up first.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    const int lo = __double2loint(v);
    const int hi = __double2hiint(v);
    return __hiloint2double(__builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, true),
                            __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, true));
}

// The same for a 32-bit integer.
template <int CTRL>
__device__ __forceinline__ int32_t dpp_i32z(int32_t v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}

// DPP move with a row mask; lanes of masked rows (or with no source) get
// `old`.
template <int CTRL, int ROWS>
__device__ __forceinline__ int32_t dpp_i32(int32_t v, int32_t old)
{
    return __builtin_amdgcn_update_dpp(old, v, CTRL, ROWS, 0xF, false);
}

template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64m(double v, double old)
{
    return __hiloint2double(
        __builtin_amdgcn_update_dpp(__double2hiint(old), __double2hiint(v), CTRL, ROWS, 0xF, false),
        __builtin_amdgcn_update_dpp(__double2loint(old), __double2loint(v), CTRL, ROWS, 0xF, false));
}

// One step of a segmented inclusive scan over a wavefront whose keys
// ascend along the lanes: add the partial of the source lane when it has
// the same key (monotone keys: the whole span between has that key).
// Shifts inside rows (all rows enabled) read 0 and key 0 where there is no
// source lane: a false key match then adds 0.  Broadcasts into some rows
// keep the lane's own key -1 / value 0 in the other rows.
// MASKED: the addition runs under an execution mask (the empty asm keeps
// the compiler from turning it into a select), one vector instruction
// instead of an addition and two 32-bit selects; it pays in the
// column-panel product, whose instruction stream bounds it.
template <int CTRL, int ROWS, bool MASKED = false>
__device__ __forceinline__ void seg_step(double &val, int32_t key)
{
    double t;
    int32_t tk;
    if (ROWS == 0xF) {
        t = dpp_f64<CTRL>(val);
        tk = dpp_i32z<CTRL>(key);
    } else {
        t = dpp_f64m<CTRL, ROWS>(val, 0.0);
        tk = dpp_i32<CTRL, ROWS>(key, -1);
    }
    if (tk == key) {
        val += t;
        if (MASKED)
            __asm__ volatile("" : "+v"(val));
    }
}

// acc += v on a double in LDS, no value returned (ds_add_f64: the wave
// does not wait for it).
__device__ __forceinline__ void lds_add_f64(double *acc, double v)
{
    (void)__hip_atomic_fetch_add(acc, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Segmented inclusive scan by key over the 64 lanes (keys ascending): row
// shifts by 1, 2, 4, 8 inside each row of 16, then the last lane of row 0
// (and of row 2) into rows 1 (and 3), then lane 31 into rows 2 and 3.
template <bool MASKED = false>
__device__ __forceinline__ double seg_scan64(double val, int32_t key)
{
    seg_step<0x111, 0xF, MASKED>(val, key);  // row_shr:1
    seg_step<0x112, 0xF, MASKED>(val, key);  // row_shr:2
    seg_step<0x114, 0xF, MASKED>(val, key);  // row_shr:4
    seg_step<0x118, 0xF, MASKED>(val, key);  // row_shr:8
    seg_step<0x142, 0xA, MASKED>(val, key);  // row_bcast:15 into rows 1 and 3
    seg_step<0x143, 0xC, MASKED>(val, key);  // row_bcast:31 into rows 2 and 3
    return val;
}

// Key of the next lane (wave_shl:1); the last lane gets -1.
__device__ __forceinline__ int32_t next_lane_key(int32_t key)
{
    return __builtin_amdgcn_update_dpp(-1, key, 0x130, 0xF, 0xF, false);
}

__device__ __forceinline__ double readlane_f64(double v, int lane)
{
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                            __builtin_amdgcn_readlane(__double2loint(v), lane));
}

// Sum over aligned groups of W lanes (W a power of two <= 64).  Inside a
// row of 16 lanes: neighbours (quad_perm 1,0,3,2), pairs (2,3,0,1), then the
// half-row and row mirrors, each adding the partner's partial; across rows
// the four row sums are read as uniform values and added in lane order.
// All lanes of a group end with the same value (x + y == y + x bitwise).
template <int W>
__device__ __forceinline__ double lane_group_sum(double v)
{
    if (W >= 2)
        v += dpp_f64<0xB1>(v);
    if (W >= 4)
        v += dpp_f64<0x4E>(v);
    if (W >= 8)
        v += dpp_f64<0x141>(v);
    if (W >= 16)
        v += dpp_f64<0x140>(v);
    if (W >= 32) {
        const double r0 = readlane_f64(v, 0), r1 = readlane_f64(v, 16);
        const double r2 = readlane_f64(v, 32), r3 = readlane_f64(v, 48);
        if (W == 32)
            v = (threadIdx.x & 32) ? r2 + r3 : r0 + r1;
        else
            v = (r0 + r1) + (r2 + r3);
    }
    return v;
}

template <int W>
__device__ __forceinline__ int32_t lane_group_or(int32_t v)
{
#pragma unroll
    for (int off = W / 2; off >= 1; off >>= 1)
        v |= __shfl_xor(v, off, 64);
    return v;
}

template <int W>
__device__ __forceinline__ int32_t lane_group_max(int32_t v)
{
#pragma unroll
    for (int off = W / 2; off >= 1; off >>= 1)
        v = max(v, __shfl_xor(v, off, 64));
    return v;
}

// Sum over a workgroup of NW wavefronts; every thread must call it and every
// thread receives the total.  lds holds NW doubles.
template <int NW>
__device__ __forceinline__ double block_sum(double v, double *lds)
{
    v = lane_group_sum<64>(v);
    __syncthreads();  // earlier readers of lds are done
    if ((threadIdx.x & 63) == 0)
        lds[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = lds[0];
#pragma unroll
    for (int i = 1; i < NW; ++i)
        t += lds[i];
    return t;
}

typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef int32_t i32x2 __attribute__((ext_vector_type(2)));
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));

// VEC consecutive values / column indices in one 16-byte (8-byte for the
// float64 indices) streaming load.  `p` is VEC-element aligned.
template <typename V, int VEC> struct Lanes;
template <typename V> struct Lanes<V, 1> {
    V v[1];
    int32_t c[1];
    __device__ __forceinline__ void load(const V *vp, const int32_t *cp)
    {
        v[0] = ld_stream(vp);
        c[0] = ld_stream(cp);
    }
};
template <> struct Lanes<double, 2> {
    double v[2];
    int32_t c[2];
    __device__ __forceinline__ void load(const double *vp, const int32_t *cp)
    {
        const f64x2 a = ld_stream((const f64x2 *)vp);
        const i32x2 b = ld_stream((const i32x2 *)cp);
        v[0] = a.x;
        v[1] = a.y;
        c[0] = b.x;
        c[1] = b.y;
    }
};
template <> struct Lanes<float, 4> {
    float v[4];
    int32_t c[4];
    __device__ __forceinline__ void load(const float *vp, const int32_t *cp)
    {
        const f32x4 a = ld_stream((const f32x4 *)vp);
        const i32x4 b = ld_stream((const i32x4 *)cp);
        v[0] = a.x;
        v[1] = a.y;
        v[2] = a.z;
        v[3] = a.w;
        c[0] = b.x;
        c[1] = b.y;
        c[2] = b.z;
        c[3] = b.w;
    }
};

// One lane's share of sum_{k in [k0,k1)} vals[k] * x[col[k]] when W lanes
// split the range.  The range is walked in passes over an aligned window
// starting at k0 rounded down to VEC: in a pass, lane l loads the VEC-element
// vectors at base + (j*W + l)*VEC for j < U, all issued before any is used
// (so U*VEC elements per lane are in flight), then gathers x for the
// elements that belong to the row.  Elements of a loaded vector outside
// [k0, k1) belong to neighbouring rows (or the array padding) and are
// skipped.  Products are formed and accumulated in binary64 (float32 data is
// widened exactly), in the order j, then element within the vector.
template <typename V, int W, int VEC, int U>
__device__ __forceinline__ double row_partial(const int32_t *__restrict__ col,
                                              const V *__restrict__ vals,
                                              const V *__restrict__ x,
                                              int32_t k0, int32_t k1, int lane)
{
    double acc = 0.0;
    const int32_t kb = k0 & ~(VEC - 1);
    for (int32_t base = kb; base < k1; base += U * W * VEC) {
        // every load is issued unconditionally (vectors past the row end
        // re-read the first one), so all U loads are in flight together
        Lanes<V, VEC> d[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const int32_t e0 = base + (j * W + lane) * VEC;
            const int32_t ea = (e0 < k1) ? e0 : kb;
            d[j].load(vals + ea, col + ea);
        }
        // column indices of loaded vectors are all valid (real entries of
        // some row or the zero padding), so the gathers need no guard
        double xv[U][VEC];
#pragma unroll
        for (int j = 0; j < U; ++j)
#pragma unroll
            for (int t = 0; t < VEC; ++t)
                xv[j][t] = (double)gld(x + d[j].c[t]);
#pragma unroll
        for (int j = 0; j < U; ++j)
#pragma unroll
            for (int t = 0; t < VEC; ++t) {
                const int32_t e = base + (j * W + lane) * VEC + t;
                if (e >= k0 && e < k1)
                    acc = fma((double)d[j].v[t], xv[j][t], acc);
            }
    }
    return acc;
}

// Vector width used by a class: 16-byte value loads for groups of 8 lanes
// or more, single elements for narrower groups (rows of a few non-zeros).
template <typename V, int W>
struct VecOf {
    static constexpr int value = (W >= 8) ? (int)(16 / sizeof(V)) : 1;
};
constexpr int kUnroll = 2;

template <typename V>
__device__ __forceinline__ V epilogue(double s, const Epi &e)
{
    if (e.mode == EPI_PAGERANK)
        s = e.d * s + e.tele;
    return (V)s;
}

// Row number of position p of a tile: contiguous tiles store the first row
// itself, others index the class-ordered row list.
__device__ __forceinline__ int32_t tile_row(const MatDesc &m, const Tile &t,
                                            int32_t p)
{
    return (t.cls & kTileContig) ? t.first + p : gld(m.bin_rows + t.first + p);
}

// Rows of a tile, W lanes per row (W <= 64).  Group g of the workgroup takes
// rows g, g+G, g+2G, ... of the tile, so consecutive groups read consecutive
// rows.  Each wavefront first loads the row numbers and bounds of all the
// rows its groups will handle (one lane per row) and hands them to the
// groups with lane shuffles, so no row waits on its own pointer loads.
template <typename V, int W, bool DOT>
__device__ __forceinline__ void rows_by_lanes(const MatDesc &m, const Tile &t,
                                              const Epi &epi, double &dacc)
{
    constexpr int G = kBlock / W;   // groups per workgroup
    constexpr int GPW = 64 / W;     // groups per wavefront
    const int wave = threadIdx.x >> 6;
    const int wl = threadIdx.x & 63;
    const int q = wl / W;           // group within the wavefront
    const int lane = wl % W;
    const int g = wave * GPW + q;
    const V *vals = (const V *)m.vals;
    const V *x = (const V *)m.x;
    V *y = (V *)m.y;
    const int32_t count = t.count;
    // prefetch: lane wl holds row i_p*G + wave*GPW + (wl % GPW)
    const int32_t jp = (wl / GPW) * G + wave * GPW + (wl % GPW);
    int32_t pr = 0, pk0 = 0, pk1 = 0;
    if (jp < count) {
        pr = tile_row(m, t, jp);
        pk0 = gld(m.row_ptr + pr);
        pk1 = gld(m.row_ptr + pr + 1);
    }
    const int32_t g0 = wave * GPW;
    const int32_t iters = (count > g0) ? (count - g0 + G - 1) / G : 0;
    for (int32_t i = 0; i < iters; ++i) {
        const int src = i * GPW + q;
        const int32_t row = __shfl(pr, src, 64);
        const int32_t k0 = __shfl(pk0, src, 64);
        const int32_t k1 = __shfl(pk1, src, 64);
        if (g + i * G < count) {
            const double s = lane_group_sum<W>(
                row_partial<V, W, VecOf<V, W>::value, kUnroll>(m.col, vals, x,
                                                                k0, k1, lane));
            if (lane == 0) {
                const V out = epilogue<V>(s, epi);
                gst(y + row, out);
                if (DOT)
                    dacc = fma((double)gld((const V *)m.w + row), (double)out, dacc);
            }
        }
    }
}

// Rows of a tile, one whole workgroup per row.
template <typename V, bool DOT>
__device__ __forceinline__ void rows_by_block(const MatDesc &m, const Tile &t,
                                              const Epi &epi, double &dacc,
                                              double *lds)
{
    const V *vals = (const V *)m.vals;
    const V *x = (const V *)m.x;
    V *y = (V *)m.y;
    for (int j = 0; j < t.count; ++j) {
        const int32_t row = tile_row(m, t, j);
        const int32_t k0 = gld(m.row_ptr + row);
        const int32_t k1 = gld(m.row_ptr + row + 1);
        const double s = block_sum<kWaves>(
            row_partial<V, kBlock, VecOf<V, kBlock>::value, kUnroll>(
                m.col, vals, x, k0, k1, threadIdx.x),
            lds);
        if (threadIdx.x == 0) {
            const V out = epilogue<V>(s, epi);
            gst(y + row, out);
            if (DOT)
                dacc = fma((double)gld((const V *)m.w + row), (double)out, dacc);
        }
    }
}

// One chunk of a split row: the workgroup's sum goes to chunk_part.
template <typename V>
__device__ __forceinline__ void split_chunk(const MatDesc &m, const Tile &t,
                                            double *lds)
{
    const int32_t c = t.first;
    const int32_t k0 = gld(m.c_k0 + c);
    const int32_t k1 = gld(m.c_k1 + c);
    const double s = block_sum<kWaves>(
        row_partial<V, kBlock, VecOf<V, kBlock>::value, kUnroll>(
            m.col, (const V *)m.vals, (const V *)m.x, k0, k1, threadIdx.x),
        lds);
    if (threadIdx.x == 0)
        gst(m.chunk_part + c, s);
}

// Persistent tile loop: workgroup b takes tiles b, b+grid, b+2*grid, ...
// (a static assignment, so the optional fused dot is summed in a fixed
// order).  Tiles are ordered longest work first.
template <typename V, bool GROUPED, bool DOT>
__global__ __launch_bounds__(kBlock) void k_spmv_tiles(
    const Tile *__restrict__ tiles, int32_t ntiles, MatDesc single,
    const MatDesc *__restrict__ mats, Epi epi, double *__restrict__ dot_part)
{
    __shared__ double lds[kWaves];
    double dacc = 0.0;
    for (int32_t ti = blockIdx.x; ti < ntiles; ti += gridDim.x) {
        const Tile t = tiles[ti];
        const MatDesc m = GROUPED ? mats[t.mat] : single;
        switch (t.cls & kTileClassMask) {
        case C_W1: rows_by_lanes<V, 1, DOT>(m, t, epi, dacc); break;
        case C_W2: rows_by_lanes<V, 2, DOT>(m, t, epi, dacc); break;
        case C_W4: rows_by_lanes<V, 4, DOT>(m, t, epi, dacc); break;
        case C_W8: rows_by_lanes<V, 8, DOT>(m, t, epi, dacc); break;
        case C_W16: rows_by_lanes<V, 16, DOT>(m, t, epi, dacc); break;
        case C_W32: rows_by_lanes<V, 32, DOT>(m, t, epi, dacc); break;
        case C_W64: rows_by_lanes<V, 64, DOT>(m, t, epi, dacc); break;
        case C_WG: rows_by_block<V, DOT>(m, t, epi, dacc, lds); break;
        default: split_chunk<V>(m, t, lds); break;
        }
    }
    if (DOT) {
        const double tot = block_sum<kWaves>(dacc, lds);
        if (threadIdx.x == 0)
            dot_part[blockIdx.x] = tot;
    }
}

// Split rows: add the chunk sums of each split row in chunk order, apply the
// epilogue and store.  One thread per split row.
template <typename V, bool GROUPED, bool DOT>
__global__ __launch_bounds__(kBlock) void k_split_finalize(
    const int32_t *__restrict__ items, int32_t n, MatDesc single,
    const MatDesc *__restrict__ mats, Epi epi, double *__restrict__ dot_part)
{
    __shared__ double lds[kWaves];
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    double dacc = 0.0;
    if (i < n) {
        const int32_t mi = GROUPED ? items[2 * i] : 0;
        const int32_t j = GROUPED ? items[2 * i + 1] : i;
        const MatDesc m = GROUPED ? mats[mi] : single;
        const int32_t row = m.bin_rows[m.split_begin + j];
        double s = 0.0;
        for (int32_t c = m.s_first[j]; c < m.s_first[j + 1]; ++c)
            s += m.chunk_part[c];
        const V out = epilogue<V>(s, epi);
        ((V *)m.y)[row] = out;
        if (DOT)
            dacc = (double)((const V *)m.w)[row] * (double)out;
    }
    if (DOT) {
        const double tot = block_sum<kWaves>(dacc, lds);
        if (threadIdx.x == 0)
            dot_part[blockIdx.x] = tot;
    }
}

// Several matrices in one launch, each with its own tile list; workgroup b
// takes virtual tiles b, b+grid, ...; virtual tile v is tile v - prefix[j]
// of matrix j (binary search over the prefix).
template <typename V>
__global__ __launch_bounds__(kBlock) void k_spmv_segments(
    const MatDesc *__restrict__ mats, const int32_t *__restrict__ prefix,
    int32_t nseg, int32_t total)
{
    __shared__ double lds[kWaves];
    const Epi epi{EPI_NONE, 0, 0.0, 0.0};
    double dacc = 0.0;
    for (int32_t v = blockIdx.x; v < total; v += gridDim.x) {
        int32_t lo = 0, hi = nseg;
        while (hi - lo > 1) {
            const int32_t mid = (lo + hi) >> 1;
            if (prefix[mid] <= v)
                lo = mid;
            else
                hi = mid;
        }
        const MatDesc m = mats[lo];
        const i32x4 tv = gld((const i32x4 *)(m.tiles + (v - prefix[lo])));
        const Tile t{tv.x, tv.y, tv.z, tv.w};
        switch (t.cls & kTileClassMask) {
        case C_W1: rows_by_lanes<V, 1, false>(m, t, epi, dacc); break;
        case C_W2: rows_by_lanes<V, 2, false>(m, t, epi, dacc); break;
        case C_W4: rows_by_lanes<V, 4, false>(m, t, epi, dacc); break;
        case C_W8: rows_by_lanes<V, 8, false>(m, t, epi, dacc); break;
        case C_W16: rows_by_lanes<V, 16, false>(m, t, epi, dacc); break;
        case C_W32: rows_by_lanes<V, 32, false>(m, t, epi, dacc); break;
        case C_W64: rows_by_lanes<V, 64, false>(m, t, epi, dacc); break;
        case C_WG: rows_by_block<V, false>(m, t, epi, dacc, lds); break;
        default: split_chunk<V>(m, t, lds); break;
        }
    }
}

// ------------------------------------------------------- column panels

// Product over the column-panel layout.  Workgroup b (one per CU, 16
// wavefronts) owns row block b; for each panel it copies that slice of x into
// LDS, and each wavefront streams its own entries of the panel in coalesced
// chunks: lane j forms vals[k] * x[col] from LDS for two consecutive
// entries, a segmented scan over the lanes (rows ascend along the chunk) adds
// up each row's run, and the last lane of a run adds it to the row's sum in
// LDS.  Rows belong to one wavefront, chunks follow in order, panels follow
// in an order fixed for the block: the additions are in a fixed order given
// by the matrix and the layout.
template <typename V, bool DOT>
__device__ __forceinline__ void panel_block(const PanelDesc &pd, int32_t b,
                                            const V *__restrict__ x,
                                            V *__restrict__ y, const Epi &epi,
                                            const V *__restrict__ w,
                                            double *__restrict__ dot_part,
                                            unsigned char *smem)
{
    double *acc = (double *)smem;                                 // row sums
    V *xs = (V *)(smem + panel_sum_bytes(pd.rb));                 // x panel
    constexpr int VV = 16 / sizeof(V);
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int32_t r0 = b * pd.rb;
    const int32_t nr = min(pd.rb, pd.rows - r0);
    const V *pv = (const V *)pd.vals;
    for (int i = threadIdx.x; i < pd.rb; i += kPanelThreads)
        acc[i] = 0.0;
    // the dot operand of this thread's row (rows <= threads), read now so
    // the epilogue does not wait for it
    double wrow = 0.0;
    if (DOT && (int32_t)threadIdx.x < nr)
        wrow = (double)gld(w + r0 + threadIdx.x);
    const bool aligned = (((uintptr_t)x) & 15) == 0;
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    typedef V pair_t __attribute__((ext_vector_type(2)));
    typedef uint32_t upair_t __attribute__((ext_vector_type(2)));
    // entry range of this wavefront in panel q; uniform over the wavefront
    // (scalar registers, scalar branches)
    // (scalar loads: the table is read-only while the kernel runs)
    auto range = [&](int32_t q, int32_t &rs, int32_t &re) {
        typedef const __attribute__((address_space(4))) int32_t *cptr;
        const cptr wp = (cptr)(pd.wptr + ((int64_t)b * pd.np + q) * (kPanelWaves + 1));
        rs = wp[wv];
        re = wp[wv + 1];
    };
    // chunks of 128 entries from an even start: lane j holds the two
    // consecutive entries at + 2j and at + 2j + 1 (one 16-byte value load,
    // one 8-byte index load).  The entries of the next step are requested
    // before this step's arithmetic (the first step of the next panel before
    // that panel is copied), so loads stay in flight while the wavefront
    // computes or waits.
    pair_t nv[kPanelChunks];
    upair_t nrc[kPanelChunks];
    auto request = [&](int32_t at, int32_t rb, int32_t re) {
#pragma unroll
        for (int u = 0; u < kPanelChunks; ++u) {
            const int32_t e = at + u * 128 + 2 * lane;
            const int32_t ea = (e < re) ? e : rb;
            nv[u] = ld_stream((const pair_t *)(pv + ea));
            nrc[u] = ld_stream((const upair_t *)(pd.rc + ea));
        }
    };
    int32_t ks = 0, ke = 0;
    // One step: chunks of 128 entries at base, base + 128, ..., all in
    // lockstep (independent scans interleave); the sums reach the rows chunk
    // by chunk, in order.  FULL: every entry of the step lies in [ks, ke)
    // (most steps), so the bound checks are compiled out; the two cases are
    // separate code, with no merge of their values.
    auto body = [&](auto fullc, const pair_t (&v)[kPanelChunks],
                    const upair_t (&rc)[kPanelChunks], int32_t base) {
        constexpr bool FULL = decltype(fullc)::value;
        int32_t k0[kPanelChunks], k1[kPanelChunks];
        double p0[kPanelChunks], incl[kPanelChunks];
        // the x values of all entries first, every LDS read in flight at
        // once.  Entries outside [ks, ke) are read too: each is some entry
        // of the matrix, whose column in its panel is below pw, so the read
        // stays inside the panel buffer; its product is dropped.
        V xa[kPanelChunks], xb[kPanelChunks];
#pragma unroll
        for (int u = 0; u < kPanelChunks; ++u) {
            xa[u] = xs[rc[u].x & 0xFFFFu];
            xb[u] = xs[rc[u].y & 0xFFFFu];
        }
#pragma unroll
        for (int u = 0; u < kPanelChunks; ++u) {
            const int32_t e = base + u * 128 + 2 * lane;
            // keys ascend along the wavefront: entries before ks belong to
            // the previous wavefront (-1), entries past ke to nobody (max)
            double p1;
            if (FULL) {
                k0[u] = (int32_t)(rc[u].x >> 16);
                k1[u] = (int32_t)(rc[u].y >> 16);
                p0[u] = (double)v[u].x * (double)xa[u];
                p1 = (double)v[u].y * (double)xb[u];
            } else {
                k0[u] = (e < ks) ? -1 : (e < ke) ? (int32_t)(rc[u].x >> 16) : kPanelMaxRb;
                k1[u] = (e + 1 < ks) ? -1
                        : (e + 1 < ke) ? (int32_t)(rc[u].y >> 16)
                                       : kPanelMaxRb;
                const bool ok0 = e >= ks && e < ke, ok1 = e + 1 >= ks && e + 1 < ke;
                p0[u] = ok0 ? (double)v[u].x * (double)xa[u] : 0.0;
                p1 = ok1 ? (double)v[u].y * (double)xb[u] : 0.0;
            }
            // this lane's part of the run of its last key (a run that
            // starts inside a lane breaks the scan because keys ascend)
            incl[u] = (k0[u] == k1[u]) ? p0[u] + p1 : p1;
        }
#pragma unroll
        for (int u = 0; u < kPanelChunks; ++u)
            incl[u] = seg_scan64<true>(incl[u], k1[u]);
#pragma unroll
        for (int u = 0; u < kPanelChunks; ++u) {
            // the previous lane's scan value and key (wave_shr:1; lane 0
            // reads 0 and key 0, which adds 0 if it matches)
            const double prev_incl = dpp_f64<0x138>(incl[u]);
            const int32_t prev_k1 = dpp_i32z<0x138>(k1[u]);
            const int32_t next_k0 = next_lane_key(k0[u]);
            // a run of k0 that ends on this lane's first entry.  A row's run
            // ends on one lane of a chunk, and a row belongs to one
            // wavefront, whose LDS operations complete in order: the
            // additions (no-return LDS adds, nothing to wait for) reach each
            // row in a fixed order.  Keys of a full step are all rows.
            if (k0[u] != k1[u] && (FULL || (k0[u] >= 0 && k0[u] < kPanelMaxRb)))
                lds_add_f64(&acc[k0[u]], (prev_k1 == k0[u]) ? prev_incl + p0[u] : p0[u]);
            // the run of k1 ends on this lane
            if (next_k0 != k1[u] && (FULL || (k1[u] >= 0 && k1[u] < kPanelMaxRb)))
                lds_add_f64(&acc[k1[u]], incl[u]);
        }
    };
    typedef std::integral_constant<bool, true> full_t;
    typedef std::integral_constant<bool, false> edge_t;
    // A matrix with many row blocks takes its panels in a rotated order:
    // the workgroups that share an XCD (b, b + 8, ...) start at different
    // panels, so their copies of x from that XCD's L2 spread over the run
    // instead of all coming at once.  The order depends only on the matrix
    // and the block, so a block sums its rows the same way in every launch.
    const int32_t rot =
        (pd.np > 1 && pd.nblk >= kPanelRotateBlocks) ? (int32_t)((b >> 3) % pd.np) : 0;
    auto panel_at = [&](int32_t i) { return (i + rot < pd.np) ? i + rot : i + rot - pd.np; };
    if (pd.np > 0)
        range(panel_at(0), ks, ke);
    if ((ks & ~1) < ke)
        request(ks & ~1, ks & ~1, ke);
    for (int32_t pk = 0; pk < pd.np; ++pk) {   // the block's pk-th panel
        const int32_t p = panel_at(pk);
        const int32_t c0 = p * pd.pw;
        const int32_t width = min(pd.pw, pd.cols - c0);
        int32_t nks = 0, nke = 0;  // the next panel's range
        if (pk + 1 < pd.np)
            range(panel_at(pk + 1), nks, nke);
        __syncthreads();  // the previous panel is no longer read
        // 16-byte pieces straight from memory into LDS (no registers): each
        // wavefront instruction fills 1 KiB at a uniform LDS address
        const int32_t nvec = aligned ? width / VV : 0;
        for (int32_t c = wv; c * 64 < nvec; c += kPanelWaves) {
            const int32_t i = c * 64 + lane;
            if (i < nvec)
                __builtin_amdgcn_global_load_lds(
                    (const __attribute__((address_space(1))) void *)(x + c0 + i * VV),
                    (__attribute__((address_space(3))) void *)(xs + c * 64 * VV), 16, 0, 0);
        }
        for (int32_t e = nvec * VV + threadIdx.x; e < width; e += kPanelThreads)
            xs[e] = gld(x + c0 + e);
        __builtin_amdgcn_s_waitcnt(0);  // the direct loads have landed
        __syncthreads();                 // the panel is in LDS
        const int32_t kb = ks & ~1;
        const int32_t nkb = nks & ~1;
        if (kb >= ke && nkb < nke)
            request(nkb, nkb, nke);  // nothing here: the next panel's first step
        for (int32_t base = kb; base < ke; base += 128 * kPanelChunks) {
            pair_t v[kPanelChunks];
            upair_t rc[kPanelChunks];
#pragma unroll
            for (int u = 0; u < kPanelChunks; ++u) {
                v[u] = nv[u];
                rc[u] = nrc[u];
            }
            if (base + 128 * kPanelChunks < ke)
                request(base + 128 * kPanelChunks, kb, ke);
            else if (nkb < nke)
                request(nkb, nkb, nke);
            if (base >= ks && base + 128 * kPanelChunks <= ke)
                body(full_t(), v, rc, base);
            else
                body(edge_t(), v, rc, base);
        }
        ks = nks;
        ke = nke;
    }
    __syncthreads();
    double dacc = 0.0;
    for (int32_t i = threadIdx.x; i < nr; i += kPanelThreads) {
        const V out = epilogue<V>(acc[i], epi);
        gst(y + r0 + i, out);
        if (DOT)
            dacc = fma(i == (int32_t)threadIdx.x ? wrow : (double)gld(w + r0 + i),
                       (double)out, dacc);
    }
    if (DOT) {
        const double tot = block_sum<kPanelWaves>(dacc, (double *)xs);
        if (threadIdx.x == 0)
            dot_part[b] = tot;
    }
}

template <typename V, bool DOT>
__global__ __launch_bounds__(kPanelThreads) void k_spmv_panels(
    PanelDesc pd, const V *__restrict__ x, V *__restrict__ y, Epi epi,
    const V *__restrict__ w, double *__restrict__ dot_part)
{
    extern __shared__ __align__(16) unsigned char smem[];
    panel_block<V, DOT>(pd, blockIdx.x, x, y, epi, w, dot_part, smem);
}

// Column-panel products of many matrices in one launch: workgroup g takes
// row block g - prefix[j] of matrix j (prefix[j] <= g < prefix[j + 1]).
// Each block runs exactly as in the single-matrix kernel.
template <typename V>
__global__ __launch_bounds__(kPanelThreads) void k_spmv_panels_grouped(
    const PanelDesc *__restrict__ descs, const PanelIO *__restrict__ io,
    const int32_t *__restrict__ prefix, int32_t nmat)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int32_t g = blockIdx.x;
    int32_t lo = 0, hi = nmat - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= g)
            lo = mid;
        else
            hi = mid - 1;
    }
    const PanelDesc pd = descs[lo];
    const Epi epi{EPI_NONE, 0, 0.0, 0.0};
    const PanelIO pio = io[lo];
    if constexpr (sizeof(V) == 8) {
        if (pio.dot) {
            panel_block<V, true>(pd, g - prefix[lo], (const V *)pio.x, (V *)pio.y, epi,
                                 (const V *)pio.x, pio.dot, smem);
            return;
        }
    }
    panel_block<V, false>(pd, g - prefix[lo], (const V *)pio.x, (V *)pio.y,
                          epi, nullptr, nullptr, smem);
}

// Distinct x cache lines among the non-zeros of sampled row groups (see
// launch_line_reuse).  The count is a union of bits, so it does not depend
// on the order of the atomic updates.
__global__ __launch_bounds__(kBlock) void k_line_reuse(int32_t rows,
                                                       const int32_t *__restrict__ rp,
                                                       const int32_t *__restrict__ col,
                                                       int32_t ngroups, int32_t shift,
                                                       int32_t *__restrict__ out)
{
    __shared__ uint32_t bits[512];
    __shared__ int32_t red[kWaves];
    for (int i = threadIdx.x; i < 512; i += kBlock)
        bits[i] = 0u;
    __syncthreads();
    const int64_t groups = ((int64_t)rows + 63) / 64;
    const int32_t grp = (int32_t)((int64_t)blockIdx.x * groups / ngroups);
    const int32_t r0 = grp * 64;
    const int32_t r1 = min(rows, r0 + 64);
    const int32_t k0 = rp[r0];
    const int32_t k1 = min(rp[r1], k0 + 8192);
    for (int32_t k = k0 + threadIdx.x; k < k1; k += kBlock) {
        const uint32_t line = (uint32_t)col[k] >> shift;
        atomicOr(&bits[(line >> 5) & 511u], 1u << (line & 31u));
    }
    __syncthreads();
    int32_t cnt = 0;
    for (int i = threadIdx.x; i < 512; i += kBlock)
        cnt += __popc(bits[i]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        cnt += __shfl_down(cnt, off, 64);
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t t = 0;
        for (int i = 0; i < kWaves; ++i)
            t += red[i];
        out[2 * blockIdx.x] = k1 - k0;
        out[2 * blockIdx.x + 1] = t;
    }
}

// Entries of each row per panel: one wavefront per row, 64 entries at a
// time, one ballot per panel (cnt pre-zeroed).
__global__ __launch_bounds__(kBlock) void k_panel_count(PanelDesc pd,
                                                        const int32_t *__restrict__ rp,
                                                        const int32_t *__restrict__ col,
                                                        int32_t *__restrict__ cnt)
{
    const int64_t i = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (i >= pd.rows)
        return;  // whole wavefronts
    const int32_t b = (int32_t)(i / pd.rb), rl = (int32_t)(i - (int64_t)b * pd.rb);
    const int32_t a = rp[i], e = rp[i + 1];
    int32_t mine = 0;  // lane p < np counts panel p
    for (int32_t base = a; base < e; base += 64) {
        const int32_t k = base + lane;
        const int32_t pan = (k < e) ? col[k] / pd.pw : -1;
        for (int32_t p = 0; p < pd.np; ++p) {
            const int32_t n = __popcll(__ballot(pan == p));
            if (lane == p)
                mine += n;
        }
    }
    if (lane < pd.np)
        cnt[(int64_t)(b * pd.np + lane) * (pd.rb + 1) + rl] = mine;
}

// Move each row's entries to their panels, keeping their order inside a
// row: one wavefront per row, 64 entries at a time, positions from ballots.
template <typename V>
__global__ __launch_bounds__(kBlock) void k_panel_scatter(
    PanelDesc pd, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
    const V *__restrict__ vals, const int32_t *__restrict__ ptr,
    V *__restrict__ pv, uint32_t *__restrict__ prc)
{
    const int64_t i = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (i >= pd.rows)
        return;  // whole wavefronts
    const int32_t b = (int32_t)(i / pd.rb), rl = (int32_t)(i - (int64_t)b * pd.rb);
    const int32_t a = rp[i], e = rp[i + 1];
    // lane p < np holds the next free position of panel p
    int32_t next = (lane < pd.np) ? ptr[(int64_t)(b * pd.np + lane) * (pd.rb + 1) + rl] : 0;
    for (int32_t base = a; base < e; base += 64) {
        const int32_t k = base + lane;
        const int32_t c = (k < e) ? col[k] : 0;
        const int32_t pan = (k < e) ? c / pd.pw : -1;
        int32_t pos = 0;
        for (int32_t p = 0; p < pd.np; ++p) {
            const uint64_t m = __ballot(pan == p);
            const int32_t start = __shfl(next, p, 64);
            if (pan == p)
                pos = start + lanes_below(m);
            if (lane == p)
                next += __popcll(m);
        }
        if (k < e) {
            pv[pos] = vals[k];
            prc[pos] = ((uint32_t)rl << 16) | (uint32_t)(c - pan * pd.pw);
        }
    }
}

// Where each wavefront's rows start, for every (row block, panel).
__global__ __launch_bounds__(kBlock) void k_panel_wptr(PanelDesc pd,
                                                       const int32_t *__restrict__ ptr,
                                                       int32_t *__restrict__ wptr)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t nseg = (int64_t)pd.nblk * pd.np;
    if (t >= nseg * (kPanelWaves + 1))
        return;
    const int64_t seg = t / (kPanelWaves + 1);
    const int32_t wv = (int32_t)(t - seg * (kPanelWaves + 1));
    wptr[t] = ptr[seg * (pd.rb + 1) + min(wv * pd.rw, pd.rb)];
}

// ------------------------------------------------------- hot columns

// Row keys inside a block are below 2^16; this one is past every row.
constexpr int32_t kKeyEnd = 1 << 16;

// The first chunk of a wavefront's share of a block part, requested ahead.
template <typename V>
struct HotChunk {
    typedef V pair_t __attribute__((ext_vector_type(2)));
    typedef uint32_t upair_t __attribute__((ext_vector_type(2)));
    typedef uint16_t kpair_t __attribute__((ext_vector_type(2)));
    pair_t v;
    upair_t rc;
    kpair_t kk;
};

// This wavefront's share [ks, ke) of a part [s, e) split evenly between NW.
template <int NW>
__device__ __forceinline__ void hot_share(int32_t s, int32_t e, int wave, int32_t &ks,
                                          int32_t &ke)
{
    const int64_t n = (int64_t)e - s;
    ks = __builtin_amdgcn_readfirstlane(s + (int32_t)(n * wave / NW));
    ke = __builtin_amdgcn_readfirstlane(s + (int32_t)(n * (wave + 1) / NW));
}

// Requests the first chunk of this wavefront's share of a part (nothing if
// the share is empty).
template <typename V, bool HOT, int NW = kPanelWaves>
__device__ __forceinline__ void hot_first(const V *__restrict__ pv,
                                          const uint32_t *__restrict__ prc,
                                          const uint16_t *__restrict__ pkey, int32_t s,
                                          int32_t e, int wave, int lane, HotChunk<V> &c)
{
    typedef typename HotChunk<V>::pair_t pair_t;
    typedef typename HotChunk<V>::upair_t upair_t;
    typedef typename HotChunk<V>::kpair_t kpair_t;
    int32_t ks, ke;
    hot_share<NW>(s, e, wave, ks, ke);
    const int32_t kb = ks & ~1;
    if (kb < ke) {
        const int32_t en = kb + 2 * lane;
        const int32_t ea = (en < ke) ? en : kb;
        c.v = ld_stream((const pair_t *)(pv + ea));
        c.rc = ld_stream((const upair_t *)(prc + ea));
        if (!HOT)
            c.kk = ld_stream((const kpair_t *)(pkey + ea));
    }
}

// One wavefront's share of a block part [s, e) of the hot-column layout.
// The part is split evenly by entries, so a row can span wavefronts: the
// run of the wavefront's first row goes to its carry slot (added after the
// block, in slot order), every other run is added to the row sum in LDS by
// the one wavefront where it ends.  A row is named by its key (its number
// among the block's non-empty rows in the hot-column layout, its offset in
// the block in the band layout).  HOT: the entry's word packs (key << 16)
// | column offset and the gather reads xsrc[offset] (the LDS copy of the
// hot columns, or x from a block's first column in the band layout);
// otherwise the word is the column of x and the key comes from key[].  The
// entries of the next chunk are requested before the gathers of the
// current one are used; with gathers from device memory the next chunk's
// gathers are requested too.  NW wavefronts share the part; XG: xsrc is in
// device memory (else in LDS).  PRE: the first chunk was requested earlier
// into *pre (hot_first, same part and wavefront).
template <typename V, bool HOT, int NW = kPanelWaves, bool XG = !HOT, bool PRE = false>
__device__ __forceinline__ void hot_part(const V *__restrict__ pv,
                                         const uint32_t *__restrict__ prc,
                                         const uint16_t *__restrict__ pkey,
                                         int32_t s, int32_t e, const V *xsrc,
                                         double *acc, int32_t *ckey, double *csum,
                                         int wave, int lane,
                                         const HotChunk<V> *pre = nullptr)
{
    typedef typename HotChunk<V>::pair_t pair_t;
    typedef typename HotChunk<V>::upair_t upair_t;
    typedef typename HotChunk<V>::kpair_t kpair_t;
    int32_t ks, ke;
    hot_share<NW>(s, e, wave, ks, ke);
    const int32_t kb = ks & ~1;
    pair_t v;
    upair_t rc;
    kpair_t kk;
    int32_t first = -1;
    if (kb < ke) {
        if (PRE) {
            v = pre->v;
            rc = pre->rc;
            if (!HOT)
                kk = pre->kk;
        } else {
            const int32_t en = kb + 2 * lane;
            const int32_t ea = (en < ke) ? en : kb;
            v = ld_stream((const pair_t *)(pv + ea));
            rc = ld_stream((const upair_t *)(prc + ea));
            if (!HOT)
                kk = ld_stream((const kpair_t *)(pkey + ea));
        }
        // the share's first entry is entry 0 or 1 of lane 0
        const int32_t f0 = HOT ? (int32_t)(rc.x >> 16) : (int32_t)kk.x;
        const int32_t f1 = HOT ? (int32_t)(rc.y >> 16) : (int32_t)kk.y;
        first = __builtin_amdgcn_readfirstlane((ks == kb) ? f0 : f1);
    }
    if (lane == 0) {
        *ckey = first;
        *csum = 0.0;
    }
    // whether entry j of the chunk at `base` lies in the share, and the
    // column it gathers (entries outside the share may belong to the other
    // part, another packing: they gather element 0, which always exists)
    auto in_share = [&](int32_t base, int j) {
        const int32_t en = base + 2 * lane + j;
        return (base >= ks && base + 128 <= ke) || (en >= ks && en < ke);
    };
    auto column = [&](uint32_t w, bool ok) {
        return ok ? (HOT ? (w & 0xFFFFu) : w) : 0u;
    };
    auto request = [&](int32_t at, pair_t &rv, upair_t &rr, kpair_t &rk) {
        const int32_t nn = at + 2 * lane;
        const int32_t ea = (nn < ke) ? nn : kb;
        rv = ld_stream((const pair_t *)(pv + ea));
        rr = ld_stream((const upair_t *)(prc + ea));
        if (!HOT)
            rk = ld_stream((const kpair_t *)(pkey + ea));
    };
    // gathers from device memory: the next chunk's entries are in hand and
    // its gathers requested before this chunk's arithmetic, with the entries
    // of the chunk after it on the way (two memory round trips per chunk,
    // the second depending on the first, kept in flight together)
    V gx0 = 0, gx1 = 0;     // gathers of the current chunk
    pair_t v2;              // entries of the next chunk
    upair_t rc2;
    kpair_t kk2;
    if (XG && kb < ke) {
        gx0 = gld(xsrc + column(rc.x, in_share(kb, 0)));
        gx1 = gld(xsrc + column(rc.y, in_share(kb, 1)));
        if (kb + 128 < ke)
            request(kb + 128, v2, rc2, kk2);
    }
    for (int32_t base = kb; base < ke; base += 128) {
        const int32_t en = base + 2 * lane;
        // chunks wholly inside [ks, ke) (most of them) need no bound checks
        const bool full = base >= ks && base + 128 <= ke;
        const bool ok0 = full || (en >= ks && en < ke);
        const bool ok1 = full || (en + 1 >= ks && en + 1 < ke);
        const int32_t r0 = HOT ? (int32_t)(rc.x >> 16) : (int32_t)kk.x;
        const int32_t r1 = HOT ? (int32_t)(rc.y >> 16) : (int32_t)kk.y;
        // keys ascend along the wavefront: entries before ks belong to the
        // previous wavefront (-1), entries past ke to nobody (kKeyEnd)
        const int32_t k0 = full ? r0 : (en < ks) ? -1 : ok0 ? r0 : kKeyEnd;
        const int32_t k1 = full ? r1 : (en + 1 < ks) ? -1 : ok1 ? r1 : kKeyEnd;
        const pair_t cv = v;
        const int32_t nb = base + 128;
        V x0, x1;
        if (XG) {
            x0 = gx0;
            x1 = gx1;
            if (nb < ke) {
                v = v2;
                rc = rc2;
                if (!HOT)
                    kk = kk2;
                gx0 = gld(xsrc + column(rc.x, in_share(nb, 0)));
                gx1 = gld(xsrc + column(rc.y, in_share(nb, 1)));
                if (nb + 128 < ke)
                    request(nb + 128, v2, rc2, kk2);
            }
        } else {
            x0 = xsrc[column(rc.x, ok0)];
            x1 = xsrc[column(rc.y, ok1)];
            if (nb < ke)
                request(nb, v, rc, kk);
        }
        const double p0 = ok0 ? (double)cv.x * (double)x0 : 0.0;
        const double p1 = ok1 ? (double)cv.y * (double)x1 : 0.0;
        // this lane's part of the run of its last key (a run that starts
        // inside a lane breaks the scan because keys ascend)
        double incl = (k0 == k1) ? p0 + p1 : p1;
        incl = seg_scan64(incl, k1);
        // previous lane's scan value and key (wave_shr:1; lane 0 reads 0)
        const double prev_incl = dpp_f64<0x138>(incl);
        const int32_t prev_k1 = dpp_i32z<0x138>(k1);
        const int32_t next_k0 = next_lane_key(k0);
        // no-return LDS adds: a row's runs end in this wavefront only (its
        // first row goes to the carry slot), in program order
        if (k0 != k1 && k0 >= 0 && k0 < kKeyEnd) {
            double *t = (k0 == first) ? csum : acc + k0;
            lds_add_f64(t, (prev_k1 == k0) ? prev_incl + p0 : p0);
        }
        if (next_k0 != k1 && k1 >= 0 && k1 < kKeyEnd) {
            double *t = (k1 == first) ? csum : acc + k1;
            lds_add_f64(t, incl);
        }
    }
}


// The same for four entries per lane (float32 values: 16-byte loads).
struct HotChunk4 {
    typedef float quad_t __attribute__((ext_vector_type(4)));
    typedef uint32_t uquad_t __attribute__((ext_vector_type(4)));
    typedef uint16_t kquad_t __attribute__((ext_vector_type(4)));
    quad_t v;
    uquad_t rc;
    kquad_t kk;
};

template <bool HOT, int NW = kPanelWaves>
__device__ __forceinline__ void hot_first4(const float *__restrict__ pv,
                                           const uint32_t *__restrict__ prc,
                                           const uint16_t *__restrict__ pkey, int32_t s,
                                           int32_t e, int wave, int lane, HotChunk4 &c)
{
    int32_t ks, ke;
    hot_share<NW>(s, e, wave, ks, ke);
    const int32_t kb = ks & ~3;
    if (kb < ke) {
        const int32_t en = kb + 4 * lane;
        const int32_t ea = (en < ke) ? en : kb;
        c.v = ld_stream((const HotChunk4::quad_t *)(pv + ea));
        c.rc = ld_stream((const HotChunk4::uquad_t *)(prc + ea));
        if (!HOT)
            c.kk = ld_stream((const HotChunk4::kquad_t *)(pkey + ea));
    }
}

// hot_part with four consecutive entries per lane and chunks of 256 from a
// multiple of four: the runs that start and end inside a lane are added
// directly, the lane's first run joins the previous lane's scan value, its
// last run enters a segmented scan over the wavefront.  Each row still
// gets one addition per chunk, from the lane where its run ends, so the
// order of the additions is fixed by the matrix and the layout.
template <bool HOT, int NW = kPanelWaves, bool XG = !HOT, bool PRE = false>
__device__ __forceinline__ void hot_part4(const float *__restrict__ pv,
                                          const uint32_t *__restrict__ prc,
                                          const uint16_t *__restrict__ pkey,
                                          int32_t s, int32_t e, const float *xsrc,
                                          double *acc, int32_t *ckey, double *csum,
                                          int wave, int lane,
                                          const HotChunk4 *pre = nullptr)
{
    typedef HotChunk4::quad_t quad_t;
    typedef HotChunk4::uquad_t uquad_t;
    typedef HotChunk4::kquad_t kquad_t;
    constexpr int32_t CH = 256;
    int32_t ks, ke;
    hot_share<NW>(s, e, wave, ks, ke);
    const int32_t kb = ks & ~3;
    quad_t v;
    uquad_t rc;
    kquad_t kk;
    int32_t first = -1;
    if (kb < ke) {
        if (PRE) {
            v = pre->v;
            rc = pre->rc;
            if (!HOT)
                kk = pre->kk;
        } else {
            const int32_t en = kb + 4 * lane;
            const int32_t ea = (en < ke) ? en : kb;
            v = ld_stream((const quad_t *)(pv + ea));
            rc = ld_stream((const uquad_t *)(prc + ea));
            if (!HOT)
                kk = ld_stream((const kquad_t *)(pkey + ea));
        }
        // the share's first entry is entry ks - kb of lane 0
        const int32_t d = ks - kb;
        const uint32_t w0 = d == 0 ? rc.x : d == 1 ? rc.y : d == 2 ? rc.z : rc.w;
        const uint32_t q0 = d == 0 ? kk.x : d == 1 ? kk.y : d == 2 ? kk.z : kk.w;
        first = __builtin_amdgcn_readfirstlane(HOT ? (int32_t)(w0 >> 16) : (int32_t)q0);
    }
    if (lane == 0) {
        *ckey = first;
        *csum = 0.0;
    }
    auto in_share = [&](int32_t base, int j) {
        const int32_t en = base + 4 * lane + j;
        return (base >= ks && base + CH <= ke) || (en >= ks && en < ke);
    };
    auto column = [&](uint32_t w, bool ok) {
        return ok ? (HOT ? (w & 0xFFFFu) : w) : 0u;
    };
    auto request = [&](int32_t at, quad_t &rv, uquad_t &rr, kquad_t &rk) {
        const int32_t nn = at + 4 * lane;
        const int32_t ea = (nn < ke) ? nn : kb;
        rv = ld_stream((const quad_t *)(pv + ea));
        rr = ld_stream((const uquad_t *)(prc + ea));
        if (!HOT)
            rk = ld_stream((const kquad_t *)(pkey + ea));
    };
    auto add = [&](int32_t k, double t) {
        lds_add_f64((k == first) ? csum : acc + k, t);
    };
    float g[4] = {0.f, 0.f, 0.f, 0.f};   // gathers of the current chunk
    quad_t v2;                           // entries of the next chunk
    uquad_t rc2;
    kquad_t kk2;
    if (XG && kb < ke) {
        g[0] = gld(xsrc + column(rc.x, in_share(kb, 0)));
        g[1] = gld(xsrc + column(rc.y, in_share(kb, 1)));
        g[2] = gld(xsrc + column(rc.z, in_share(kb, 2)));
        g[3] = gld(xsrc + column(rc.w, in_share(kb, 3)));
        if (kb + CH < ke)
            request(kb + CH, v2, rc2, kk2);
    }
    // one chunk; FULL: every entry lies in [ks, ke) (most chunks), so the
    // bound checks are compiled out (full and edge chunks are separate code)
    auto body = [&](int32_t base, auto fullc) {
        const int32_t en = base + 4 * lane;
        constexpr bool full = decltype(fullc)::value;
        const uint32_t wv[4] = {rc.x, rc.y, rc.z, rc.w};
        const int32_t rw[4] = {HOT ? (int32_t)(rc.x >> 16) : (int32_t)kk.x,
                               HOT ? (int32_t)(rc.y >> 16) : (int32_t)kk.y,
                               HOT ? (int32_t)(rc.z >> 16) : (int32_t)kk.z,
                               HOT ? (int32_t)(rc.w >> 16) : (int32_t)kk.w};
        const float cv[4] = {v.x, v.y, v.z, v.w};
        bool ok[4];
        int32_t k[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            ok[t] = full || (en + t >= ks && en + t < ke);
            k[t] = full ? rw[t] : (en + t < ks) ? -1 : ok[t] ? rw[t] : kKeyEnd;
        }
        float xv[4];
        const int32_t nb = base + CH;
        if (XG) {
#pragma unroll
            for (int t = 0; t < 4; ++t)
                xv[t] = g[t];
            if (nb < ke) {
                v = v2;
                rc = rc2;
                if (!HOT)
                    kk = kk2;
                g[0] = gld(xsrc + column(rc.x, in_share(nb, 0)));
                g[1] = gld(xsrc + column(rc.y, in_share(nb, 1)));
                g[2] = gld(xsrc + column(rc.z, in_share(nb, 2)));
                g[3] = gld(xsrc + column(rc.w, in_share(nb, 3)));
                if (nb + CH < ke)
                    request(nb + CH, v2, rc2, kk2);
            }
        } else {
#pragma unroll
            for (int t = 0; t < 4; ++t)
                xv[t] = xsrc[column(wv[t], ok[t])];
            if (nb < ke)
                request(nb, v, rc, kk);
        }
        double pr[4];
#pragma unroll
        for (int t = 0; t < 4; ++t)
            pr[t] = ok[t] ? (double)cv[t] * (double)xv[t] : 0.0;
        // runs inside the lane (keys ascend)
        double run = pr[0], head = 0.0;
        int32_t rk = k[0];
        bool split = false;
#pragma unroll
        for (int t = 1; t < 4; ++t) {
            if (k[t] == rk) {
                run += pr[t];
            } else {
                if (!split) {
                    head = run;
                    split = true;
                } else if (full || (rk >= 0 && rk < kKeyEnd)) {
                    add(rk, run);   // a run wholly inside this lane
                }
                rk = k[t];
                run = pr[t];
            }
        }
        const double incl = seg_scan64(run, k[3]);
        const double prev_incl = dpp_f64<0x138>(incl);
        const int32_t prev_kl = dpp_i32z<0x138>(k[3]);
        const int32_t next_kf = next_lane_key(k[0]);
        if (split && (full || (k[0] >= 0 && k[0] < kKeyEnd)))
            add(k[0], (prev_kl == k[0]) ? prev_incl + head : head);
        if (next_kf != k[3] && (full || (k[3] >= 0 && k[3] < kKeyEnd)))
            add(k[3], incl);
    };
    for (int32_t base = kb; base < ke; base += CH) {
        if (base >= ks && base + CH <= ke)
            body(base, std::true_type());
        else
            body(base, std::false_type());
    }
}

// Product over the hot-column layout.  Persistent: workgroup g copies the
// hot columns of x into LDS once, then takes its own list of row blocks
// (assigned on the host, balanced by work).
// Each wavefront streams its share of the block's hot part and of its cold
// part (odd wavefronts cold first, so LDS and global gathers overlap); the
// two parts add into separate row sums, so no wavefront waits for another
// between them.  The carries are then summed in slot order by one lane per
// row, and each row's result is its hot sum plus its cold sum: every sum is
// formed in an order fixed by the matrix and the layout.  float32 matrices
// take four entries per lane (hot_part4), float64 two (hot_part).
template <typename V, bool DOT>
__global__ __launch_bounds__(kPanelThreads) void k_spmv_hot(
    HotDesc hd, const V *__restrict__ x, V *__restrict__ y, Epi epi,
    const V *__restrict__ w, double *__restrict__ dot_part)
{
    extern __shared__ __align__(16) unsigned char smem[];
    double *acc_h = (double *)smem;                                    // hot row sums
    double *acc_c = (double *)(smem + kHotRows * 8);                   // cold row sums
    double *csum = (double *)(smem + 2 * kHotRows * 8);                // 32 carries
    int32_t *ckey = (int32_t *)(smem + 2 * kHotRows * 8 + 32 * 8);     // their rows
    V *xs = (V *)(smem + kHotLdsHead);                                 // hot columns
    constexpr int VV = 16 / sizeof(V);
    typedef V vec_t __attribute__((ext_vector_type(VV)));
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const V *pv = (const V *)hd.vals;
    const int32_t width = hd.hot;
    const bool aligned = (((uintptr_t)x) & 15) == 0;
    const int32_t nvec = aligned ? width / VV : 0;
    for (int32_t i = threadIdx.x; i < nvec; i += kPanelThreads)
        *(vec_t *)(xs + i * VV) = gld((const vec_t *)(x + i * VV));
    for (int32_t e = nvec * VV + threadIdx.x; e < width; e += kPanelThreads)
        xs[e] = gld(x + e);
    for (int i = threadIdx.x; i < 2 * kHotRows; i += kPanelThreads)
        acc_h[i] = 0.0;  // both sum arrays
    double dacc = 0.0;
    // the first chunk of the wavefront's first part of block bb is requested
    // before the barriers that end the previous block
    typedef const __attribute__((address_space(4))) int32_t *cptr;
    constexpr bool Q = sizeof(V) == 4;   // float32: four entries per lane
    HotChunk<V> pre;
    HotChunk4 pre4;
    auto prefetch = [&](int32_t bb) {
        const int32_t pe0 = ((cptr)hd.bent)[bb], pes = ((cptr)hd.bsplit)[bb];
        const int32_t pe1 = ((cptr)hd.bent)[bb + 1];
        if constexpr (Q) {
            if (wave & 1)
                hot_first4<false>((const float *)pv, hd.rc, hd.key, pes, pe1, wave, lane, pre4);
            else
                hot_first4<true>((const float *)pv, hd.rc, hd.key, pe0, pes, wave, lane, pre4);
        } else {
            if (wave & 1)
                hot_first<V, false>(pv, hd.rc, hd.key, pes, pe1, wave, lane, pre);
            else
                hot_first<V, true>(pv, hd.rc, hd.key, pe0, pes, wave, lane, pre);
        }
    };
    // this workgroup's blocks (a static assignment balanced by work)
    const int32_t i0 = ((cptr)hd.gptr)[blockIdx.x];
    const int32_t i1 = ((cptr)hd.gptr)[blockIdx.x + 1];
    if (i0 < i1)
        prefetch(((cptr)hd.gblk)[i0]);
    for (int32_t i = i0; i < i1; ++i) {
        const int32_t b = ((cptr)hd.gblk)[i];
        const int32_t r0 = ((cptr)hd.brow)[b];
        const int32_t nr = ((cptr)hd.brow)[b + 1] - r0;
        const int32_t e0 = ((cptr)hd.bent)[b], es = ((cptr)hd.bsplit)[b];
        const int32_t e1 = ((cptr)hd.bent)[b + 1];
        __syncthreads();  // hot columns staged, sums of the last block cleared
        if constexpr (Q) {
            const float *fv = (const float *)pv;
            const float *fx = (const float *)x;
            const float *fs = (const float *)xs;
            if (wave & 1) {
                hot_part4<false, kPanelWaves, true, true>(
                    fv, hd.rc, hd.key, es, e1, fx, acc_c, ckey + kPanelWaves + wave,
                    csum + kPanelWaves + wave, wave, lane, &pre4);
                hot_part4<true>(fv, hd.rc, hd.key, e0, es, fs, acc_h, ckey + wave,
                                csum + wave, wave, lane);
            } else {
                hot_part4<true, kPanelWaves, false, true>(fv, hd.rc, hd.key, e0, es, fs,
                                                          acc_h, ckey + wave, csum + wave,
                                                          wave, lane, &pre4);
                hot_part4<false>(fv, hd.rc, hd.key, es, e1, fx, acc_c,
                                 ckey + kPanelWaves + wave, csum + kPanelWaves + wave,
                                 wave, lane);
            }
        } else {
            if (wave & 1) {
                hot_part<V, false, kPanelWaves, true, true>(
                    pv, hd.rc, hd.key, es, e1, x, acc_c, ckey + kPanelWaves + wave,
                    csum + kPanelWaves + wave, wave, lane, &pre);
                hot_part<V, true>(pv, hd.rc, hd.key, e0, es, xs, acc_h, ckey + wave,
                                  csum + wave, wave, lane);
            } else {
                hot_part<V, true, kPanelWaves, false, true>(pv, hd.rc, hd.key, e0, es, xs,
                                                            acc_h, ckey + wave, csum + wave,
                                                            wave, lane, &pre);
                hot_part<V, false>(pv, hd.rc, hd.key, es, e1, x, acc_c,
                                   ckey + kPanelWaves + wave, csum + kPanelWaves + wave,
                                   wave, lane);
            }
        }
        if (i + 1 < i1)
            prefetch(((cptr)hd.gblk)[i + 1]);
        __syncthreads();  // all runs are in
        if (wave == 0) {
            // lanes 0-15: hot slots, 16-31: cold slots.  A slot leads its
            // row if no earlier slot of its part has it; the leader adds the
            // row's carries of that part in slot order (distinct rows per part)
            const int32_t k = (lane < 2 * kPanelWaves) ? ckey[lane] : -1;
            const double c = (lane < 2 * kPanelWaves) ? csum[lane] : 0.0;
            const bool cold = lane >= kPanelWaves;
            bool lead = k >= 0;
            double t = 0.0;
            for (int j = 0; j < 2 * kPanelWaves; ++j) {
                const int32_t kj = __builtin_amdgcn_readlane(k, j);
                const double cj = readlane_f64(c, j);
                if ((j >= kPanelWaves) == cold && kj == k) {
                    if (j < lane)
                        lead = false;
                    else
                        t += cj;
                }
            }
            if (lead)
                (cold ? acc_c : acc_h)[k] += t;
        }
        __syncthreads();  // carries are in
        for (int32_t r = threadIdx.x; r < nr; r += kPanelThreads) {
            const uint16_t k = gld(hd.rmap + r0 + r);
            double sum = 0.0;
            if (k != kHotEmpty) {
                sum = acc_h[k] + acc_c[k];
                acc_h[k] = 0.0;  // the thread that reads a sum clears it
                acc_c[k] = 0.0;
            }
            const V out = epilogue<V>(sum, epi);
            gst(y + r0 + r, out);
            if (DOT)
                dacc = fma((double)gld(w + r0 + r), (double)out, dacc);
        }
    }
    if (DOT) {
        const double tot = block_sum<kPanelWaves>(dacc, csum);
        if (threadIdx.x == 0)
            dot_part[blockIdx.x] = tot;
    }
}

// ------------------------------------------------------------- band

// Product over the band layout (see BandDesc): one workgroup per row block,
// its wavefronts share the block's entries evenly (a row can span them),
// gather from x starting at the block's first column, and the carries of
// rows split between wavefronts are added in slot order by one lane each.
template <typename V, bool DOT>
__device__ __forceinline__ void band_block(const BandDesc &bd, int32_t b,
                                           const V *__restrict__ x,
                                           V *__restrict__ y, const Epi &epi,
                                           const V *__restrict__ w,
                                           double *__restrict__ dot_part,
                                           unsigned char *smem)
{
    double *acc = (double *)smem;                                  // row sums
    double *csum = (double *)(smem + kBandRows * 8);               // carries
    int32_t *ckey = (int32_t *)(smem + kBandRows * 8 + kBandWaves * 8);
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int32_t r0 = gld(bd.brow + b);
    const int32_t nr = gld(bd.brow + b + 1) - r0;
    for (int32_t i = threadIdx.x; i < nr; i += kBandThreads)
        acc[i] = 0.0;
    __syncthreads();
    hot_part<V, true, kBandWaves, true>((const V *)bd.vals, bd.rc, nullptr,
                                  gld(bd.bent + b), gld(bd.bent + b + 1),
                                  x + gld(bd.cbase + b), acc, ckey + wave,
                                  csum + wave, wave, lane);
    __syncthreads();
    if (wave == 0) {
        const int32_t k = (lane < kBandWaves) ? ckey[lane] : -1;
        const double c = (lane < kBandWaves) ? csum[lane] : 0.0;
        bool lead = k >= 0;
        double t = 0.0;
        for (int j = 0; j < kBandWaves; ++j) {
            const int32_t kj = __builtin_amdgcn_readlane(k, j);
            const double cj = readlane_f64(c, j);
            if (kj == k) {
                if (j < lane)
                    lead = false;
                else
                    t += cj;
            }
        }
        if (lead)
            acc[k] += t;
    }
    __syncthreads();
    double dacc = 0.0;
    for (int32_t i = threadIdx.x; i < nr; i += kBandThreads) {
        const V out = epilogue<V>(acc[i], epi);
        gst(y + r0 + i, out);
        if (DOT)
            dacc = fma((double)gld(w + r0 + i), (double)out, dacc);
    }
    if (DOT) {
        const double tot = block_sum<kBandWaves>(dacc, csum);
        if (threadIdx.x == 0)
            dot_part[b] = tot;
    }
}

template <typename V, bool DOT>
__global__ __launch_bounds__(kBandThreads) void k_spmv_band(
    BandDesc bd, const V *__restrict__ x, V *__restrict__ y, Epi epi,
    const V *__restrict__ w, double *__restrict__ dot_part)
{
    __shared__ __align__(16) unsigned char smem[kBandLds];
    band_block<V, DOT>(bd, blockIdx.x, x, y, epi, w, dot_part, smem);
}

// Band products of many matrices in one launch: workgroup g takes row
// block g - prefix[j] of matrix j, exactly as its single launch does.
template <typename V>
__global__ __launch_bounds__(kBandThreads) void k_spmv_band_grouped(
    const BandDesc *__restrict__ descs, const PanelIO *__restrict__ io,
    const int32_t *__restrict__ prefix, int32_t nmat)
{
    __shared__ __align__(16) unsigned char smem[kBandLds];
    const int32_t g = blockIdx.x;
    int32_t lo = 0, hi = nmat - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= g)
            lo = mid;
        else
            hi = mid - 1;
    }
    const BandDesc bd = descs[lo];
    const Epi epi{EPI_NONE, 0, 0.0, 0.0};
    const PanelIO bio = io[lo];
    if constexpr (sizeof(V) == 8) {
        if (bio.dot) {
            band_block<V, true>(bd, g - prefix[lo], (const V *)bio.x, (V *)bio.y, epi,
                                (const V *)bio.x, bio.dot, smem);
            return;
        }
    }
    band_block<V, false>(bd, g - prefix[lo], (const V *)bio.x, (V *)bio.y, epi,
                         nullptr, nullptr, smem);
}

// Smallest and largest column of every row (INT_MAX / -1 for empty rows).
__global__ __launch_bounds__(kBlock) void k_row_span(int32_t rows,
                                                     const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ col,
                                                     int32_t *__restrict__ lo,
                                                     int32_t *__restrict__ hi)
{
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= rows)
        return;
    int32_t a = INT_MAX, z = -1;
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
        a = min(a, col[k]);
        z = max(z, col[k]);
    }
    lo[i] = a;
    hi[i] = z;
}

// Band words of every entry: (row in block << 16) | (col - block's base).
__global__ __launch_bounds__(kBlock) void k_band_pack(BandDesc bd,
                                                      const int32_t *__restrict__ rp,
                                                      const int32_t *__restrict__ col,
                                                      uint32_t *__restrict__ rc)
{
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= bd.rows)
        return;
    int32_t lo = 0, hi = bd.nblk - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (bd.brow[mid] <= i)
            lo = mid;
        else
            hi = mid - 1;
    }
    const uint32_t rl = (uint32_t)(i - bd.brow[lo]);
    const int32_t base = bd.cbase[lo];
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
        rc[k] = (rl << 16) | (uint32_t)(col[k] - base);
}

// Hot entries of each row: one wavefront per row, 64 entries at a time.
__global__ __launch_bounds__(kBlock) void k_hot_count(HotDesc hd,
                                                      const int32_t *__restrict__ rp,
                                                      const int32_t *__restrict__ col,
                                                      int32_t *__restrict__ cnt)
{
    const int64_t i = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (i >= hd.rows)
        return;  // whole wavefronts
    int32_t n = 0;
    for (int32_t k = rp[i] + lane; k < rp[i + 1]; k += 64)
        n += (col[k] < hd.hot) ? 1 : 0;
    n = wave_sum_i32(n);
    if (lane == 0)
        cnt[i] = n;
}

__global__ __launch_bounds__(kBlock) void k_hot_split(HotDesc hd,
                                                      const int32_t *__restrict__ hx,
                                                      int32_t *__restrict__ bsplit)
{
    const int32_t b = blockIdx.x * kBlock + threadIdx.x;
    if (b >= hd.nblk)
        return;
    bsplit[b] = hd.bent[b] + (hx[hd.brow[b + 1]] - hx[hd.brow[b]]);
}

// Move each row's entries to the hot or cold part of its block (order kept
// inside a row): one wavefront per row, positions from ballots.  hx:
// exclusive scan of the per-row hot counts.
template <typename V>
__global__ __launch_bounds__(kBlock) void k_hot_scatter(
    HotDesc hd, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
    const V *__restrict__ vals, const int32_t *__restrict__ hx,
    V *__restrict__ hv, uint32_t *__restrict__ hrc, uint16_t *__restrict__ hkey)
{
    const int64_t iw = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (iw >= hd.rows)
        return;  // whole wavefronts
    const int32_t i = (int32_t)iw;
    // block of row i: the last b with brow[b] <= i
    int32_t lo = 0, hi = hd.nblk - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (hd.brow[mid] <= i)
            lo = mid;
        else
            hi = mid - 1;
    }
    const int32_t b = lo;
    const uint32_t rl = hd.rmap[i];   // used only if the row has entries
    const int32_t before = hx[i] - hx[hd.brow[b]];   // hot entries of earlier rows
    int32_t hp = hd.bent[b] + before;
    int32_t cp = hd.bsplit[b] + (rp[i] - hd.bent[b]) - before;
    const int32_t e = rp[i + 1];
    for (int32_t base = rp[i]; base < e; base += 64) {
        const int32_t k = base + lane;
        const bool in = k < e;
        const int32_t c = in ? col[k] : 0;
        const bool hot = in && c < hd.hot;
        const uint64_t mh = __ballot(hot), mc = __ballot(in && !hot);
        if (hot) {
            const int32_t pos = hp + lanes_below(mh);
            hv[pos] = vals[k];
            hrc[pos] = (rl << 16) | (uint32_t)c;
        } else if (in) {
            const int32_t pos = cp + lanes_below(mc);
            hv[pos] = vals[k];
            hrc[pos] = (uint32_t)c;
            hkey[pos] = (uint16_t)rl;
        }
        hp += __popcll(mh);
        cp += __popcll(mc);
    }
}

// ------------------------------------------------------------------ BFS

// Rows of a tile, W lanes per row, Boolean (or, and) product against the
// current frontier {u : level[u] == depth}.
template <int W>
__device__ __forceinline__ void bfs_rows(const MatDesc &m, const Tile &t,
                                         int32_t *__restrict__ level,
                                         int32_t depth, int32_t *changed)
{
    constexpr int G = kBlock / W;
    const int g = threadIdx.x / W;
    const int lane = threadIdx.x % W;
    for (int j = g; j < t.count; j += G) {
        const int32_t row = tile_row(m, t, j);
        if (level[row] != -1)
            continue;  // uniform over the group
        const int32_t k0 = m.row_ptr[row], k1 = m.row_ptr[row + 1];
        int32_t hit = 0;
        for (int32_t k = k0 + lane; k < k1 && !hit; k += W)
            hit = (level[m.col[k]] == depth) ? 1 : 0;
        hit = lane_group_or<W>(hit);
        if (hit && lane == 0) {
            level[row] = depth + 1;
            *changed = 1;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_bfs_step(
    const Tile *__restrict__ tiles, int32_t ntiles, MatDesc m,
    int32_t *__restrict__ level, int32_t depth, int32_t *__restrict__ changed)
{
    for (int32_t ti = blockIdx.x; ti < ntiles; ti += gridDim.x) {
        const Tile t = tiles[ti];
        switch (t.cls & kTileClassMask) {
        case C_W1: bfs_rows<1>(m, t, level, depth, changed); break;
        case C_W2: bfs_rows<2>(m, t, level, depth, changed); break;
        case C_W4: bfs_rows<4>(m, t, level, depth, changed); break;
        case C_W8: bfs_rows<8>(m, t, level, depth, changed); break;
        case C_W16: bfs_rows<16>(m, t, level, depth, changed); break;
        case C_W32: bfs_rows<32>(m, t, level, depth, changed); break;
        case C_W64: bfs_rows<64>(m, t, level, depth, changed); break;
        case C_WG: {
            for (int j = 0; j < t.count; ++j) {
                const int32_t row = tile_row(m, t, j);
                if (level[row] != -1)
                    continue;  // uniform over the workgroup
                int32_t hit = 0;
                for (int32_t k = m.row_ptr[row] + threadIdx.x; k < m.row_ptr[row + 1];
                     k += kBlock)
                    hit |= (level[m.col[k]] == depth) ? 1 : 0;
                if (__syncthreads_or(hit) && threadIdx.x == 0) {
                    level[row] = depth + 1;
                    *changed = 1;
                }
            }
            break;
        }
        default: {  // one chunk of a split row
            const int32_t c = t.first;
            const int32_t row = m.c_row[c];
            if (level[row] != -1)
                break;
            int32_t hit = 0;
            for (int32_t k = m.c_k0[c] + threadIdx.x; k < m.c_k1[c]; k += kBlock)
                hit |= (level[m.col[k]] == depth) ? 1 : 0;
            if (__syncthreads_or(hit) && threadIdx.x == 0) {
                level[row] = depth + 1;
                *changed = 1;
            }
            break;
        }
        }
    }
}

// --------------------------------------------------- graph relabelling

__global__ __launch_bounds__(kBlock) void k_count_cols(int64_t nnz,
                                                       const int32_t *__restrict__ col,
                                                       int32_t *__restrict__ deg)
{
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < nnz;
         k += (int64_t)gridDim.x * kBlock)
        atomicAdd(&deg[col[k]], 1);
}

// key 0 holds the largest degrees (2^31..), key 31 degree 1, key 32 degree 0
__global__ __launch_bounds__(kBlock) void k_degree_keys(int32_t n,
                                                        const int32_t *__restrict__ deg,
                                                        int32_t *__restrict__ key)
{
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) {
        const int32_t d = deg[i];
        key[i] = (d <= 0) ? 32 : __clz(d);
    }
}

__global__ __launch_bounds__(kBlock) void k_key_hist(int32_t n,
                                                     const int32_t *__restrict__ key,
                                                     int32_t *__restrict__ hist,
                                                     int32_t nblk)
{
    __shared__ int32_t cnt[kDegKeys];
    if (threadIdx.x < kDegKeys)
        cnt[threadIdx.x] = 0;
    __syncthreads();
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n)
        atomicAdd(&cnt[key[i]], 1);
    __syncthreads();
    if (threadIdx.x < kDegKeys)
        hist[threadIdx.x * nblk + blockIdx.x] = cnt[threadIdx.x];
}

// Stable placement by key (same scheme as the row-class scatter).
__global__ __launch_bounds__(kBlock) void k_key_scatter(int32_t n,
                                                        const int32_t *__restrict__ key,
                                                        const int32_t *__restrict__ hist,
                                                        int32_t nblk,
                                                        int32_t *__restrict__ newid)
{
    __shared__ int32_t wcnt[kWaves][kDegKeys];
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int32_t c = (i < n) ? key[i] : -1;
    const unsigned long long below = (lane == 0) ? 0ull : ((1ull << lane) - 1ull);
    int32_t rank = 0;
    for (int b = 0; b < kDegKeys; ++b) {
        const unsigned long long m = __ballot(c == b);
        if (lane == 0)
            wcnt[wave][b] = __popcll(m);
        if (c == b)
            rank = __popcll(m & below);
    }
    __syncthreads();
    if (c >= 0) {
        int32_t off = hist[c * nblk + blockIdx.x];
        for (int w = 0; w < wave; ++w)
            off += wcnt[w][c];
        newid[i] = off + rank;
    }
}

__global__ __launch_bounds__(kBlock) void k_perm_lengths(int32_t rows,
                                                         const int32_t *__restrict__ rp,
                                                         const int32_t *__restrict__ newid,
                                                         int32_t *__restrict__ len2)
{
    const int32_t v = blockIdx.x * kBlock + threadIdx.x;
    if (v < rows)
        len2[newid[v]] = rp[v + 1] - rp[v];
    else if (v == rows)
        len2[rows] = 0;
}

// One thread per entry: its row by binary search in row_ptr.
template <typename V>
__global__ __launch_bounds__(kBlock) void k_perm_entries(
    int32_t rows, int64_t nnz, const int32_t *__restrict__ rp,
    const int32_t *__restrict__ col, const V *__restrict__ vals,
    const int32_t *__restrict__ newid, const int32_t *__restrict__ rp2,
    int32_t *__restrict__ col2, V *__restrict__ vals2)
{
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < nnz;
         k += (int64_t)gridDim.x * kBlock) {
        int32_t lo = 0, hi = rows;  // rp[lo] <= k < rp[hi]
        while (hi - lo > 1) {
            const int32_t mid = (lo + hi) >> 1;
            if (rp[mid] <= k)
                lo = mid;
            else
                hi = mid;
        }
        const int64_t dst = (int64_t)rp2[newid[lo]] + (k - rp[lo]);
        col2[dst] = newid[col[k]];
        vals2[dst] = vals[k];
    }
}

__global__ __launch_bounds__(kBlock) void k_permute_f32(int32_t n,
                                                        const int32_t *__restrict__ newid,
                                                        const float *__restrict__ in,
                                                        float *__restrict__ out, int to)
{
    const int32_t v = blockIdx.x * kBlock + threadIdx.x;
    if (v < n) {
        if (to)
            out[newid[v]] = in[v];
        else
            out[v] = in[newid[v]];
    }
}

// ------------------------------------------------------------------ JDS

// Thread p handles the row at JDS position p: diagonal j holds its j-th
// entry at jd_ptr[j] + p, so consecutive threads read consecutive entries.
// Entries outside [0, nnz) and diagonals past max_len are never touched,
// whatever the arrays hold; a position whose original row is unknown (perm
// not a permutation) is not stored.
__global__ __launch_bounds__(kBlock) void k_spmv_jds(
    int32_t rows, int32_t max_len, int32_t nnz, const int32_t *__restrict__ iperm,
    const int32_t *__restrict__ nzcnt, const int32_t *__restrict__ jd_ptr,
    const int32_t *__restrict__ jd_col, const double *__restrict__ jd_val,
    const double *__restrict__ x, double *__restrict__ y)
{
#pragma clang fp contract(off)
    const int32_t p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= rows)
        return;
    const int32_t n = min(nzcnt[p], max_len);
    double s = 0.0;
    for (int32_t j = 0; j < n; ++j) {
        const int32_t k = jd_ptr[j] + p;
        if (k < 0 || k >= nnz)
            break;
        const double prod = jd_val[k] * x[jd_col[k]];
        s = s + prod;
    }
    const int32_t i = iperm[p];
    if (i >= 0 && i < rows)
        y[i] = s;
}

__global__ __launch_bounds__(kBlock) void k_invert_perm(
    int32_t rows, const int32_t *__restrict__ perm, int32_t *__restrict__ iperm)
{
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < rows) {
        const int32_t q = perm[i];
        if (q >= 0 && q < rows)
            iperm[q] = i;
    }
}

// ---------------------------------------------------------- batched CG

// Segment of workgroup blockIdx.x (segments ordered by blk0).
__device__ __forceinline__ int32_t cg_seg_of(const CgSeg *__restrict__ segs,
                                             int32_t nseg)
{
    int32_t lo = 0, hi = nseg;
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (segs[mid].blk0 <= (int32_t)blockIdx.x)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// Sum of part[0..n) (n <= kBlock) by one workgroup, the same in every
// workgroup that calls it.
__device__ __forceinline__ double sum_small(const double *__restrict__ part,
                                            int32_t n, double *lds)
{
    const double v = ((int32_t)threadIdx.x < n) ? part[threadIdx.x] : 0.0;
    return block_sum<kWaves>(v, lds);
}

__global__ __launch_bounds__(kBlock) void k_cgb_init(const CgSeg *__restrict__ segs,
                                                     int32_t nseg)
{
    __shared__ double lds[kWaves];
    const CgSeg sg = segs[cg_seg_of(segs, nseg)];
    const int32_t lb = blockIdx.x - sg.blk0;
    double acc = 0.0;
    for (int64_t i = (int64_t)lb * kBlock + threadIdx.x; i < sg.n;
         i += (int64_t)sg.nb * kBlock) {
        const double bi = sg.b[i];
        sg.x[i] = 0.0;
        sg.r[i] = bi;
        sg.p[i] = 0.0;
        sg.s[i] = 0.0;
        acc = fma(bi, bi, acc);
    }
    const double t = block_sum<kWaves>(acc, lds);
    if (threadIdx.x == 0) {
        sg.rr_part[lb] = t;  // parity of iteration 0
        if (lb == 0)
            *sg.done = 0;
    }
}

// Partial sums of r.w after the product w = A r (segments whose product
// wrote them, nrw > 0, are skipped).
__global__ __launch_bounds__(kBlock) void k_cgb_rw(const CgSeg *__restrict__ segs,
                                                   int32_t nseg)
{
    __shared__ double lds[kWaves];
    const CgSeg sg = segs[cg_seg_of(segs, nseg)];
    if (sg.nrw > 0)
        return;   // the product wrote them
    const int32_t lb = blockIdx.x - sg.blk0;
    double acc = 0.0;
    for (int64_t i = (int64_t)lb * kBlock + threadIdx.x; i < sg.n;
         i += (int64_t)sg.nb * kBlock)
        acc = fma(sg.r[i], sg.w[i], acc);
    const double t = block_sum<kWaves>(acc, lds);
    if (threadIdx.x == 0)
        sg.rw_part[lb] = t;
}

// gamma = r.r, delta = r.w; beta = gamma / gamma_old (0 at k = 0),
// p.Ap = delta - beta gamma / alpha_old, alpha = gamma / p.Ap; then
// p = r + beta p, s = w + beta s, x += alpha p, r -= alpha s and the
// partial sums of the new r.r.
__global__ __launch_bounds__(kBlock) void k_cgb_step(const CgSeg *__restrict__ segs,
                                                     int32_t nseg)
{
    __shared__ double lds[kWaves];
    const CgSeg sg = segs[cg_seg_of(segs, nseg)];
    if (*sg.done)
        return;
    const int32_t lb = blockIdx.x - sg.blk0;
    const int par = sg.iter & 1;
    const double g = sum_small(sg.rr_part + par * sg.nb, sg.nb, lds);
    const double d = sum_small(sg.rw_part, sg.nrw > 0 ? sg.nrw : sg.nb, lds);
    const double beta = (sg.iter > 0) ? g / sg.sc[par ^ 1] : 0.0;
    const double pap = (sg.iter > 0) ? d - beta * g / sg.sc[2 + (par ^ 1)] : d;
    if (g == 0.0 || pap == 0.0) {
        if (lb == 0 && threadIdx.x == 0)
            *sg.done = 1;
        return;
    }
    const double alpha = g / pap;
    double acc = 0.0;
    for (int64_t i = (int64_t)lb * kBlock + threadIdx.x; i < sg.n;
         i += (int64_t)sg.nb * kBlock) {
        const double ri = sg.r[i];
        const double pi = fma(beta, sg.p[i], ri);
        const double si = fma(beta, sg.s[i], sg.w[i]);
        sg.p[i] = pi;
        sg.s[i] = si;
        sg.x[i] = fma(alpha, pi, sg.x[i]);
        const double rn = fma(-alpha, si, ri);
        sg.r[i] = rn;
        acc = fma(rn, rn, acc);
    }
    const double t = block_sum<kWaves>(acc, lds);
    if (threadIdx.x == 0) {
        sg.rr_part[(par ^ 1) * sg.nb + lb] = t;
        if (lb == 0) {
            sg.sc[par] = g;
            sg.sc[2 + par] = alpha;
        }
    }
}

// ---------------------------------------------------------------- analysis

__global__ __launch_bounds__(kBlock) void k_validate(
    int32_t rows, const int32_t *__restrict__ rp, int64_t nnz,
    const int32_t *__restrict__ col, int32_t cols_given,
    int32_t *__restrict__ status)
{
    int32_t flags = 0, mx = -1;
    const int64_t tid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = tid; i < rows; i += stride)
        if (rp[i + 1] < rp[i])
            flags |= 2;
    if (tid == 0) {
        if (rp[0] != 0)
            flags |= 1;
        if ((int64_t)rp[rows] != nnz)
            flags |= 4;
    }
    for (int64_t k = tid; k < nnz; k += stride) {
        const int32_t c = col[k];
        if (c < 0 || (cols_given >= 0 && c >= cols_given))
            flags |= 8;
        mx = max(mx, c);
    }
    flags = lane_group_or<64>(flags);
    mx = lane_group_max<64>(mx);
    if ((threadIdx.x & 63) == 0) {
        if (flags)
            atomicOr(&status[0], flags);
        atomicMax(&status[1], mx);
    }
}

// Class of a row = number of class bounds it exceeds (bounds ascending), i.e.
// the first class whose inclusive upper bound holds it.
__device__ __forceinline__ int32_t row_class(int32_t len, const Thresholds &th)
{
    int32_t c = 0;
#pragma unroll
    for (int b = 0; b < NCLASS - 1; ++b)
        c += (len > th.upper[b]) ? 1 : 0;
    return c;
}

// hist is class-major: hist[c * nblk + block] = rows of class c in block.
__global__ __launch_bounds__(kBlock) void k_bin_count(
    int32_t rows, const int32_t *__restrict__ rp, Thresholds th,
    int32_t *__restrict__ hist, int32_t nblk)
{
    __shared__ int32_t cnt[NCLASS];
    if (threadIdx.x < NCLASS)
        cnt[threadIdx.x] = 0;
    __syncthreads();
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < rows)
        atomicAdd(&cnt[row_class(rp[i + 1] - rp[i], th)], 1);
    __syncthreads();
    if (threadIdx.x < NCLASS)
        hist[threadIdx.x * nblk + blockIdx.x] = cnt[threadIdx.x];
}

// Stable scatter: after the exclusive scan, hist[c*nblk+b] is where block
// b's rows of class c start; inside the block rows keep ascending order
// (wave by wave, lane by lane, ranks from ballots).
__global__ __launch_bounds__(kBlock) void k_bin_scatter(
    int32_t rows, const int32_t *__restrict__ rp, Thresholds th,
    const int32_t *__restrict__ hist, int32_t nblk,
    int32_t *__restrict__ bin_rows)
{
    __shared__ int32_t wcnt[kWaves][NCLASS];
    const int32_t i = blockIdx.x * kBlock + threadIdx.x;
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int32_t c = (i < rows) ? row_class(rp[i + 1] - rp[i], th) : -1;
    const unsigned long long below = (lane == 0) ? 0ull : ((1ull << lane) - 1ull);
    int32_t rank = 0;
#pragma unroll
    for (int b = 0; b < NCLASS; ++b) {
        const unsigned long long m = __ballot(c == b);
        if (lane == 0)
            wcnt[wave][b] = __popcll(m);
        if (c == b)
            rank = __popcll(m & below);
    }
    __syncthreads();
    if (c >= 0) {
        int32_t off = hist[c * nblk + blockIdx.x];
        for (int w = 0; w < wave; ++w)
            off += wcnt[w][c];
        bin_rows[off + rank] = i;
    }
}

// Exclusive prefix sum of a[0..n) in place by one 1024-thread workgroup;
// *total (if non-null) receives the sum.
__global__ __launch_bounds__(1024) void k_scan_excl(int32_t *__restrict__ a,
                                                    int64_t n,
                                                    int32_t *__restrict__ total)
{
    __shared__ int32_t s[1024];
    int32_t carry = 0;
    for (int64_t base = 0; base < n; base += 1024) {
        const int64_t i = base + threadIdx.x;
        const int32_t v = (i < n) ? a[i] : 0;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const int32_t t = ((int)threadIdx.x >= off) ? s[threadIdx.x - off] : 0;
            __syncthreads();
            s[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < n)
            a[i] = carry + s[threadIdx.x] - v;
        carry += s[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0 && total)
        *total = carry;
}

// Exclusive scan of 8192-element tiles of a (8 consecutive per thread); the
// tile totals go to aux[tile].
__global__ __launch_bounds__(1024) void k_scan_tiles(int32_t *__restrict__ a,
                                                     int64_t n,
                                                     int32_t *__restrict__ aux)
{
    __shared__ int32_t ws[16];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * 8192 + (int64_t)threadIdx.x * 8;
    int32_t v[8];
    int32_t t = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        v[j] = (base + j < n) ? a[base + j] : 0;
        t += v[j];
    }
    int32_t inc = t;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t u = __shfl_up(inc, o, 64);
        if (lane >= o)
            inc += u;
    }
    if (lane == 63)
        ws[wave] = inc;
    __syncthreads();
    int32_t run = inc - t;
    for (int i = 0; i < wave; ++i)
        run += ws[i];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        if (base + j < n)
            a[base + j] = run;
        run += v[j];
    }
    if (threadIdx.x == 1023)
        aux[blockIdx.x] = run;
}

// Adds the scanned tile totals to every element of the tile.
__global__ __launch_bounds__(1024) void k_scan_add(int32_t *__restrict__ a,
                                                   int64_t n,
                                                   const int32_t *__restrict__ aux)
{
    const int32_t add = aux[blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * 8192;
    for (int j = threadIdx.x; j < 8192; j += 1024)
        if (base + j < n)
            a[base + j] += add;
}

__global__ __launch_bounds__(kBlock) void k_chunk_count(
    int32_t nsplit, const int32_t *__restrict__ split_rows,
    const int32_t *__restrict__ rp, int32_t chunk, int32_t *__restrict__ cnt)
{
    const int32_t j = blockIdx.x * kBlock + threadIdx.x;
    if (j < nsplit) {
        const int32_t r = split_rows[j];
        const int64_t len = (int64_t)rp[r + 1] - rp[r];
        cnt[j] = (int32_t)((len + chunk - 1) / chunk);
    } else if (j == nsplit) {
        cnt[j] = 0;
    }
}

__global__ __launch_bounds__(kBlock) void k_chunk_fill(
    int32_t nsplit, const int32_t *__restrict__ split_rows,
    const int32_t *__restrict__ rp, int32_t chunk,
    const int32_t *__restrict__ s_first, int32_t *__restrict__ c_row,
    int32_t *__restrict__ c_k0, int32_t *__restrict__ c_k1)
{
    const int32_t j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= nsplit)
        return;
    const int32_t r = split_rows[j];
    const int64_t a = rp[r], e = rp[r + 1];
    int32_t c = s_first[j];
    for (int64_t k = a; k < e; k += chunk, ++c) {
        c_row[c] = r;
        c_k0[c] = (int32_t)k;
        c_k1[c] = (int32_t)((e - k > chunk) ? k + chunk : e);
    }
}

__global__ __launch_bounds__(kBlock) void k_fill_i32(int32_t *__restrict__ p,
                                                     int64_t n, int32_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        p[i] = v;
}

__global__ __launch_bounds__(kBlock) void k_fill_f64(double *__restrict__ p, int64_t n,
                                                     double v)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        p[i] = v;
}

__global__ __launch_bounds__(kBlock) void k_zero_bytes(
    unsigned char *__restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        p[i] = 0;
}

// ---------------------------------------------------------------- BLAS-1

// Sum of part[0..n) by a 1024-thread workgroup in a fixed order.
__device__ __forceinline__ double sum_parts_1024(const double *__restrict__ part,
                                                 int32_t n, double *lds)
{
    double acc = 0.0;
    for (int32_t i = threadIdx.x; i < n; i += 1024)
        acc += part[i];
    return block_sum<16>(acc, lds);
}

// Partial dot products, one per workgroup (float32 data is widened exactly
// and accumulated in binary64).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_dot_parts(
    int64_t n, const T *__restrict__ a, const T *__restrict__ b,
    double *__restrict__ part)
{
    __shared__ double lds[kWaves];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        acc = fma((double)a[i], (double)b[i], acc);
    const double t = block_sum<kWaves>(acc, lds);
    if (threadIdx.x == 0)
        part[blockIdx.x] = t;
}

// The total of the partials, stored as TOut: a float32 result is the
// binary64 total rounded once.
template <typename TOut>
__global__ __launch_bounds__(1024) void k_sum_parts(
    const double *__restrict__ part, int32_t n, TOut *__restrict__ out)
{
    __shared__ double lds[16];
    const double t = sum_parts_1024(part, n, lds);
    if (threadIdx.x == 0)
        *out = (TOut)t;
}

// HBM stream ceiling: every 16-byte piece of src read once with
// non-temporal loads, U pieces per thread in flight; with dst, each piece is
// also stored there (a copy).  The read-only form folds the data into a
// value that is stored only if it equals a constant nothing in practice
// produces, so the loads stay.  Workgroup g streams the contiguous range of
// pieces [g * per, (g + 1) * per).
template <int U, bool COPY>
__global__ __launch_bounds__(kBlock) void k_stream(const i32x4 *__restrict__ src,
                                                   i32x4 *__restrict__ dst, int64_t n,
                                                   int64_t per, uint32_t *__restrict__ sink)
{
    const int64_t lo = (int64_t)blockIdx.x * per;
    const int64_t hi = min(n, lo + per);
    int32_t fold = 0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += (int64_t)U * kBlock) {
        i32x4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t k = i + (int64_t)u * kBlock;
            v[u] = (k < hi) ? ld_stream(src + k) : i32x4{0, 0, 0, 0};
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t k = i + (int64_t)u * kBlock;
            if (COPY) {
                if (k < hi)
                    __builtin_nontemporal_store(
                        v[u], (__attribute__((address_space(1))) i32x4 *)(dst + k));
            } else {
                fold ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
            }
        }
    }
    if (!COPY && fold == (int32_t)0x9E3779B9)
        sink[0] = (uint32_t)fold;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_copy(int64_t n,
                                                 const T *__restrict__ src,
                                                 T *__restrict__ dst)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock)
        dst[i] = src[i];
}

// Conjugate gradient in the arrangement of Chronopoulos and Gear (1989):
// the same iterates as the textbook loop in exact arithmetic, with both
// inner products of an iteration (r.r and r.Ar) available together, so an
// iteration is one product w = A r (with the partials of w.r fused into it)
// and one vector kernel.  Recurrences (s = A p kept alongside p):
//   gamma = r.r, delta = w.r, beta = gamma / gamma_old (0 at first),
//   p.Ap = delta - beta * gamma / alpha_old, alpha = gamma / p.Ap,
//   p = r + beta p, s = w + beta s, x += alpha p, r -= alpha s.
// The scalars of iteration k go to slot k & 1 of gamma[] and alpha[], so an
// iteration reads the previous slot while it writes its own.

// Start: x = 0, r = b, p = s = 0, partial sums of b.b into rr (parity 0).
__global__ __launch_bounds__(kBlock) void k_cg_init(
    int64_t n, const double *__restrict__ b, double *__restrict__ x,
    double *__restrict__ r, double *__restrict__ p, double *__restrict__ sv,
    double *__restrict__ rr, CgScalars *__restrict__ sc)
{
    __shared__ double lds[kWaves];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kBlock) {
        const double bi = b[i];
        x[i] = 0.0;
        r[i] = bi;
        p[i] = 0.0;
        sv[i] = 0.0;
        acc = fma(bi, bi, acc);
    }
    const double t = block_sum<kWaves>(acc, lds);
    if (threadIdx.x == 0) {
        rr[blockIdx.x] = t;
        if (blockIdx.x == 0) {
            sc->rho = 0.0;
            sc->gamma[0] = sc->gamma[1] = 1.0;
            sc->alpha[0] = sc->alpha[1] = 1.0;
            sc->done = 0;
            sc->iters = 0;
        }
    }
}

// Sums of two values over the workgroup at once, each in the order of
// block_sum (so each equals block_sum of that value).
__device__ __forceinline__ void block_sum2(double &a, double &b, double *lds)
{
    a = lane_group_sum<64>(a);
    b = lane_group_sum<64>(b);
    __syncthreads();  // earlier readers of lds are done
    if ((threadIdx.x & 63) == 0) {
        lds[threadIdx.x >> 6] = a;
        lds[kWaves + (threadIdx.x >> 6)] = b;
    }
    __syncthreads();
    double ta = lds[0], tb = lds[kWaves];
#pragma unroll
    for (int i = 1; i < kWaves; ++i) {
        ta += lds[i];
        tb += lds[kWaves + i];
    }
    a = ta;
    b = tb;
}

// Iteration k (slot par = k & 1), after w = A r with the w.r partials in
// dot_part: every workgroup forms gamma, delta, beta and alpha itself, in
// the same order; the solve stops (x kept) when gamma or p.Ap is exactly 0.
// Each thread's first elements are read before the sums, so their loads
// overlap; the partials of the new r.r go to rr[par ^ 1].
__global__ __launch_bounds__(kBlock) void k_cg_step(
    int64_t n, CgScalars *__restrict__ sc, const double *__restrict__ w,
    double *__restrict__ p, double *__restrict__ sv, double *__restrict__ x,
    double *__restrict__ r, const double *__restrict__ dot_part, int32_t ndot,
    double *__restrict__ rr, int32_t nparts, int32_t k)
{
    __shared__ double lds[2 * kWaves];
    const int32_t par = k & 1;
    const int64_t i0 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t step = (int64_t)gridDim.x * kBlock;
    double w0 = 0.0, p0 = 0.0, s0 = 0.0, x0 = 0.0, r0 = 0.0;
    if (i0 < n) {
        w0 = w[i0];
        p0 = p[i0];
        s0 = sv[i0];
        x0 = x[i0];
        r0 = r[i0];
    }
    const int32_t done = sc->done;
    const double g_old = sc->gamma[par ^ 1], a_old = sc->alpha[par ^ 1];
    double g = 0.0, d = 0.0;
    for (int32_t i = threadIdx.x; i < nparts; i += kBlock)
        g += rr[par * kDotParts + i];
    for (int32_t i = threadIdx.x; i < ndot; i += kBlock)
        d += dot_part[i];
    if (done)
        return;
    block_sum2(g, d, lds);
    const double beta = (k > 0) ? g / g_old : 0.0;
    const double pap = d - beta * g / a_old;
    if (g == 0.0 || pap == 0.0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            sc->done = 1;
            sc->rho = g;
        }
        return;
    }
    const double alpha = g / pap;
    double acc = 0.0;
    if (i0 < n) {
        const double pi = fma(beta, p0, r0);
        const double si = fma(beta, s0, w0);
        p[i0] = pi;
        sv[i0] = si;
        x[i0] = fma(alpha, pi, x0);
        const double ri = fma(-alpha, si, r0);
        r[i0] = ri;
        acc = ri * ri;
    }
    for (int64_t i = i0 + step; i < n; i += step) {
        const double pi = fma(beta, p[i], r[i]);
        const double si = fma(beta, sv[i], w[i]);
        p[i] = pi;
        sv[i] = si;
        x[i] = fma(alpha, pi, x[i]);
        const double ri = fma(-alpha, si, r[i]);
        r[i] = ri;
        acc = fma(ri, ri, acc);
    }
    const double t = block_sum<kWaves>(acc, lds);
    if (threadIdx.x == 0) {
        rr[(par ^ 1) * kDotParts + blockIdx.x] = t;
        if (blockIdx.x == 0) {
            sc->gamma[par] = g;
            sc->alpha[par] = alpha;
            sc->iters = k + 1;
        }
    }
}

// After the last iteration: rho = r.r of the final residual (partials in
// rr[par]), unless the solve stopped early (rho was set then).
__global__ __launch_bounds__(1024) void k_cg_final(CgScalars *__restrict__ sc,
                                                   const double *__restrict__ rr,
                                                   int32_t nparts, int32_t par)
{
    __shared__ double lds[16];
    const double t = sum_parts_1024(rr + par * kDotParts, nparts, lds);
    if (threadIdx.x == 0 && !sc->done)
        sc->rho = t;
}

inline int32_t grid_for(int64_t n, int32_t per_block, int32_t cap)
{
    int64_t g = (n + per_block - 1) / per_block;
    if (g < 1)
        g = 1;
    if (g > cap)
        g = cap;
    return (int32_t)g;
}

inline void check_launch(const char *what)
{
    hip_check(hipGetLastError(), what, __FILE__, __LINE__);
}

}  // namespace

// ------------------------------------------------------------- launchers

int32_t blas1_parts(int64_t n) { return grid_for(n, kBlock, kDotParts); }

int occupancy_tiles(lilac_dtype dt)
{
    int n = 0;
    hipError_t e = (dt == LILAC_F64)
        ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
              &n, k_spmv_tiles<double, true, false>, kBlock, 0)
        : hipOccupancyMaxActiveBlocksPerMultiprocessor(
              &n, k_spmv_tiles<float, true, false>, kBlock, 0);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return n;
}

void launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s)
{
    if (n <= 0)
        return;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n, kBlock, 4096)),
                       dim3(kBlock), 0, s, p, n, v);
    check_launch("k_fill_i32");
}

void launch_fill_f64(double *p, int64_t n, double v, hipStream_t s)
{
    if (n <= 0)
        return;
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(n, kBlock, 4096)), dim3(kBlock), 0, s, p,
                       n, v);
    check_launch("k_fill_f64");
}

void launch_fill_bytes_zero(void *p, int64_t bytes, hipStream_t s)
{
    if (bytes <= 0)
        return;
    hipLaunchKernelGGL(k_zero_bytes, dim3(grid_for(bytes, kBlock, 4096)),
                       dim3(kBlock), 0, s, (unsigned char *)p, bytes);
    check_launch("k_zero_bytes");
}

void launch_validate(int32_t rows, const int32_t *rp, int64_t nnz,
                     const int32_t *col, int32_t cols_given, int32_t *status,
                     hipStream_t s)
{
    const int64_t work = nnz > rows ? nnz : (int64_t)rows + 1;
    hipLaunchKernelGGL(k_validate, dim3(grid_for(work, kBlock * 4, 4096)),
                       dim3(kBlock), 0, s, rows, rp, nnz, col, cols_given,
                       status);
    check_launch("k_validate");
}

void launch_bin_count(int32_t rows, const int32_t *rp, const Thresholds &th,
                      int32_t *hist, int32_t nblk, hipStream_t s)
{
    hipLaunchKernelGGL(k_bin_count, dim3(nblk), dim3(kBlock), 0, s, rows, rp,
                       th, hist, nblk);
    check_launch("k_bin_count");
}

void launch_scan_excl(int32_t *a, int64_t n, int32_t *total, hipStream_t s)
{
    if (n <= 65536) {
        hipLaunchKernelGGL(k_scan_excl, dim3(1), dim3(1024), 0, s, a, n, total);
        check_launch("k_scan_excl");
        return;
    }
    // tiles of 8192, then the tile totals, then the offsets back into the tiles
    const int64_t nt = (n + 8191) / 8192;
    if (nt > INT32_MAX)
        fail(LILAC_ERR_ARG, "scan too long");
    int32_t *aux = (int32_t *)dev_alloc((size_t)nt * 4);
    hipLaunchKernelGGL(k_scan_tiles, dim3((uint32_t)nt), dim3(1024), 0, s, a, n, aux);
    check_launch("k_scan_tiles");
    hipLaunchKernelGGL(k_scan_excl, dim3(1), dim3(1024), 0, s, aux, nt, total);
    check_launch("k_scan_excl");
    hipLaunchKernelGGL(k_scan_add, dim3((uint32_t)nt), dim3(1024), 0, s, a, n,
                       (const int32_t *)aux);
    check_launch("k_scan_add");
    HIPC(hipStreamSynchronize(s));
    dev_free(aux);
}

void launch_bin_scatter(int32_t rows, const int32_t *rp, const Thresholds &th,
                        const int32_t *hist, int32_t nblk, int32_t *bin_rows,
                        hipStream_t s)
{
    hipLaunchKernelGGL(k_bin_scatter, dim3(nblk), dim3(kBlock), 0, s, rows, rp,
                       th, hist, nblk, bin_rows);
    check_launch("k_bin_scatter");
}

void launch_chunk_count(int32_t nsplit, const int32_t *split_rows,
                        const int32_t *rp, int32_t chunk, int32_t *cnt,
                        hipStream_t s)
{
    hipLaunchKernelGGL(k_chunk_count, dim3(grid_for((int64_t)nsplit + 1, kBlock, INT_MAX)),
                       dim3(kBlock), 0, s, nsplit, split_rows, rp, chunk, cnt);
    check_launch("k_chunk_count");
}

void launch_chunk_fill(int32_t nsplit, const int32_t *split_rows,
                       const int32_t *rp, int32_t chunk, const int32_t *s_first,
                       int32_t *c_row, int32_t *c_k0, int32_t *c_k1,
                       hipStream_t s)
{
    if (nsplit <= 0)
        return;
    hipLaunchKernelGGL(k_chunk_fill, dim3(grid_for(nsplit, kBlock, INT_MAX)),
                       dim3(kBlock), 0, s, nsplit, split_rows, rp, chunk,
                       s_first, c_row, c_k0, c_k1);
    check_launch("k_chunk_fill");
}

void launch_spmv_tiles(lilac_dtype dt, const Tile *tiles, int32_t ntiles,
                       int32_t grid, const MatDesc &single,
                       const MatDesc *mats, const Epi &epi, double *dot_part,
                       hipStream_t s)
{
    if (ntiles <= 0 || grid <= 0)
        return;
    const bool grouped = mats != nullptr;
    const bool dot = dot_part != nullptr;
    dim3 g(grid), b(kBlock);
    if (dt == LILAC_F64) {
        if (grouped && dot)
            hipLaunchKernelGGL((k_spmv_tiles<double, true, true>), g, b, 0, s, tiles, ntiles, single, mats, epi, dot_part);
        else if (grouped)
            hipLaunchKernelGGL((k_spmv_tiles<double, true, false>), g, b, 0, s, tiles, ntiles, single, mats, epi, dot_part);
        else if (dot)
            hipLaunchKernelGGL((k_spmv_tiles<double, false, true>), g, b, 0, s, tiles, ntiles, single, mats, epi, dot_part);
        else
            hipLaunchKernelGGL((k_spmv_tiles<double, false, false>), g, b, 0, s, tiles, ntiles, single, mats, epi, dot_part);
    } else {
        if (dot)
            fail(LILAC_ERR_UNSUPPORTED, "fused dot is only provided for float64");
        if (grouped)
            hipLaunchKernelGGL((k_spmv_tiles<float, true, false>), g, b, 0, s, tiles, ntiles, single, mats, epi, dot_part);
        else
            hipLaunchKernelGGL((k_spmv_tiles<float, false, false>), g, b, 0, s, tiles, ntiles, single, mats, epi, dot_part);
    }
    check_launch("k_spmv_tiles");
}

void launch_split_finalize(lilac_dtype dt, const int32_t *items, int32_t n,
                           const MatDesc &single, const MatDesc *mats,
                           const Epi &epi, double *dot_part, hipStream_t s)
{
    if (n <= 0)
        return;
    const bool grouped = mats != nullptr;
    const bool dot = dot_part != nullptr;
    dim3 g(grid_for(n, kBlock, INT_MAX)), b(kBlock);
    if (dt == LILAC_F64) {
        if (grouped)
            hipLaunchKernelGGL((k_split_finalize<double, true, false>), g, b, 0, s, items, n, single, mats, epi, dot_part);
        else if (dot)
            hipLaunchKernelGGL((k_split_finalize<double, false, true>), g, b, 0, s, items, n, single, mats, epi, dot_part);
        else
            hipLaunchKernelGGL((k_split_finalize<double, false, false>), g, b, 0, s, items, n, single, mats, epi, dot_part);
    } else {
        if (grouped)
            hipLaunchKernelGGL((k_split_finalize<float, true, false>), g, b, 0, s, items, n, single, mats, epi, dot_part);
        else
            hipLaunchKernelGGL((k_split_finalize<float, false, false>), g, b, 0, s, items, n, single, mats, epi, dot_part);
    }
    check_launch("k_split_finalize");
}

void launch_spmv_segments(lilac_dtype dt, const MatDesc *mats,
                          const int32_t *prefix, int32_t nseg, int32_t total,
                          int32_t grid, hipStream_t s)
{
    if (total <= 0 || nseg <= 0)
        return;
    grid = std::min(grid, total);
    if (dt == LILAC_F64)
        hipLaunchKernelGGL(k_spmv_segments<double>, dim3(grid), dim3(kBlock), 0, s,
                           mats, prefix, nseg, total);
    else
        hipLaunchKernelGGL(k_spmv_segments<float>, dim3(grid), dim3(kBlock), 0, s,
                           mats, prefix, nseg, total);
    check_launch("k_spmv_segments");
}

void launch_spmv_panels(lilac_dtype dt, const PanelDesc &pd, const void *x,
                        void *y, const Epi &epi, const void *w, double *dot_part,
                        hipStream_t s)
{
    if (pd.nblk <= 0)
        return;
    dim3 g(pd.nblk), b(kPanelThreads);
    if (dt == LILAC_F64) {
        if (dot_part)
            hipLaunchKernelGGL((k_spmv_panels<double, true>), g, b, kPanelLds, s, pd,
                               (const double *)x, (double *)y, epi, (const double *)w, dot_part);
        else
            hipLaunchKernelGGL((k_spmv_panels<double, false>), g, b, kPanelLds, s, pd,
                               (const double *)x, (double *)y, epi, (const double *)w, dot_part);
    } else {
        if (dot_part)
            fail(LILAC_ERR_UNSUPPORTED, "fused dot is only provided for float64");
        hipLaunchKernelGGL((k_spmv_panels<float, false>), g, b, kPanelLds, s, pd,
                           (const float *)x, (float *)y, epi, (const float *)w, dot_part);
    }
    check_launch("k_spmv_panels");
}

void launch_spmv_panels_grouped(lilac_dtype dt, const PanelDesc *descs,
                                const PanelIO *io, const int32_t *prefix,
                                int32_t nmat, int32_t nblocks, hipStream_t s)
{
    if (nmat <= 0 || nblocks <= 0)
        return;
    dim3 g(nblocks), b(kPanelThreads);
    if (dt == LILAC_F64)
        hipLaunchKernelGGL(k_spmv_panels_grouped<double>, g, b, kPanelLds, s, descs,
                           io, prefix, nmat);
    else
        hipLaunchKernelGGL(k_spmv_panels_grouped<float>, g, b, kPanelLds, s, descs,
                           io, prefix, nmat);
    check_launch("k_spmv_panels_grouped");
}

void launch_spmv_band(lilac_dtype dt, const BandDesc &bd, const void *x, void *y,
                      const Epi &epi, const void *w, double *dot_part, hipStream_t s)
{
    if (bd.nblk <= 0)
        return;
    dim3 g(bd.nblk), b(kBandThreads);
    if (dt == LILAC_F64) {
        if (dot_part)
            hipLaunchKernelGGL((k_spmv_band<double, true>), g, b, 0, s, bd,
                               (const double *)x, (double *)y, epi, (const double *)w, dot_part);
        else
            hipLaunchKernelGGL((k_spmv_band<double, false>), g, b, 0, s, bd,
                               (const double *)x, (double *)y, epi, (const double *)w, dot_part);
    } else {
        if (dot_part)
            fail(LILAC_ERR_UNSUPPORTED, "fused dot is only provided for float64");
        hipLaunchKernelGGL((k_spmv_band<float, false>), g, b, 0, s, bd,
                           (const float *)x, (float *)y, epi, (const float *)w, dot_part);
    }
    check_launch("k_spmv_band");
}

void launch_spmv_band_grouped(lilac_dtype dt, const BandDesc *descs, const PanelIO *io,
                              const int32_t *prefix, int32_t nmat, int32_t nblocks,
                              hipStream_t s)
{
    if (nmat <= 0 || nblocks <= 0)
        return;
    dim3 g(nblocks), b(kBandThreads);
    if (dt == LILAC_F64)
        hipLaunchKernelGGL(k_spmv_band_grouped<double>, g, b, 0, s, descs, io, prefix, nmat);
    else
        hipLaunchKernelGGL(k_spmv_band_grouped<float>, g, b, 0, s, descs, io, prefix, nmat);
    check_launch("k_spmv_band_grouped");
}

void launch_row_span(int32_t rows, const int32_t *rp, const int32_t *col, int32_t *lo,
                     int32_t *hi, hipStream_t s)
{
    if (rows <= 0)
        return;
    hipLaunchKernelGGL(k_row_span, dim3(grid_for(rows, kBlock, INT_MAX)), dim3(kBlock), 0,
                       s, rows, rp, col, lo, hi);
    check_launch("k_row_span");
}

void launch_band_pack(const BandDesc &bd, const int32_t *rp, const int32_t *col,
                      uint32_t *rc, hipStream_t s)
{
    hipLaunchKernelGGL(k_band_pack, dim3(grid_for(bd.rows, kBlock, INT_MAX)), dim3(kBlock),
                       0, s, bd, rp, col, rc);
    check_launch("k_band_pack");
}

void launch_line_reuse(int32_t rows, const int32_t *rp, const int32_t *col,
                       int32_t ngroups, int32_t shift, int32_t *out, hipStream_t s)
{
    if (rows <= 0 || ngroups <= 0)
        return;
    hipLaunchKernelGGL(k_line_reuse, dim3(ngroups), dim3(kBlock), 0, s, rows, rp, col,
                       ngroups, shift, out);
    check_launch("k_line_reuse");
}

void launch_spmv_hot(lilac_dtype dt, const HotDesc &hd, const void *x, void *y,
                     const Epi &epi, const void *w, double *dot_part, hipStream_t s)
{
    if (hd.nblk <= 0 || hd.grid <= 0)
        return;
    dim3 g(hd.grid), b(kPanelThreads);
    if (dt == LILAC_F64) {
        if (dot_part)
            hipLaunchKernelGGL((k_spmv_hot<double, true>), g, b, kPanelLds, s, hd,
                               (const double *)x, (double *)y, epi, (const double *)w, dot_part);
        else
            hipLaunchKernelGGL((k_spmv_hot<double, false>), g, b, kPanelLds, s, hd,
                               (const double *)x, (double *)y, epi, (const double *)w, dot_part);
    } else {
        if (dot_part)
            fail(LILAC_ERR_UNSUPPORTED, "fused dot is only provided for float64");
        hipLaunchKernelGGL((k_spmv_hot<float, false>), g, b, kPanelLds, s, hd,
                           (const float *)x, (float *)y, epi, (const float *)w, dot_part);
    }
    check_launch("k_spmv_hot");
}

void launch_hot_count(const HotDesc &hd, const int32_t *rp, const int32_t *col,
                      int32_t *cnt, hipStream_t s)
{
    hipLaunchKernelGGL(k_hot_count, dim3(grid_for((int64_t)hd.rows * 64, kBlock, INT_MAX)),
                       dim3(kBlock), 0, s, hd, rp, col, cnt);
    check_launch("k_hot_count");
}

void launch_hot_split(const HotDesc &hd, const int32_t *hx, int32_t *bsplit,
                      hipStream_t s)
{
    hipLaunchKernelGGL(k_hot_split, dim3(grid_for(hd.nblk, kBlock, INT_MAX)),
                       dim3(kBlock), 0, s, hd, hx, bsplit);
    check_launch("k_hot_split");
}

void launch_hot_scatter(lilac_dtype dt, const HotDesc &hd, const int32_t *rp,
                        const int32_t *col, const void *vals, const int32_t *hx,
                        void *hv, uint32_t *hrc, uint16_t *hkey, hipStream_t s)
{
    dim3 g(grid_for((int64_t)hd.rows * 64, kBlock, INT_MAX)), b(kBlock);
    if (dt == LILAC_F64)
        hipLaunchKernelGGL(k_hot_scatter<double>, g, b, 0, s, hd, rp, col,
                           (const double *)vals, hx, (double *)hv, hrc, hkey);
    else
        hipLaunchKernelGGL(k_hot_scatter<float>, g, b, 0, s, hd, rp, col,
                           (const float *)vals, hx, (float *)hv, hrc, hkey);
    check_launch("k_hot_scatter");
}

void panels_prepare()
{
    static bool done = false;
    if (done)
        return;
    HIPC(hipFuncSetAttribute((const void *)k_spmv_panels_grouped<double>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, kPanelLds));
    HIPC(hipFuncSetAttribute((const void *)k_spmv_panels_grouped<float>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, kPanelLds));
    HIPC(hipFuncSetAttribute((const void *)k_spmv_hot<double, true>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, kPanelLds));
    HIPC(hipFuncSetAttribute((const void *)k_spmv_hot<double, false>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, kPanelLds));
    HIPC(hipFuncSetAttribute((const void *)k_spmv_hot<float, false>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, kPanelLds));
    HIPC(hipFuncSetAttribute((const void *)k_spmv_panels<double, true>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, kPanelLds));
    HIPC(hipFuncSetAttribute((const void *)k_spmv_panels<double, false>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, kPanelLds));
    HIPC(hipFuncSetAttribute((const void *)k_spmv_panels<float, false>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, kPanelLds));
    done = true;
}

void launch_panel_count(const PanelDesc &pd, const int32_t *rp,
                        const int32_t *col, int32_t *cnt, hipStream_t s)
{
    hipLaunchKernelGGL(k_panel_count, dim3(grid_for((int64_t)pd.rows * 64, kBlock, INT_MAX)),
                       dim3(kBlock), 0, s, pd, rp, col, cnt);
    check_launch("k_panel_count");
}

void launch_panel_scatter(lilac_dtype dt, const PanelDesc &pd, const int32_t *rp,
                          const int32_t *col, const void *vals, const int32_t *ptr,
                          void *pv, uint32_t *prc, hipStream_t s)
{
    dim3 g(grid_for((int64_t)pd.rows * 64, kBlock, INT_MAX)), b(kBlock);
    if (dt == LILAC_F64)
        hipLaunchKernelGGL(k_panel_scatter<double>, g, b, 0, s, pd, rp, col,
                           (const double *)vals, ptr, (double *)pv, prc);
    else
        hipLaunchKernelGGL(k_panel_scatter<float>, g, b, 0, s, pd, rp, col,
                           (const float *)vals, ptr, (float *)pv, prc);
    check_launch("k_panel_scatter");
}

void launch_panel_wptr(const PanelDesc &pd, const int32_t *ptr, int32_t *wptr,
                       hipStream_t s)
{
    const int64_t n = (int64_t)pd.nblk * pd.np * (kPanelWaves + 1);
    hipLaunchKernelGGL(k_panel_wptr, dim3(grid_for(n, kBlock, INT_MAX)), dim3(kBlock),
                       0, s, pd, ptr, wptr);
    check_launch("k_panel_wptr");
}

void launch_bfs_step(const Tile *tiles, int32_t ntiles, int32_t grid,
                     const MatDesc &m, int32_t *level, int32_t depth,
                     int32_t *changed, hipStream_t s)
{
    if (ntiles <= 0)
        return;
    hipLaunchKernelGGL(k_bfs_step, dim3(std::min(grid, ntiles)), dim3(kBlock), 0, s,
                       tiles, ntiles, m, level, depth, changed);
    check_launch("k_bfs_step");
}

void launch_spmv_jds(int32_t rows, int32_t max_len, int32_t nnz,
                     const int32_t *iperm, const int32_t *nzcnt,
                     const int32_t *jd_ptr, const int32_t *jd_col,
                     const double *jd_val, const double *x, double *y,
                     hipStream_t s)
{
    if (rows <= 0)
        return;
    hipLaunchKernelGGL(k_spmv_jds, dim3(grid_for(rows, kBlock, INT_MAX)), dim3(kBlock),
                       0, s, rows, max_len, nnz, iperm, nzcnt, jd_ptr, jd_col, jd_val,
                       x, y);
    check_launch("k_spmv_jds");
}

void launch_invert_perm(int32_t rows, const int32_t *perm, int32_t *iperm,
                        hipStream_t s)
{
    if (rows <= 0)
        return;
    hipLaunchKernelGGL(k_invert_perm, dim3(grid_for(rows, kBlock, INT_MAX)), dim3(kBlock),
                       0, s, rows, perm, iperm);
    check_launch("k_invert_perm");
}

void launch_count_cols(int64_t nnz, const int32_t *col, int32_t *deg, hipStream_t s)
{
    if (nnz <= 0)
        return;
    hipLaunchKernelGGL(k_count_cols, dim3(grid_for(nnz, kBlock * 8, 8192)), dim3(kBlock),
                       0, s, nnz, col, deg);
    check_launch("k_count_cols");
}

void launch_degree_keys(int32_t n, const int32_t *deg, int32_t *key, hipStream_t s)
{
    hipLaunchKernelGGL(k_degree_keys, dim3(grid_for(n, kBlock, INT_MAX)), dim3(kBlock),
                       0, s, n, deg, key);
    check_launch("k_degree_keys");
}

void launch_key_hist(int32_t n, const int32_t *key, int32_t *hist, int32_t nblk,
                     hipStream_t s)
{
    hipLaunchKernelGGL(k_key_hist, dim3(nblk), dim3(kBlock), 0, s, n, key, hist, nblk);
    check_launch("k_key_hist");
}

void launch_key_scatter(int32_t n, const int32_t *key, const int32_t *hist,
                        int32_t nblk, int32_t *newid, hipStream_t s)
{
    hipLaunchKernelGGL(k_key_scatter, dim3(nblk), dim3(kBlock), 0, s, n, key, hist,
                       nblk, newid);
    check_launch("k_key_scatter");
}

void launch_perm_lengths(int32_t rows, const int32_t *rp, const int32_t *newid,
                         int32_t *len2, hipStream_t s)
{
    hipLaunchKernelGGL(k_perm_lengths, dim3(grid_for((int64_t)rows + 1, kBlock, INT_MAX)),
                       dim3(kBlock), 0, s, rows, rp, newid, len2);
    check_launch("k_perm_lengths");
}

void launch_perm_entries(lilac_dtype dt, int32_t rows, int64_t nnz, const int32_t *rp,
                         const int32_t *col, const void *vals, const int32_t *newid,
                         const int32_t *rp2, int32_t *col2, void *vals2, hipStream_t s)
{
    if (nnz <= 0)
        return;
    dim3 g(grid_for(nnz, kBlock, 65536)), b(kBlock);
    if (dt == LILAC_F64)
        hipLaunchKernelGGL(k_perm_entries<double>, g, b, 0, s, rows, nnz, rp, col,
                           (const double *)vals, newid, rp2, col2, (double *)vals2);
    else
        hipLaunchKernelGGL(k_perm_entries<float>, g, b, 0, s, rows, nnz, rp, col,
                           (const float *)vals, newid, rp2, col2, (float *)vals2);
    check_launch("k_perm_entries");
}

void launch_permute_f32(int32_t n, const int32_t *newid, const float *in, float *out,
                        bool to, hipStream_t s)
{
    if (n <= 0)
        return;
    hipLaunchKernelGGL(k_permute_f32, dim3(grid_for(n, kBlock, INT_MAX)), dim3(kBlock), 0,
                       s, n, newid, in, out, to ? 1 : 0);
    check_launch("k_permute_f32");
}

int32_t cg_seg_blocks(int64_t n) { return grid_for(n, kBlock, kBlock); }

void launch_cgb_init(const CgSeg *segs, int32_t nseg, int32_t blocks, hipStream_t s)
{
    if (blocks <= 0)
        return;
    hipLaunchKernelGGL(k_cgb_init, dim3(blocks), dim3(kBlock), 0, s, segs, nseg);
    check_launch("k_cgb_init");
}

void launch_cgb_rw(const CgSeg *segs, int32_t nseg, int32_t blocks, hipStream_t s)
{
    if (blocks <= 0)
        return;
    hipLaunchKernelGGL(k_cgb_rw, dim3(blocks), dim3(kBlock), 0, s, segs, nseg);
    check_launch("k_cgb_rw");
}

void launch_cgb_step(const CgSeg *segs, int32_t nseg, int32_t blocks, hipStream_t s)
{
    if (blocks <= 0)
        return;
    hipLaunchKernelGGL(k_cgb_step, dim3(blocks), dim3(kBlock), 0, s, segs, nseg);
    check_launch("k_cgb_step");
}

void launch_dot_parts(int64_t n, const double *a, const double *b,
                      double *part, int32_t nparts, hipStream_t s)
{
    hipLaunchKernelGGL(k_dot_parts<double>, dim3(nparts), dim3(kBlock), 0, s, n, a, b,
                       part);
    check_launch("k_dot_parts");
}

void launch_dot_parts_f32(int64_t n, const float *a, const float *b,
                          double *part, int32_t nparts, hipStream_t s)
{
    hipLaunchKernelGGL(k_dot_parts<float>, dim3(nparts), dim3(kBlock), 0, s, n, a, b,
                       part);
    check_launch("k_dot_parts");
}

void launch_sum_parts(const double *part, int32_t nparts, double *out,
                      hipStream_t s)
{
    hipLaunchKernelGGL(k_sum_parts<double>, dim3(1), dim3(1024), 0, s, part, nparts,
                       out);
    check_launch("k_sum_parts");
}

void launch_sum_parts_f32(const double *part, int32_t nparts, float *out,
                          hipStream_t s)
{
    hipLaunchKernelGGL(k_sum_parts<float>, dim3(1), dim3(1024), 0, s, part, nparts,
                       out);
    check_launch("k_sum_parts");
}

void launch_stream(const void *src, void *dst, int64_t bytes, int32_t groups,
                   uint32_t *sink, hipStream_t s)
{
    const int64_t n = bytes / 16;
    if (n <= 0)
        return;
    const int64_t per = (n + groups - 1) / groups;
    if (dst)
        hipLaunchKernelGGL((k_stream<4, true>), dim3(groups), dim3(kBlock), 0, s,
                           (const i32x4 *)src, (i32x4 *)dst, n, per, sink);
    else
        hipLaunchKernelGGL((k_stream<8, false>), dim3(groups), dim3(kBlock), 0, s,
                           (const i32x4 *)src, (i32x4 *)nullptr, n, per, sink);
    check_launch("k_stream");
}

void launch_copy_f64(int64_t n, const double *src, double *dst, hipStream_t s)
{
    if (n <= 0)
        return;
    hipLaunchKernelGGL(k_copy<double>, dim3(grid_for(n, kBlock, 8192)),
                       dim3(kBlock), 0, s, n, src, dst);
    check_launch("k_copy");
}

void launch_copy_f32(int64_t n, const float *src, float *dst, hipStream_t s)
{
    if (n <= 0)
        return;
    hipLaunchKernelGGL(k_copy<float>, dim3(grid_for(n, kBlock, 8192)),
                       dim3(kBlock), 0, s, n, src, dst);
    check_launch("k_copy");
}

void launch_cg_init(int64_t n, const double *b, double *x, double *r, double *p,
                    double *sv, double *rr, int32_t nparts, CgScalars *sc, hipStream_t s)
{
    hipLaunchKernelGGL(k_cg_init, dim3(nparts), dim3(kBlock), 0, s, n, b, x, r, p, sv, rr,
                       sc);
    check_launch("k_cg_init");
}

void launch_cg_step(int64_t n, CgScalars *sc, const double *w, double *p, double *sv,
                    double *x, double *r, const double *dot_part, int32_t ndot, double *rr,
                    int32_t nparts, int32_t k, hipStream_t s)
{
    hipLaunchKernelGGL(k_cg_step, dim3(nparts), dim3(kBlock), 0, s, n, sc, w, p, sv, x, r,
                       dot_part, ndot, rr, nparts, k);
    check_launch("k_cg_step");
}

void launch_cg_final(CgScalars *sc, const double *rr, int32_t nparts, int32_t par,
                     hipStream_t s)
{
    hipLaunchKernelGGL(k_cg_final, dim3(1), dim3(1024), 0, s, sc, rr, nparts, par);
    check_launch("k_cg_final");
}

}  // namespace lilac
