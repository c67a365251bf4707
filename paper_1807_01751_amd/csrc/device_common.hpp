// Device helpers shared by the gfx950 kernels of libbfm: operator-table access,
// series loads and the chunked row streamer.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bfm {
namespace dev {

// The shared operator tables never change during a launch: reading them through
// the constant address space lets every wave fetch them with scalar loads into
// SGPRs (one fetch per wave, no vector registers, no per-lane traffic).
using ctab = const __attribute__((address_space(4))) double*;

__device__ __forceinline__ ctab as_const(const double* p)
{
    return (ctab)(const __attribute__((address_space(4))) void*)(p);
}

// Raw buffer loads keep a time row's base address in SGPRs (a buffer
// resource) and the lane's byte offset in one VGPR, so stepping to the next
// row costs scalar adds only.  The series is read exactly once, so the loads
// carry the non-temporal hint.
constexpr int kRsrcWord3 = 0x00020000;  // raw access, gfx9-family descriptor layout
constexpr int kLoadNT = 2;              // cache-policy bits of the load: nt

__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const void* row)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(row), 0, -1, kRsrcWord3);
}

__device__ __forceinline__ float load_obs(const float* row, uint32_t lane_bytes)
{
    return __uint_as_float(
        __builtin_amdgcn_raw_buffer_load_b32(row_rsrc(row), (int)lane_bytes, 0, kLoadNT));
}

// A BF16 observation as stored: the high half of the float32 of the same value
// (decoding is exact: the low 16 bits of the float are zero).
struct bf16_t {
    uint16_t bits;
};

// An IEEE binary16 observation as stored (decoding to float32 is exact).
struct f16_t {
    uint16_t bits;
};

__device__ __forceinline__ float decode(bf16_t, uint32_t b) { return __uint_as_float(b << 16); }
__device__ __forceinline__ float decode(f16_t, uint32_t b)
{
    return (float)__builtin_bit_cast(_Float16, (uint16_t)b);
}

__device__ __forceinline__ float to_float(float v) { return v; }
__device__ __forceinline__ float to_float(bf16_t v) { return decode(v, v.bits); }
__device__ __forceinline__ float to_float(f16_t v) { return decode(v, v.bits); }

// 16-bit storage types: one 2-byte load per lane, decoded in a register.
template <typename T>
__device__ __forceinline__ float load_obs(const T* row, uint32_t lane_bytes)
{
    static_assert(sizeof(T) == 2, "16-bit storage types only");
    const uint32_t b = __builtin_amdgcn_raw_buffer_load_b16(row_rsrc(row), (int)lane_bytes, 0, kLoadNT);
    return decode(T{}, b);
}

__device__ __forceinline__ uint32_t load_flag(const uint8_t* row, uint32_t lane)
{
    return __builtin_amdgcn_raw_buffer_load_b8(row_rsrc(row), (int)lane, 0, kLoadNT);
}

// max and min of a running extreme and a value that is either a number or the
// quiet NaN 0x7ff8... (every value here is the result of arithmetic): in IEEE
// mode the hardware returns the other operand for a quiet NaN, so the
// compiler's quieting of the loop-carried operand (one more instruction per
// row) is not needed.
__device__ __forceinline__ double max_num(double a, double b)
{
    double r;
    asm volatile("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ double min_num(double a, double b)
{
    double r;
    asm volatile("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ float max_num(float a, float b)
{
    float r;
    asm volatile("v_max_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ float min_num(float a, float b)
{
    float r;
    asm volatile("v_min_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

template <typename T>
__device__ __forceinline__ void put(void* base, int64_t idx, double v)
{
    static_cast<T*>(base)[idx] = static_cast<T>(v);
}

__device__ __forceinline__ void put_out(void* base, int64_t idx, double v, int f64)
{
    if (f64)
        put<double>(base, idx, v);
    else
        put<float>(base, idx, v);
}

// One observation of element type T by raw buffer load at a lane offset and a
// scalar (row) offset, decoded to float32.
__device__ __forceinline__ float load_at(const float*, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, kLoadNT));
}
template <typename T>
__device__ __forceinline__ float load_at(const T*, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    static_assert(sizeof(T) == 2, "16-bit storage types only");
    const uint32_t b = __builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, (int)soff, kLoadNT);
    return decode(T{}, b);
}

// Cursor over rows of one pixel column for block-wise streaming: one buffer
// resource based at the current row, row u ahead of it at the scalar byte
// offset u * ld * sizeof(T) (the caller keeps the rows of a block below 2^31
// bytes of offset).  Hands out float32 values.
template <typename T>
struct BlockCursorT {
    using value_type = float;
    const T* row;
    int64_t ld;
    uint32_t ldb;         // ld * sizeof(T)
    uint32_t lane_bytes;  // lane * sizeof(T)
    __amdgpu_buffer_rsrc_t rsrc;
    __device__ BlockCursorT(const T* row_, int64_t ld_, uint32_t lane)
        : row(row_), ld(ld_), ldb((uint32_t)ld_ * (uint32_t)sizeof(T)),
          lane_bytes(lane * (uint32_t)sizeof(T)), rsrc(row_rsrc(row_))
    {
    }
    __device__ __forceinline__ value_type load(int u) const
    {
        return load_at(static_cast<const T*>(nullptr), rsrc, lane_bytes, (uint32_t)u * ldb);
    }
    __device__ __forceinline__ void advance(int k)
    {
        row += (int64_t)k * ld;
        rsrc = row_rsrc(row);
    }
};

// Cursor over one pixel column of the time-major series (stored as T: float or
// bf16_t); it hands out float32 values.
template <typename T>
struct ObsCursorT {
    using value_type = float;
    const T* row;  // wave-uniform address of the current time row
    int64_t ld;
    uint32_t lane_bytes;  // lane * sizeof(T)
    __device__ __forceinline__ value_type load(int u) const
    {
        return load_obs(row + (int64_t)u * ld, lane_bytes);
    }
    __device__ __forceinline__ void advance(int k) { row += (int64_t)k * ld; }
};
using ObsCursor = ObsCursorT<float>;

// An observation and its caller-supplied validity flag (nonzero = observed).
struct FlaggedObs {
    float y;
    uint32_t ok;
};

template <typename T>
struct FlaggedCursorT {
    using value_type = FlaggedObs;
    const T* row;
    const uint8_t* vrow;
    int64_t ld, ldv;
    uint32_t lane;
    __device__ __forceinline__ value_type load(int u) const
    {
        return {load_obs(row + (int64_t)u * ld, lane * (uint32_t)sizeof(T)),
                load_flag(vrow + (int64_t)u * ldv, lane)};
    }
    __device__ __forceinline__ void advance(int k)
    {
        row += (int64_t)k * ld;
        vrow += (int64_t)k * ldv;
    }
};
using FlaggedCursor = FlaggedCursorT<float>;

// Streams rows [t0, t1) of one pixel column; `cur` must point at row t0.
// Rows are fetched in chunks of U, one chunk ahead of the arithmetic, with two
// register buffers used in turn.  Before the rows [t, t + count) of a chunk
// are handed over, pre(t, count) runs; then body(u, t + u, value) runs for each
// row, u being the row's position in the chunk (a compile-time constant after
// unrolling).  The loop over full chunks is straight-line code, so the
// compiler's wait counts keep the next chunk's loads in flight while a chunk
// is processed.  The last chunk may be short: it is fetched ahead like the
// others, its positions past t1 re-reading its last row (never handed over),
// so no row at the end of a stream waits for its load alone.
template <int U, typename Cursor, typename Body, typename Pre>
__device__ __forceinline__ void stream_rows(Cursor cur, int t0, int t1, Body&& body, Pre&& pre)
{
    using V = typename Cursor::value_type;
    auto load_full = [&](V* buf) {
#pragma unroll
        for (int u = 0; u < U; ++u) buf[u] = cur.load(u);
        cur.advance(U);
    };
    auto load_part = [&](V* buf, int count) {  // 1 <= count < U
        // The index of the positions past the end is opaque to the compiler,
        // so that no position is proved equal to another and turned into a
        // register copy (which would wait for the load).  Inline-asm results
        // count as divergent, hence the readfirstlane.
        int last = __builtin_amdgcn_readfirstlane(count - 1);
        asm volatile("" : "+s"(last));
        last = __builtin_amdgcn_readfirstlane(last);
#pragma unroll
        for (int u = 0; u < U; ++u) buf[u] = cur.load(u < count ? u : last);
        cur.advance(count);
    };
    auto run_full = [&](const V* buf, int t) {
        pre(t, U);
#pragma unroll
        for (int u = 0; u < U; ++u) body(u, t + u, buf[u]);
    };
    auto run_part = [&](const V* buf, int t, int count) {  // 1 <= count < U
        pre(t, count);
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (u < count) body(u, t + u, buf[u]);
    };
    V a[U], b[U];
    if (t1 - t0 < U) {
        if (t1 > t0) {
            load_part(a, t1 - t0);
            run_part(a, t0, t1 - t0);
        }
        return;
    }
    int t = t0;
    load_full(a);
    for (; t + 3 * U <= t1; t += 2 * U) {
        load_full(b);
        run_full(a, t);
        load_full(a);
        run_full(b, t + U);
    }
    // a holds the full chunk at t; U <= t1 - t < 3U rows remain.
    const int R = t1 - t;
    if (R > 2 * U) {
        load_full(b);
        run_full(a, t);
        load_part(a, R - 2 * U);
        run_full(b, t + U);
        run_part(a, t + 2 * U, R - 2 * U);
    } else if (R == 2 * U) {
        load_full(b);
        run_full(a, t);
        run_full(b, t + U);
    } else if (R > U) {
        load_part(b, R - U);
        run_full(a, t);
        run_part(b, t + U, R - U);
    } else {
        run_full(a, t);
    }
}

template <int U, typename Cursor, typename Body>
__device__ __forceinline__ void stream_rows(Cursor cur, int t0, int t1, Body&& body)
{
    stream_rows<U>(cur, t0, t1, [&](int, int t, typename Cursor::value_type v) { body(t, v); },
                   [](int, int) {});
}

// A lean form for rarely taken passes: chunks of U rows, each chunk's loads
// issued together (the last chunk's positions past t1 re-read row t1 - 1) and
// then its rows processed, with no fetch ahead of the arithmetic; one copy of
// the body, so that such a pass adds little code.
template <int U, typename Cursor, typename Body>
__device__ __forceinline__ void stream_rows_lean(Cursor cur, int t0, int t1, Body&& body)
{
    using V = typename Cursor::value_type;
    for (int t = t0; t < t1; t += U) {
        const int count = t1 - t < U ? t1 - t : U;
        V buf[U];
#pragma unroll
        for (int u = 0; u < U; ++u) buf[u] = cur.load(u < count ? u : count - 1);
        cur.advance(count);
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (u < count) body(t + u, buf[u]);
    }
}

// Streams rows [t0, t1) in blocks aligned to multiples of F in absolute time:
// block tb covers rows [tb, tb + F) with tb % F == 0, and a row's position
// u = t - tb (its phase t mod F) is a compile-time constant in the unrolled
// body.  The first and last blocks may be partial.  `cur` must point at row t0.
// Blocks are fetched one ahead of the arithmetic into two register buffers.
// For each block, pre(tb, lo, hi) runs before body(u, tb + u, value) is called
// for u in [lo, hi).
template <int F, typename Cursor, typename Body, typename Pre>
__device__ __forceinline__ void stream_aligned(Cursor cur, int t0, int t1, Body&& body, Pre&& pre)
{
    using V = typename Cursor::value_type;
    if (t0 >= t1) return;
    // A partial block reads its rows [lo, hi); the other positions re-read the
    // nearest of them (never handed over), so both forms are straight-line code.
    auto load_block = [&](V* buf, int lo, int hi) {
        if (lo == 0 && hi == F) {
#pragma unroll
            for (int u = 0; u < F; ++u) buf[u] = cur.load(u);
        } else {
#pragma unroll
            for (int u = 0; u < F; ++u) buf[u] = cur.load(u < lo ? 0 : (u < hi ? u - lo : hi - 1 - lo));
        }
        cur.advance(hi - lo);
    };
    // pre sees its range as compile-time constants for a whole block, so that
    // per-row work in it becomes straight-line code there.
    auto run_block = [&](V* buf, int tb, int lo, int hi) {
        if (lo == 0 && hi == F) {
            pre(tb, 0, F);
#pragma unroll
            for (int u = 0; u < F; ++u) body(u, tb + u, buf[u]);
        } else {
            pre(tb, lo, hi);
#pragma unroll
            for (int u = 0; u < F; ++u)
                if (u >= lo && u < hi) body(u, tb + u, buf[u]);
        }
    };
    V a[F], b[F];
    int tb = t0 - t0 % F;
    int lo = t0 - tb;
    int hi = t1 - tb < F ? t1 - tb : F;
    load_block(a, lo, hi);
    for (;;) {
        int nb = tb + F;
        int nhi = t1 - nb < F ? t1 - nb : F;
        if (nb < t1) load_block(b, 0, nhi);
        run_block(a, tb, lo, hi);
        if (nb >= t1) break;
        tb = nb;
        hi = nhi;
        nb = tb + F;
        nhi = t1 - nb < F ? t1 - nb : F;
        if (nb < t1) load_block(a, 0, nhi);
        run_block(b, tb, 0, hi);
        if (nb >= t1) break;
        tb = nb;
        lo = 0;
        hi = nhi;
    }
}

// Filling of missing observations (the footnote of Section 3): a non-finite
// observation takes the last finite one before it, and those before a lane's
// first finite observation take that one.  first_finite scans rows from the
// top until every lane of the wave has found its first finite value (the loop
// is wave-uniform; a lane with none keeps a NaN); Filler then fills each row
// as it is consumed, in time order.
template <typename T>
__device__ __forceinline__ float first_finite(const T* __restrict__ Y, int64_t ld, uint32_t lane, int N)
{
    float v = to_float(Y[lane]);
    for (int t = 1; t < N && __ballot(!__builtin_isfinite(v)) != 0; ++t) {
        const float w = to_float(Y[(int64_t)t * ld + lane]);
        v = __builtin_isfinite(v) ? v : w;
    }
    return v;
}

struct Filler {
    float last;
    __device__ __forceinline__ float operator()(float v)
    {
        v = __builtin_isfinite(v) ? v : last;
        last = v;
        return v;
    }
};

}  // namespace dev
}  // namespace bfm
