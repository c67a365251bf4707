// C ABI of libbfm: argument validation, contexts, the per-parameter-set cache of
// shared operators, and dispatch to the gfx950 kernels.  Declarations and the
// contract of every entry point are in include/bfm.h.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <type_traits>
#include <vector>

#include "bfm_internal.hpp"

// Device memory of one cached operator block: a range of the context's
// arena (or, for a block larger than the whole arena, its own allocation), the
// event recorded after the last launch that reads it, and its last-use stamp.
struct OpBlock {
    size_t off = 0, bytes = 0;
    char* own = nullptr;
    hipEvent_t last = nullptr;
    uint64_t stamp = 0;
};

struct bfm_ctx {
    int device = 0;
    size_t max_lds = 0;  // dynamic LDS bytes one workgroup may use
    int cus = 0;         // compute units
    std::mutex mu;
    // Operator cache: one device arena of op_budget bytes, allocated at the
    // first parameter set and carved first-fit; least recently used blocks are
    // evicted when a new one does not fit, each after its own last launch has
    // finished (no device-wide synchronisation).
    size_t op_budget = (size_t)64 << 20;
    char* arena = nullptr;
    std::map<size_t, size_t> arena_free;  // offset -> length
    uint64_t clock = 0;
    int64_t evictions = 0;
    size_t cached_bytes = 0;
    struct Entry {
        bfm::PlainOps ops;
        double* dev = nullptr;  // q | w | bnd | bmap
        bfm::PeriodicOps per;   // per.F == 0: the period-blocked kernel does not apply
        double* pdev = nullptr; // rt | ri | hh | wh | bnd
        std::vector<double> times;  // observation times the operators were built for
        OpBlock blk;
    };
    // (N, n, k, h_window, f, h_frac, lambda, hash of the observation times or 0)
    using Key = std::tuple<int, int, int, int, double, double, double, uint64_t>;
    std::map<Key, Entry> plain;
    // Autotuned time split of the period-blocked plain and missing-value
    // kernels, per tile shape: (order, F, H (plain) or ring capacity (missing
    // values), N, n, y_dtype, ceil(log2(waves)), mask mode) -> waves per 64 pixels.
    using TuneKey = std::tuple<int, int, int, int, int, int, int, int>;
    std::map<TuneKey, int> tune;
    struct MEntry {
        bfm::MaskedOps ops;
        double* dev = nullptr;  // x | g | ph
        std::vector<double> times;
        OpBlock blk;
    };
    std::map<Key, MEntry> masked;
};

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what)
{
    return fail(e == hipErrorOutOfMemory ? BFM_E_NOMEM : BFM_E_HIP, "%s: %s", what,
                hipGetErrorString(e));
}

int check(const bfm_params* prm, int64_t P, int64_t ld)
{
    if (!prm) return fail(BFM_E_INVAL, "params is NULL");
    const bfm_params& p = *prm;
    if (p.n_hist < 1) return fail(BFM_E_INVAL, "n_hist must be >= 1 (got %d)", p.n_hist);
    if (p.n_obs <= p.n_hist)
        return fail(BFM_E_INVAL, "n_obs (%d) must exceed n_hist (%d)", p.n_obs, p.n_hist);
    if (p.order < 0 || p.order > bfm::kMaxOrder)
        return fail(BFM_E_INVAL, "order must be in [0, %d] (got %d)", bfm::kMaxOrder, p.order);
    if (!(p.freq > 0) || !std::isfinite(p.freq))
        return fail(BFM_E_INVAL, "freq must be positive and finite");
    if (!(p.lambda > 0) || !std::isfinite(p.lambda))
        return fail(BFM_E_INVAL, "lambda must be positive and finite");
    if (p.h_window < 0 || p.h_window > p.n_hist)
        return fail(BFM_E_INVAL, "h_window must be in [0, n_hist] (got %d)", p.h_window);
    if (p.h_window == 0 && !(p.h_frac > 0 && p.h_frac <= 1))
        return fail(BFM_E_INVAL, "h_frac must be in (0, 1] when h_window is 0");
    if (p.mask_mode < BFM_MASK_NONE || p.mask_mode > BFM_MASK_FILL)
        return fail(BFM_E_INVAL, "unknown mask_mode %d", p.mask_mode);
    if (p.times)
        for (int t = 0; t < p.n_obs; ++t)
            if (!std::isfinite(p.times[t]) || (t > 0 && !(p.times[t] > p.times[t - 1])))
                return fail(BFM_E_INVAL, "times must be finite and strictly increasing (index %d)", t);
    if (p.precision != BFM_PREC_FP64 && p.precision != BFM_PREC_FP32)
        return fail(BFM_E_INVAL, "unknown precision %d", p.precision);
    if (P < 0) return fail(BFM_E_INVAL, "P must be >= 0");
    if (P > ((int64_t)1 << 30)) return fail(BFM_E_INVAL, "P must be <= 2^30 per call");
    if (ld < P) return fail(BFM_E_LAYOUT, "ld (%lld) must be >= P (%lld)", (long long)ld, (long long)P);
    g_err.clear();
    return BFM_SUCCESS;
}

// Restores the caller's current device on scope exit.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

int log2_ceil(int64_t v)
{
    int k = 0;
    while (((int64_t)1 << k) < v) ++k;
    return k;
}

bfm_ctx::TuneKey tune_key(const bfm_params& p, int y_dtype, int64_t P, int H, int F)
{
    return bfm_ctx::TuneKey{p.order, F, H, p.n_obs, p.n_hist, y_dtype, log2_ceil((P + 63) / 64), p.mask_mode};
}

// Waves per 64 pixels that share a pixel's rows in the period-blocked plain
// kernel: the tuned (or pinned) choice for this tile shape, else a rule taken
// from timings on MI355X.  A tile of at most one wave per compute unit over a
// series of 512 rows or more runs 2-2.7x faster with eight waves per 64 pixels
// (4096 or 16384 pixels x 1000-4600 rows); with more waves than compute units,
// or over shorter series (4096 x 228), one wave per 64 pixels is as fast or
// faster.
int choose_split(bfm_ctx* ctx, const bfm_params& p, int y_dtype, int64_t P, int H, int F)
{
    auto it = ctx->tune.find(tune_key(p, y_dtype, P, H, F));
    if (it != ctx->tune.end()) return it->second;
    const int64_t waves = (P + 63) / 64;
    if (waves <= ctx->cus && p.n_obs >= 512 &&
        bfm::periodic_split_lds(p.order, F, 8, H) <= ctx->max_lds)
        return 8;
    return 1;
}

// FNV-1a over the bytes of the observation times (0: index time).
uint64_t times_hash(const bfm_params& p)
{
    if (!p.times) return 0;
    uint64_t h = 1469598103934665603ull;
    const unsigned char* b = reinterpret_cast<const unsigned char*>(p.times);
    for (size_t i = 0; i < (size_t)p.n_obs * sizeof(double); ++i) h = (h ^ b[i]) * 1099511628211ull;
    return h | 1;
}

std::vector<double> times_of(const bfm_params& p)
{
    return p.times ? std::vector<double>(p.times, p.times + p.n_obs) : std::vector<double>();
}

constexpr size_t kBlockAlign = 256;
size_t align_up(size_t n) { return (n + kBlockAlign - 1) / kBlockAlign * kBlockAlign; }

// Returns a block's memory once its last launch has finished (a wait on that
// block's event only: launches on other streams go on).  Call with ctx->mu held.
void block_free(bfm_ctx* ctx, OpBlock& b)
{
    if (b.last) {
        (void)hipEventSynchronize(b.last);
        (void)hipEventDestroy(b.last);
    }
    if (b.own) {
        (void)hipFree(b.own);
    } else if (b.bytes) {
        auto it = ctx->arena_free.emplace(b.off, b.bytes).first;
        auto next = std::next(it);
        if (next != ctx->arena_free.end() && it->first + it->second == next->first) {
            it->second += next->second;
            ctx->arena_free.erase(next);
        }
        if (it != ctx->arena_free.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                ctx->arena_free.erase(it);
            }
        }
    }
    ctx->cached_bytes -= b.bytes;
    b = OpBlock{};
}

bool block_idle(const OpBlock& b) { return !b.last || hipEventQuery(b.last) == hipSuccess; }

// Evicts the least recently used cached entry (only an idle one if
// idle_only).  Returns false if there was none to evict.
bool evict_lru(bfm_ctx* ctx, bool idle_only)
{
    uint64_t best = UINT64_MAX;
    int which = -1;
    bfm_ctx::Key key;
    for (auto& kv : ctx->plain)
        if (kv.second.blk.stamp < best && (!idle_only || block_idle(kv.second.blk))) {
            best = kv.second.blk.stamp;
            which = 0;
            key = kv.first;
        }
    for (auto& kv : ctx->masked)
        if (kv.second.blk.stamp < best && (!idle_only || block_idle(kv.second.blk))) {
            best = kv.second.blk.stamp;
            which = 1;
            key = kv.first;
        }
    if (which < 0) return false;
    if (which == 0) {
        auto it = ctx->plain.find(key);
        block_free(ctx, it->second.blk);
        ctx->plain.erase(it);
    } else {
        auto it = ctx->masked.find(key);
        block_free(ctx, it->second.blk);
        ctx->masked.erase(it);
    }
    ++ctx->evictions;
    return true;
}

// Device memory for a new operator block of `bytes`, evicting least recently
// used blocks (idle ones first) while it does not fit.  Call with ctx->mu held.
int block_get(bfm_ctx* ctx, size_t bytes, OpBlock* b, char** base)
{
    const size_t n = align_up(bytes);
    *b = OpBlock{};
    hipError_t e;
    if (!ctx->arena && ctx->op_budget > 0) {
        e = hipMalloc(&ctx->arena, ctx->op_budget);
        if (e != hipSuccess) {
            ctx->arena = nullptr;
            return hip_fail(e, "hipMalloc(operator arena)");
        }
        ctx->arena_free[0] = ctx->op_budget;
    }
    if (n > ctx->op_budget) {  // larger than the whole arena: a block of its own
        e = hipMalloc(&b->own, n);
        if (e != hipSuccess) return hip_fail(e, "hipMalloc(operators)");
        *base = b->own;
    } else {
        for (;;) {
            auto it = std::find_if(ctx->arena_free.begin(), ctx->arena_free.end(),
                                   [&](const std::pair<const size_t, size_t>& f) { return f.second >= n; });
            if (it != ctx->arena_free.end()) {
                b->off = it->first;
                const size_t rest = it->second - n, at = it->first + n;
                ctx->arena_free.erase(it);
                if (rest) ctx->arena_free[at] = rest;
                break;
            }
            if (!evict_lru(ctx, true) && !evict_lru(ctx, false))
                return fail(BFM_E_NOMEM, "operator block of %zu B does not fit the %zu B budget", n,
                            ctx->op_budget);
        }
        *base = ctx->arena + b->off;
    }
    b->bytes = n;
    ctx->cached_bytes += n;
    e = hipEventCreateWithFlags(&b->last, hipEventDisableTiming);
    if (e != hipSuccess) {
        block_free(ctx, *b);
        return hip_fail(e, "hipEventCreate(operators)");
    }
    return BFM_SUCCESS;
}

// Marks a block as read by the launch just enqueued on `s`.
void block_used(bfm_ctx* ctx, OpBlock& b, hipStream_t s)
{
    b.stamp = ++ctx->clock;
    (void)hipEventRecord(b.last, s);
}

// A cached entry built for other observation times under the same hash is
// dropped (its block returned once its last launch has finished) so that it
// is rebuilt.
template <typename Map>
void drop_if_stale(bfm_ctx* ctx, Map& m, const bfm_ctx::Key& key, const bfm_params& p)
{
    auto it = m.find(key);
    if (it == m.end() || !p.times) return;
    if (it->second.times.size() == (size_t)p.n_obs &&
        std::memcmp(it->second.times.data(), p.times, (size_t)p.n_obs * sizeof(double)) == 0)
        return;
    block_free(ctx, it->second.blk);
    m.erase(it);
}

// The plain-path operators of a parameter set (built and copied to the device
// on first use).  Call with ctx->mu held.
int plain_entry(bfm_ctx* ctx, const bfm_params& p, bfm_ctx::Entry** out)
{
    bfm_ctx::Key key{p.n_obs, p.n_hist, p.order, p.h_window, p.freq, p.h_frac, p.lambda, times_hash(p)};
    drop_if_stale(ctx, ctx->plain, key, p);
    auto it = ctx->plain.find(key);
    if (it == ctx->plain.end()) {
        bfm_ctx::Entry ent;
        ent.times = times_of(p);
        bfm::build_plain_ops(p, &ent.ops);
        // One block: q | w | bnd | bmap, then (period-blocked kernel) rt | ri | hh | wh | bnd.
        std::vector<double> host;
        host.insert(host.end(), ent.ops.q.begin(), ent.ops.q.end());
        host.insert(host.end(), ent.ops.w.begin(), ent.ops.w.end());
        host.insert(host.end(), ent.ops.bnd.begin(), ent.ops.bnd.end());
        host.insert(host.end(), ent.ops.bmap.begin(), ent.ops.bmap.end());
        const size_t nplain = host.size();
        const int F = bfm::periodic_period(p, ent.ops);
        if (F > 0) {
            bfm::build_periodic_ops(p, ent.ops, F, &ent.per);
            host.insert(host.end(), ent.per.rt.begin(), ent.per.rt.end());
            host.insert(host.end(), ent.per.ri.begin(), ent.per.ri.end());
            host.insert(host.end(), ent.per.hh.begin(), ent.per.hh.end());
            host.insert(host.end(), ent.per.wh.begin(), ent.per.wh.end());
            host.insert(host.end(), ent.ops.bnd.begin(), ent.ops.bnd.end());
        }
        char* base = nullptr;
        int rc = block_get(ctx, host.size() * sizeof(double), &ent.blk, &base);
        if (rc) return rc;
        // A synchronous copy: the operator block is a few tens of KB and this
        // happens once per parameter set.
        hipError_t e = hipMemcpy(base, host.data(), host.size() * sizeof(double), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            block_free(ctx, ent.blk);
            return hip_fail(e, "hipMemcpy(operators)");
        }
        ent.dev = reinterpret_cast<double*>(base);
        ent.pdev = F > 0 ? ent.dev + nplain : nullptr;
        it = ctx->plain.emplace(key, std::move(ent)).first;
    }
    *out = &it->second;
    return BFM_SUCCESS;
}

// Missing-value modes: per-pixel masked fit (csrc/masked_kernel.hip).
int fit_masked(bfm_ctx* ctx, const bfm_params& p, const void* Y, int y_dtype, int64_t P, int64_t ld,
               const uint8_t* valid, int64_t ldv, const bfm_outputs& out, hipStream_t s)
{
    bfm_ctx::Key key{p.n_obs, p.n_hist, p.order, p.h_window, p.freq, p.h_frac, 0.0, times_hash(p)};
    drop_if_stale(ctx, ctx->masked, key, p);
    auto it = ctx->masked.find(key);
    if (it == ctx->masked.end()) {
        bfm_ctx::MEntry ent;
        ent.times = times_of(p);
        bfm::build_masked_ops(p, &ent.ops);
        std::vector<double> host(ent.ops.x);
        host.insert(host.end(), ent.ops.g.begin(), ent.ops.g.end());
        host.insert(host.end(), ent.ops.ph.begin(), ent.ops.ph.end());
        char* base = nullptr;
        int rc = block_get(ctx, host.size() * sizeof(double), &ent.blk, &base);
        if (rc) return rc;
        hipError_t e = hipMemcpy(base, host.data(), host.size() * sizeof(double), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            block_free(ctx, ent.blk);
            return hip_fail(e, "hipMemcpy(masked operators)");
        }
        ent.dev = reinterpret_cast<double*>(base);
        it = ctx->masked.emplace(key, std::move(ent)).first;
    }
    const bfm::MaskedOps& ops = it->second.ops;
    // The period-blocked kernel addresses F rows of one block with 32-bit offsets.
    const int64_t lim = (int64_t)1 << 31;
    const bool blocked = ops.F > 0 && ld * 4 * ops.F < lim &&
                         (p.mask_mode != BFM_MASK_EXPLICIT || ldv * ops.F < lim);
    if (y_dtype != BFM_Y_F32 && !blocked)
        return fail(BFM_E_UNSUPPORTED, "a 16-bit series needs f in {12, 23, 24}, n_hist <= %d and "
                    "ld * 4 * f < 2^31 on the missing-value path", bfm::kMaskedPeriodicMaxHist);
    // History split of the period-blocked kernel: the tuned (or pinned) choice
    // for this tile shape, else a rule taken from timings on MI355X (25% NaN,
    // k = 3): four waves per 64 pixels for a tile of at most one wave per
    // compute unit (4096 x 228: -8%, 4096 and 16384 x 1000: -20%), two up to
    // four waves per compute unit (65536 x 400: -8%), else one (a full tile
    // loses occupancy to the larger workgroup LDS).  A split that does not fit
    // (LDS, a block of history rows per wave) is halved until it does.
    int split = 1;
    if (blocked) {
        auto tt = ctx->tune.find(tune_key(p, y_dtype, P, ops.cap, ops.F));
        if (tt != ctx->tune.end()) {
            split = tt->second;
        } else {
            const int64_t waves = (P + 63) / 64;
            split = waves <= ctx->cus ? 4 : (waves <= 4 * (int64_t)ctx->cus ? 2 : 1);
        }
        while (split > 1 && (split > (p.n_hist + ops.F - 1) / ops.F ||
                             bfm::masked_periodic_lds_bytes(ops.cap, ops.F, split) > ctx->max_lds))
            split /= 2;
    }
    const size_t lds = blocked ? bfm::masked_periodic_lds_bytes(ops.cap, ops.F, split)
                               : bfm::masked_lds_bytes(ops.cap);
    if (lds > ctx->max_lds)
        return fail(BFM_E_UNSUPPORTED, "window H=%d needs %zu B of LDS per workgroup (max %zu)",
                    ops.Hmax, lds, ctx->max_lds);
    bfm::MaskedArgs a{};
    a.Y = Y;
    a.y_dtype = y_dtype;
    a.ld = ld;
    a.valid = valid;
    a.ldv = ldv;
    a.P = P;
    a.x = it->second.dev;
    a.g = it->second.dev + ops.x.size();
    a.ph = a.g + ops.g.size();
    a.F = ops.F;
    a.m32 = p.precision == BFM_PREC_FP32;
    a.split = split;
    a.N = p.n_obs;
    a.n = p.n_hist;
    a.h_window = p.h_window;
    a.cap = ops.cap;
    a.h_frac = p.h_frac;
    a.lambda = p.lambda;
    a.tc = ops.tc;
    a.ts = ops.ts;
    a.brk = out.brk;
    a.mag = out.mag;
    a.sigma = out.sigma;
    a.status = out.status;
    a.beta = out.beta;
    a.resid = out.resid;
    a.mosum = out.mosum;
    a.out_f64 = out.out_dtype == BFM_OUT_F64;
    hipError_t e = blocked ? bfm::launch_masked_periodic(a, p.order, p.mask_mode, s)
                           : bfm::launch_masked(a, p.order, p.mask_mode, s);
    if (e != hipSuccess) return hip_fail(e, "masked kernel launch");
    block_used(ctx, it->second.blk, s);
    return BFM_SUCCESS;
}

}  // namespace

namespace bfm {

size_t operator_block_bound(const bfm_params& p)
{
    const size_t N = (size_t)p.n_obs, n = (size_t)p.n_hist, k = (size_t)p.order, np = 2 + 2 * k;
    const size_t M = N > n ? N - n : 0;
    int F = 0;
    for (int f : kPeriods)
        if (!p.times && p.freq == (double)f) F = f;
    size_t doubles;
    if (p.mask_mode == BFM_MASK_NAN || p.mask_mode == BFM_MASK_EXPLICIT) {
        const bool blocked = F > 0 && p.order <= kMaskedMaxOrder && p.n_hist <= kMaskedPeriodicMaxHist;
        doubles = N * np + n * (2 + 6 * k) + (blocked ? (size_t)F * 4 * k : 0);
    } else {
        doubles = N * np + M * np + M + np * np;
        if (F > 0 && p.order <= kPeriodicMaxOrder && window_length(p, p.n_hist) >= F)
            doubles += 2 * np * np + 2 * (size_t)F * 2 * k + M;
    }
    return align_up(doubles * sizeof(double));
}

bool operator_room(bfm_ctx* ctx, const bfm_params& p)
{
    std::lock_guard<std::mutex> lock(ctx->mu);
    const bool masked = p.mask_mode == BFM_MASK_NAN || p.mask_mode == BFM_MASK_EXPLICIT;
    const bfm_ctx::Key key{p.n_obs, p.n_hist, p.order, p.h_window, p.freq, p.h_frac,
                           masked ? 0.0 : p.lambda, times_hash(p)};
    if (masked ? ctx->masked.count(key) != 0 : ctx->plain.count(key) != 0) return true;
    const size_t need = operator_block_bound(p);
    if (need > ctx->op_budget) return true;  // a block of its own
    size_t busy = 0;
    for (auto& kv : ctx->plain)
        if (!block_idle(kv.second.blk)) busy += kv.second.blk.bytes;
    for (auto& kv : ctx->masked)
        if (!block_idle(kv.second.blk)) busy += kv.second.blk.bytes;
    return need + busy <= ctx->op_budget;
}

size_t operator_budget_of(bfm_ctx* ctx)
{
    std::lock_guard<std::mutex> lock(ctx->mu);
    return ctx->op_budget;
}

}  // namespace bfm

extern "C" {

int bfm_operator_budget(bfm_ctx* ctx, size_t bytes)
{
    if (!ctx) return fail(BFM_E_INVAL, "ctx is NULL");
    std::lock_guard<std::mutex> lock(ctx->mu);
    if (ctx->arena || !ctx->plain.empty() || !ctx->masked.empty())
        return fail(BFM_E_INVAL, "the operator budget is set before the first call on the context");
    ctx->op_budget = align_up(bytes);
    return BFM_SUCCESS;
}

int bfm_cache_get_stats(bfm_ctx* ctx, bfm_cache_stats* st)
{
    if (!ctx || !st) return fail(BFM_E_INVAL, "ctx and st are required");
    std::lock_guard<std::mutex> lock(ctx->mu);
    st->entries = (int64_t)(ctx->plain.size() + ctx->masked.size());
    st->bytes = (int64_t)ctx->cached_bytes;
    st->budget = (int64_t)ctx->op_budget;
    st->evictions = ctx->evictions;
    return BFM_SUCCESS;
}

int bfm_version(void) { return BFM_VERSION; }

const char* bfm_last_error(void) { return g_err.c_str(); }

int bfm_check_params(const bfm_params* prm, int64_t P, int64_t ld) { return check(prm, P, ld); }

int bfm_create(bfm_ctx** out, int device)
{
    if (!out) return fail(BFM_E_INVAL, "out is NULL");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count == 0) return fail(BFM_E_NODEVICE, "no HIP device");
    if (device < 0 || device >= count)
        return fail(BFM_E_NODEVICE, "device %d out of range [0, %d)", device, count);
    hipDeviceProp_t prop;
    if ((e = hipGetDeviceProperties(&prop, device)) != hipSuccess)
        return hip_fail(e, "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(BFM_E_UNSUPPORTED, "device %d is %s; libbfm is built for gfx950", device,
                    prop.gcnArchName);
    {
        // The device address of the no-allocation scratch array, once per device.
        DeviceGuard g(device);
        if ((e = bfm::noalloc_scratch_init(device)) != hipSuccess)
            return hip_fail(e, "hipGetSymbolAddress(scratch)");
    }
    bfm_ctx* ctx = new (std::nothrow) bfm_ctx;
    if (!ctx) return fail(BFM_E_NOMEM, "context allocation failed");
    ctx->device = device;
    ctx->max_lds = prop.sharedMemPerBlock;
    ctx->cus = prop.multiProcessorCount;
    *out = ctx;
    g_err.clear();
    return BFM_SUCCESS;
}

int bfm_destroy(bfm_ctx* ctx)
{
    if (!ctx) return BFM_SUCCESS;
    {
        DeviceGuard g(ctx->device);
        std::lock_guard<std::mutex> lock(ctx->mu);
        for (auto& kv : ctx->plain) block_free(ctx, kv.second.blk);
        for (auto& kv : ctx->masked) block_free(ctx, kv.second.blk);
        if (ctx->arena) (void)hipFree(ctx->arena);
    }
    delete ctx;
    return BFM_SUCCESS;
}

int bfm_workspace_bytes(const bfm_params* prm, int64_t P, size_t* out)
{
    int rc = check(prm, P, P);
    if (rc) return rc;
    if (!out) return fail(BFM_E_INVAL, "out is NULL");
    size_t doubles = 0;
    if (prm->mask_mode == BFM_MASK_NAN || prm->mask_mode == BFM_MASK_EXPLICIT) {
        bfm::MaskedOps ops;
        bfm::build_masked_ops(*prm, &ops);
        doubles = ops.x.size() + ops.g.size() + ops.ph.size();
    } else {
        bfm::PlainOps ops;
        bfm::build_plain_ops(*prm, &ops);
        doubles = ops.q.size() + ops.w.size() + ops.bnd.size() + ops.bmap.size();
        const int F = bfm::periodic_period(*prm, ops);
        if (F > 0) {
            bfm::PeriodicOps per;
            bfm::build_periodic_ops(*prm, ops, F, &per);
            doubles += per.rt.size() + per.ri.size() + per.hh.size() + per.wh.size() + ops.bnd.size();
        }
    }
    *out = doubles * sizeof(double);
    return BFM_SUCCESS;
}

int bfm_host_operators(const bfm_params* prm, double* q, double* w, double* bnd, double* bmap)
{
    int rc = check(prm, 0, 0);
    if (rc) return rc;
    bfm::PlainOps ops;
    bfm::build_plain_ops(*prm, &ops);
    if (q) std::memcpy(q, ops.q.data(), ops.q.size() * sizeof(double));
    if (w) std::memcpy(w, ops.w.data(), ops.w.size() * sizeof(double));
    if (bnd) std::memcpy(bnd, ops.bnd.data(), ops.bnd.size() * sizeof(double));
    if (bmap) std::memcpy(bmap, ops.bmap.data(), ops.bmap.size() * sizeof(double));
    if (ops.n <= ops.p) return fail(BFM_E_INVAL, "n_hist (%d) must exceed p (%d)", ops.n, ops.p);
    if (ops.H < 1) return fail(BFM_E_INVAL, "window length is < 1");
    if (!ops.rank_ok) return fail(BFM_E_UNSUPPORTED, "history design is rank deficient");
    return BFM_SUCCESS;
}

int bfm_fit_monitor(bfm_ctx* ctx, const bfm_params* prm, const float* Y, int64_t P, int64_t ld,
                    const uint8_t* valid, int64_t ldv, const bfm_outputs* out, void* stream)
{
    return bfm_fit_monitor_typed(ctx, prm, Y, BFM_Y_F32, P, ld, valid, ldv, out, stream);
}

int bfm_fit_monitor_typed(bfm_ctx* ctx, const bfm_params* prm, const void* Y, int32_t y_dtype,
                          int64_t P, int64_t ld, const uint8_t* valid, int64_t ldv,
                          const bfm_outputs* out, void* stream)
{
    if (!ctx) return fail(BFM_E_INVAL, "ctx is NULL");
    if (y_dtype != BFM_Y_F32 && y_dtype != BFM_Y_BF16 && y_dtype != BFM_Y_F16)
        return fail(BFM_E_INVAL, "unknown y_dtype %d", y_dtype);
    const int narrow = y_dtype != BFM_Y_F32;  // 16-bit storage: period-blocked kernels only
    int rc = check(prm, P, ld);
    if (rc) return rc;
    if (!out) return fail(BFM_E_INVAL, "out is NULL");
    if (P == 0) return BFM_SUCCESS;
    if (!Y || !out->brk) return fail(BFM_E_INVAL, "Y and out->brk are required");
    if (out->out_dtype != BFM_OUT_F32 && out->out_dtype != BFM_OUT_F64)
        return fail(BFM_E_INVAL, "unknown out_dtype %d", out->out_dtype);
    if (prm->mask_mode == BFM_MASK_EXPLICIT) {
        if (!valid) return fail(BFM_E_INVAL, "valid is required with BFM_MASK_EXPLICIT");
        if (ldv < P) return fail(BFM_E_LAYOUT, "ldv must be >= P");
    }
    const bool fill = prm->mask_mode == BFM_MASK_FILL;
    const bool masked = prm->mask_mode == BFM_MASK_NAN || prm->mask_mode == BFM_MASK_EXPLICIT;
    if (masked && prm->order > bfm::kMaskedMaxOrder)
        return fail(BFM_E_UNSUPPORTED, "missing-value modes support order <= %d (got %d)",
                    bfm::kMaskedMaxOrder, prm->order);
    if (fill && narrow) return fail(BFM_E_UNSUPPORTED, "BFM_MASK_FILL takes float32 series");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bfm_params& p = *prm;
    const int np = 2 + 2 * p.order;

    std::lock_guard<std::mutex> lock(ctx->mu);
    DeviceGuard g(ctx->device);
    if (masked) return fit_masked(ctx, p, Y, y_dtype, P, ld, valid, ldv, *out, s);
    bfm_ctx::Entry* ent = nullptr;
    rc = plain_entry(ctx, p, &ent);
    if (rc) return rc;
    const bfm::PlainOps& ops = ent->ops;

    uint8_t global_st = BFM_ST_OK;
    if (ops.n <= ops.p || ops.H < 1)
        global_st = BFM_ST_INSUFFICIENT;
    else if (!ops.rank_ok)
        global_st = BFM_ST_RANK_DEFICIENT;
    hipError_t e;
    if (global_st != BFM_ST_OK) {
        e = bfm::launch_fill_status(Y, y_dtype, ld, P, p.n_obs, p.n_hist, np, global_st, *out,
                                    p.mask_mode, valid, ldv, s);
        return e == hipSuccess ? BFM_SUCCESS : hip_fail(e, "fill_status launch");
    }
    ent->blk.stamp = ++ctx->clock;
    const size_t lds = (size_t)ops.H * bfm::kPlainBlock * sizeof(float);
    if (lds > ctx->max_lds)
        return fail(BFM_E_UNSUPPORTED, "window H=%d needs %zu B of LDS per workgroup (max %zu)",
                    ops.H, lds, ctx->max_lds);
    // The period-blocked kernel addresses the F rows of a block with 32-bit
    // offsets, and its workgroup's window rings need H KB of LDS.
    const int64_t esize = y_dtype == BFM_Y_F32 ? 4 : 2;
    if (ent->per.F > 0 && ld * esize * ent->per.F < ((int64_t)1 << 31) &&
        bfm::periodic_split_lds(p.order, ent->per.F, 1, ops.H) <= ctx->max_lds) {
        bfm::PeriodicArgs a{};
        a.Y = Y;
        a.y_dtype = y_dtype;
        a.fill = fill;
        a.split = y_dtype == BFM_Y_F32 && !fill && !out->resid && !out->mosum
                      ? choose_split(ctx, p, y_dtype, P, ops.H, ent->per.F)
                      : 1;
        a.ld = ld;
        a.P = P;
        a.tab = ent->pdev;
        a.N = p.n_obs;
        a.n = p.n_hist;
        a.H = ops.H;
        a.m_flat = ops.m_flat;
        a.lambda = p.lambda;
        a.sqrt_n = std::sqrt((double)p.n_hist);
        a.inv_dof = 1.0 / (double)(p.n_hist - np);
        a.brk = out->brk;
        a.mag = out->mag;
        a.sigma = out->sigma;
        a.status = out->status;
        a.beta = out->beta;
        a.resid = out->resid;
        a.mosum = out->mosum;
        a.out_f64 = out->out_dtype == BFM_OUT_F64;
        e = bfm::launch_periodic(a, p.order, ent->per.F, s);
        if (e != hipSuccess) return hip_fail(e, "periodic kernel launch");
        block_used(ctx, ent->blk, s);
        return BFM_SUCCESS;
    }
    if (narrow)
        return fail(BFM_E_UNSUPPORTED, "a 16-bit series needs f in {12, 23, 24}, order <= %d, a "
                    "window f <= H <= %zu and ld * 2 * f < 2^31 on this path", bfm::kPeriodicMaxOrder,
                    ctx->max_lds / (bfm::kPeriodicBlock * sizeof(float)));
    const double* d = ent->dev;
    const size_t nq = ops.q.size(), nw = ops.w.size(), nb = ops.bnd.size();
    bfm::PlainArgs a{};
    a.Y = static_cast<const float*>(Y);
    a.ld = ld;
    a.P = P;
    a.q = d;
    a.w = d + nq;
    a.bnd = d + nq + nw;
    a.bmap = d + nq + nw + nb;
    a.N = p.n_obs;
    a.n = p.n_hist;
    a.H = ops.H;
    a.m_flat = ops.m_flat;
    a.lambda = p.lambda;
    a.sqrt_n = std::sqrt((double)p.n_hist);
    a.inv_dof = 1.0 / (double)(p.n_hist - np);
    a.fill = fill;
    a.brk = out->brk;
    a.mag = out->mag;
    a.sigma = out->sigma;
    a.status = out->status;
    a.beta = out->beta;
    a.resid = out->resid;
    a.mosum = out->mosum;
    a.out_f64 = out->out_dtype == BFM_OUT_F64;
    e = bfm::launch_plain(a, np, s);
    if (e != hipSuccess) return hip_fail(e, "plain kernel launch");
    block_used(ctx, ent->blk, s);
    return BFM_SUCCESS;
}

namespace {

// The time split applies: the period-blocked plain kernel serves these parameters.
int split_shape(bfm_ctx* ctx, const bfm_params* prm, int32_t y_dtype, int64_t P, int64_t ld, int* H,
                int* F)
{
    if (!ctx) return fail(BFM_E_INVAL, "ctx is NULL");
    int rc = check(prm, P, ld);
    if (rc) return rc;
    if (y_dtype != BFM_Y_F32 && y_dtype != BFM_Y_BF16 && y_dtype != BFM_Y_F16)
        return fail(BFM_E_INVAL, "unknown y_dtype %d", y_dtype);
    if (prm->mask_mode == BFM_MASK_NAN || prm->mask_mode == BFM_MASK_EXPLICIT) {
        // The history split of the period-blocked missing-value kernel.
        bfm::MaskedOps ops;
        bfm::build_masked_ops(*prm, &ops);
        const int64_t lim = (int64_t)1 << 31;
        if (ops.F == 0 || ld * 4 * ops.F >= lim ||
            bfm::masked_periodic_lds_bytes(ops.cap, ops.F, 1) > ctx->max_lds)
            return fail(BFM_E_UNSUPPORTED, "these parameters do not take the period-blocked "
                        "missing-value kernel");
        *H = ops.cap;
        *F = ops.F;
        return BFM_SUCCESS;
    }
    if (prm->mask_mode != BFM_MASK_NONE || y_dtype != BFM_Y_F32)
        return fail(BFM_E_UNSUPPORTED, "tile tuning applies to the plain path on float32 series and "
                    "to the missing-value path with f in {12, 23, 24}");
    std::lock_guard<std::mutex> lock(ctx->mu);
    DeviceGuard g(ctx->device);
    bfm_ctx::Entry* ent = nullptr;
    rc = plain_entry(ctx, *prm, &ent);
    if (rc) return rc;
    const int64_t esize = y_dtype == BFM_Y_F32 ? 4 : 2;
    if (ent->per.F == 0 || !ent->ops.rank_ok || ent->ops.n <= ent->ops.p || ent->ops.H < 1 ||
        ld * esize * ent->per.F >= ((int64_t)1 << 31) ||
        bfm::periodic_split_lds(prm->order, ent->per.F, 1, ent->ops.H) > ctx->max_lds)
        return fail(BFM_E_UNSUPPORTED, "these parameters do not take the period-blocked plain kernel");
    *H = ent->ops.H;
    *F = ent->per.F;
    return BFM_SUCCESS;
}

// Whether `split` waves per 64 pixels fit the kernel that split_shape found
// (H: the plain window, or the missing-value ring capacity).
bool split_fits(bfm_ctx* ctx, const bfm_params* prm, int split, int H, int F)
{
    if (prm->mask_mode == BFM_MASK_NAN || prm->mask_mode == BFM_MASK_EXPLICIT)
        return split <= (prm->n_hist + F - 1) / F &&
               bfm::masked_periodic_lds_bytes(H, F, split) <= ctx->max_lds;
    return bfm::periodic_split_lds(prm->order, F, split, H) <= ctx->max_lds;
}

}  // namespace

namespace {

// Window and sizes of the simulated null MOSUM for these parameters.
int null_shape(bfm_ctx* ctx, const bfm_params* prm, int* H)
{
    if (!ctx) return fail(BFM_E_INVAL, "ctx is NULL");
    int rc = check(prm, 0, 0);
    if (rc) return rc;
    *H = bfm::window_length(*prm, prm->n_hist);
    if (*H < 1 || *H > prm->n_hist)
        return fail(BFM_E_INVAL, "window length %d must be in [1, n_hist]", *H);
    return BFM_SUCCESS;
}

}  // namespace

int bfm_mosum_null_sup(bfm_ctx* ctx, const bfm_params* prm, uint64_t seed, int64_t path0, int64_t paths,
                       double* sup, void* stream)
{
    int H = 0;
    int rc = null_shape(ctx, prm, &H);
    if (rc) return rc;
    if (paths < 0 || path0 < 0) return fail(BFM_E_INVAL, "path0 and paths must be >= 0");
    if (paths == 0) return BFM_SUCCESS;
    if (!sup) return fail(BFM_E_INVAL, "sup is NULL");
    DeviceGuard g(ctx->device);
    hipError_t e = bfm::launch_mosum_null_sup(prm->n_hist, prm->n_obs, H, seed, path0, paths, sup,
                                              static_cast<hipStream_t>(stream));
    return e == hipSuccess ? BFM_SUCCESS : hip_fail(e, "null MOSUM kernel launch");
}

namespace {

// Checks of both critical-value entry points; *H the window, *rank the order
// statistic.
int critical_args(bfm_ctx* ctx, const bfm_params* prm, double alpha, int64_t paths, int64_t max_paths,
                  const double* lambda, int* H, int64_t* rank)
{
    int rc = null_shape(ctx, prm, H);
    if (rc) return rc;
    if (!(alpha > 0 && alpha < 1)) return fail(BFM_E_INVAL, "alpha must be in (0, 1)");
    if (paths < 1 || paths > max_paths)
        return fail(BFM_E_INVAL, "paths must be in [1, %lld] (got %lld)", (long long)max_paths,
                    (long long)paths);
    if (!lambda) return fail(BFM_E_INVAL, "lambda is NULL");
    *rank = (int64_t)std::ceil((1.0 - alpha) * (double)paths - 1e-9);
    *rank = std::max<int64_t>(1, std::min(*rank, paths));
    return BFM_SUCCESS;
}

// Simulation and selection over `sup` (paths doubles) and `counts` (256 uint32).
hipError_t critical_on(const bfm_params* prm, int H, int64_t paths, uint64_t seed, int64_t rank,
                       double* sup, uint32_t* counts, double* lambda, hipStream_t s)
{
    hipError_t e = bfm::launch_mosum_null_sup(prm->n_hist, prm->n_obs, H, seed, 0, paths, sup, s);
    if (e == hipSuccess) e = bfm::select_rank(sup, paths, rank, counts, lambda, s);
    return e;
}

}  // namespace

int bfm_critical_value(bfm_ctx* ctx, const bfm_params* prm, double alpha, int64_t paths, uint64_t seed,
                       double* lambda, void* stream)
{
    int H = 0;
    int64_t rank = 0;
    int rc = critical_args(ctx, prm, alpha, paths, (int64_t)1 << 31, lambda, &H, &rank);
    if (rc) return rc;
    DeviceGuard g(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    void* buf = nullptr;
    hipError_t e = hipMalloc(&buf, (size_t)paths * sizeof(double) + 256 * sizeof(uint32_t));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(null paths)");
    double* sup = static_cast<double*>(buf);
    e = critical_on(prm, H, paths, seed, rank, sup, reinterpret_cast<uint32_t*>(sup + paths), lambda, s);
    // select_rank has synchronised the stream; the buffer is idle.
    hipError_t ef = hipFree(buf);
    if (e != hipSuccess) return hip_fail(e, "critical value");
    if (ef != hipSuccess) return hip_fail(ef, "hipFree(null paths)");
    return BFM_SUCCESS;
}

int bfm_critical_value_noalloc(bfm_ctx* ctx, const bfm_params* prm, double alpha, int64_t paths,
                               uint64_t seed, double* lambda, void* stream)
{
    int H = 0;
    int64_t rank = 0;
    int rc = critical_args(ctx, prm, alpha, paths, BFM_NOALLOC_MAX_PATHS, lambda, &H, &rank);
    if (rc) return rc;
    void* buf = bfm::noalloc_scratch(ctx->device);  // looked up by bfm_create
    if (!buf) return fail(BFM_E_HIP, "no scratch address for device %d", ctx->device);
    DeviceGuard g(ctx->device);
    double* sup = static_cast<double*>(buf);
    uint32_t* counts = reinterpret_cast<uint32_t*>(static_cast<unsigned char*>(buf) +
                                                   (size_t)BFM_NOALLOC_MAX_PATHS * sizeof(double));
    hipError_t e = critical_on(prm, H, paths, seed, rank, sup, counts, lambda, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? BFM_SUCCESS : hip_fail(e, "critical value (no allocation)");
}

int bfm_tune_set(bfm_ctx* ctx, const bfm_params* prm, int32_t y_dtype, int64_t P, int32_t split)
{
    int H = 0, F = 0;
    int rc = split_shape(ctx, prm, y_dtype, P, P, &H, &F);
    if (rc) return rc;
    if (split != 1 && split != 2 && split != 4 && split != 8)
        return fail(BFM_E_INVAL, "split must be 1, 2, 4 or 8 (got %d)", split);
    if (!split_fits(ctx, prm, split, H, F))
        return fail(BFM_E_UNSUPPORTED, "split %d needs more LDS than a workgroup has, or more waves than "
                    "the history has blocks", split);
    std::lock_guard<std::mutex> lock(ctx->mu);
    ctx->tune[tune_key(*prm, y_dtype, P, H, F)] = split;
    return BFM_SUCCESS;
}

int bfm_autotune(bfm_ctx* ctx, const bfm_params* prm, const void* Y, int32_t y_dtype, int64_t P,
                 int64_t ld, void* stream, int32_t* split, double* times_us)
{
    int H = 0, F = 0;
    int rc = split_shape(ctx, prm, y_dtype, P, ld, &H, &F);
    if (rc) return rc;
    if (P < 1 || !Y) return fail(BFM_E_INVAL, "autotune needs P >= 1 and Y");
    if (prm->mask_mode == BFM_MASK_EXPLICIT)
        return fail(BFM_E_UNSUPPORTED, "autotune times the NaN mask mode (no validity mask is passed); "
                    "pin a split for BFM_MASK_EXPLICIT with bfm_tune_set");
    DeviceGuard g(ctx->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    bfm_outputs out{};
    out.out_dtype = BFM_OUT_F32;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(&out.brk, (size_t)P * 4);
    if (e == hipSuccess) e = hipMalloc(&out.mag, (size_t)P * 4);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    const int cand[4] = {1, 2, 4, 8};
    double med[4] = {0, 0, 0, 0};
    int best = 0;
    const auto key = tune_key(*prm, y_dtype, P, H, F);
    for (int i = 0; i < 4 && e == hipSuccess && rc == BFM_SUCCESS; ++i) {
        if (!split_fits(ctx, prm, cand[i], H, F)) continue;
        {
            std::lock_guard<std::mutex> lock(ctx->mu);
            ctx->tune[key] = cand[i];
        }
        std::vector<double> t;
        for (int r = 0; r < 7 && rc == BFM_SUCCESS && e == hipSuccess; ++r) {
            (void)hipEventRecord(e0, st);
            rc = bfm_fit_monitor_typed(ctx, prm, Y, y_dtype, P, ld, nullptr, 0, &out, st);
            (void)hipEventRecord(e1, st);
            e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (r >= 2) t.push_back(1e3 * (double)ms);  // the first two warm up
        }
        if (t.empty()) continue;
        std::sort(t.begin(), t.end());
        med[i] = t[t.size() / 2];
        if (med[best] == 0.0 || med[i] < med[best]) best = i;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (out.brk) (void)hipFree(out.brk);
    if (out.mag) (void)hipFree(out.mag);
    if (rc) return rc;
    if (e != hipSuccess) return hip_fail(e, "autotune");
    {
        std::lock_guard<std::mutex> lock(ctx->mu);
        ctx->tune[key] = cand[best];
    }
    if (split) *split = cand[best];
    if (times_us)
        for (int i = 0; i < 4; ++i) times_us[i] = med[i];
    return BFM_SUCCESS;
}

}  // extern "C"
