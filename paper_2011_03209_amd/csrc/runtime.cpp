// runtime.cpp -- host side of libmapper_gpu: the C ABI of include/mapper_gpu.h.
//
// One mapper_run is a fixed sequence of device stages on one stream (lens ->
// range -> cover -> pullback sets -> panels -> distance tiles -> FP64 band
// recheck -> components -> labels -> border -> nodes/edges).  The host reads
// back only what sizes the next stage: the lens range (to place the interval
// endpoints), the element sizes (to lay out tiles and the bitmask), the band
// count and the node/edge counts, then the finished graph.
//
// Device memory is sub-allocated from the caller's arena (first fit, 256-byte
// aligned).  Requests submitted for serving run on worker threads, one per
// caller-provided stream; a request that cannot get its workspace releases
// everything it holds and waits for memory to be returned, so admission never
// deadlocks.
#include "internal.h"
#include "../../include/mapper_gpu.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <exception>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

using namespace mgpu;

namespace {

thread_local std::string g_last_error = "no error";

mapper_status fail(mapper_status st, const std::string &msg) {
    g_last_error = msg;
    return st;
}

struct DevError {
    hipError_t e;
    int line;
};

#define HIPCHK(x)                                                        \
    do {                                                                 \
        hipError_t _e = (x);                                             \
        if (_e != hipSuccess) throw DevError{_e, __LINE__};              \
    } while (0)

struct NoMem {
    uint64_t want;
};

// ------------------------------------------------------------------ arena
class Arena {
  public:
    void init(char *base, uint64_t bytes) {
        base_ = base;
        size_ = bytes;
        free_.clear();
        if (bytes) free_[0] = bytes;
    }
    // First fit; returns nullptr if no block fits.
    void *alloc(uint64_t bytes) {
        std::lock_guard<std::mutex> lk(mu_);
        return alloc_locked(bytes);
    }
    void release(void *p) {
        if (!p) return;
        {
            std::lock_guard<std::mutex> lk(mu_);
            uint64_t off = (uint64_t)((char *)p - base_);
            auto it = used_.find(off);
            if (it == used_.end()) return;
            uint64_t sz = it->second;
            used_.erase(it);
            in_use_ -= sz;
            auto nx = free_.lower_bound(off);
            if (nx != free_.end() && off + sz == nx->first) {
                sz += nx->second;
                nx = free_.erase(nx);
            }
            if (nx != free_.begin()) {
                auto pv = std::prev(nx);
                if (pv->first + pv->second == off) {
                    pv->second += sz;
                    ++epoch_;
                    cv_.notify_all();
                    return;
                }
            }
            free_[off] = sz;
            ++epoch_;
        }
        cv_.notify_all();
    }
    uint64_t in_use() const { return in_use_; }
    uint64_t peak() const { return peak_; }
    uint64_t epoch() {
        std::lock_guard<std::mutex> lk(mu_);
        return epoch_;
    }
    // Wait until memory is returned after `seen` or the timeout passes.
    void wait_release(uint64_t seen, int ms) {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait_for(lk, std::chrono::milliseconds(ms), [&] { return epoch_ != seen; });
    }

  private:
    void *alloc_locked(uint64_t bytes) {
        bytes = (bytes + 255) & ~(uint64_t)255;
        if (bytes == 0) bytes = 256;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                const uint64_t off = it->first, rest = it->second - bytes;
                free_.erase(it);
                if (rest) free_[off + bytes] = rest;
                used_[off] = bytes;
                in_use_ += bytes;
                peak_ = std::max(peak_.load(), in_use_.load());
                return base_ + off;
            }
        }
        return nullptr;
    }
    char *base_ = nullptr;
    uint64_t size_ = 0;
    std::map<uint64_t, uint64_t> free_, used_;
    std::atomic<uint64_t> in_use_{0}, peak_{0};
    uint64_t epoch_ = 0;
    std::mutex mu_;
    std::condition_variable cv_;
};

// Allocations of one run, released together.
// s: the stream whose work uses the allocations.  Normal paths release a
// scope only after synchronizing that stream.  When an exception unwinds a
// scope (an arena allocation that fails mid-run, a HIP error), kernels queued
// earlier may still be running: the stream is synchronized here first, so
// that memory they use is not handed to another stream's request meanwhile.
// A scope over a run's reservation may fall back to the context arena for
// what the reservation cannot hold (counted in overflow()).
class Scope {
  public:
    Scope(Arena &a, hipStream_t s, Arena *fallback = nullptr)
        : a_(a), fb_(fallback), s_(s), exc_(std::uncaught_exceptions()) {}
    ~Scope() {
        if (!held_.empty() && std::uncaught_exceptions() > exc_) (void)hipStreamSynchronize(s_);
        release_all();
    }
    template <typename T>
    T *get(uint64_t count) {
        const uint64_t b = count * sizeof(T) + 16;
        Arena *src = &a_;
        void *p = a_.alloc(b);
        if (!p && fb_) {
            src = fb_;
            p = fb_->alloc(b);
            if (p) overflow_ += b;
        }
        if (!p) throw NoMem{count * sizeof(T)};
        held_.push_back({p, src});
        bytes_ += count * sizeof(T);
        return (T *)p;
    }
    // Hold a block taken from arena a directly (released with the scope).
    void adopt(void *p, Arena &a) {
        if (p) held_.push_back({p, &a});
    }
    // Release one allocation early (its stream work must be complete or
    // ordered before any reuse: callers synchronize first).
    void release(void *p) {
        for (size_t i = 0; i < held_.size(); ++i)
            if (held_[i].first == p) {
                held_[i].second->release(p);
                held_.erase(held_.begin() + (std::ptrdiff_t)i);
                return;
            }
    }
    void release_all() {
        for (auto &h : held_) h.second->release(h.first);
        held_.clear();
        bytes_ = 0;
    }
    uint64_t bytes() const { return bytes_; }
    uint64_t overflow() const { return overflow_; }

  private:
    Arena &a_;
    Arena *fb_;
    hipStream_t s_;
    int exc_;
    std::vector<std::pair<void *, Arena *>> held_;
    uint64_t bytes_ = 0, overflow_ = 0;
};

// Thrown when a serving request's reservation (taken after binning, before
// the tile pass) does not fit: the request waits and retries from the start,
// having run no tile pass.
struct AdmitWait {
    uint64_t want;
};

// HIP events for stage timings, kept for reuse: a run marks about a dozen
// stage boundaries, and serving runs many small requests.
class EventPool {
  public:
    ~EventPool() {
        for (hipEvent_t e : free_) (void)hipEventDestroy(e);
    }
    hipEvent_t get() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            if (!free_.empty()) {
                hipEvent_t e = free_.back();
                free_.pop_back();
                return e;
            }
        }
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        return e;
    }
    void put(hipEvent_t e) {
        std::lock_guard<std::mutex> lk(mu_);
        free_.push_back(e);
    }

  private:
    std::mutex mu_;
    std::vector<hipEvent_t> free_;
};

int bits_for(uint64_t maxval) {   // bits needed to hold values in [0, maxval]
    int b = 0;
    while (b < 64 && (maxval >> b) != 0) ++b;
    return b;
}

}  // namespace

// ---------------------------------------------------------------- objects

struct ParamsCopy {
    mapper_params p{};
    std::vector<float> dir[2];
    std::vector<double> val[2];
};

struct Request;

struct mapper_context {
    int device = 0;
    int cus = 256;
    Arena arena;
    hipStream_t stream = nullptr;
    std::vector<hipStream_t> slots;
    // serving
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Request *> pending;
    std::unordered_map<uint64_t, Request *> tickets;
    std::vector<std::thread> workers;
    uint64_t next_ticket = 1;
    int active = 0;
    bool stop = false;
    // a request that had to wait for its reservation: no other request is
    // started until it has its reservation (so a large request is not
    // overtaken forever by a stream of small ones)
    const void *hol = nullptr;
    EventPool events;
    // autotuner cache: (d, eps bucket, norm bucket) -> precision
    std::mutex tune_mu;
    std::map<std::tuple<int, int, int>, int> tune;   // TuneKey -> precision
};

struct mapper_cloud {
    mapper_context *ctx = nullptr;
    float *X = nullptr;
    int64_t n = 0;
    int32_t d = 0;
    float maxabs = 0.f;
    uint8_t *cell = nullptr;           // landmark cell of each point (locality order), or null
    uint8_t *farcell = nullptr;        // per point: its farthest landmark's cell (the eccentricity's first pass)
    float *ogap = nullptr;             // per point of the outlier cell: distance bound to every landmark cell
    uint16_t *okey = nullptr;          // per point: cell << 8 | rank of its outlier gap (the slot order key)
    uint32_t *korder = nullptr;        // the points in okey order (stable): slots of the screened k-NN
    int32_t cell_bits = 0;             // bits of okey in the binning key
    int32_t ncell = 0;
    std::vector<double> cell_gap;      // ncell x ncell: lower bound of the distance between two cells' points
                                       // before eps (landmark distance - both radii), FP64
    std::vector<double> cell_far;      // ncell x ncell: upper bound of it (+inf where the outlier cell takes part)
    std::atomic<int> inflight{0};
    mutable double med_norm2 = -1.0;   // median squared row norm (autotuner key; under tune_mu)
};

struct mapper_graph {
    std::vector<int32_t> node_element;
    std::vector<int64_t> node_offsets;
    std::vector<int32_t> node_members;
    std::vector<int32_t> edges;
    std::vector<int32_t> weights;
    mapper_run_stats stats{};
    std::map<std::string, std::pair<std::vector<char>, int64_t>> stages;
};

struct Request {
    uint64_t ticket = 0;
    int32_t waits = 0;         // times it waited for its reservation
    int32_t redone = 0;        // tile passes it lost to a later shortage
    const mapper_cloud *cloud = nullptr;
    ParamsCopy params;
    bool done = false;
    mapper_status status = MAPPER_OK;
    std::string err;
    mapper_graph *graph = nullptr;
};

namespace {

mapper_status validate(const mapper_cloud *c, const mapper_params *p) {
    if (!c || !p) return fail(MAPPER_EINVAL, "null cloud or params");
    if (p->n_axes < 1 || p->n_axes > 2) return fail(MAPPER_EINVAL, "n_axes must be 1 or 2");
    if (!(p->eps >= 0.0) || !std::isfinite(p->eps)) return fail(MAPPER_EINVAL, "eps must be finite and >= 0");
    if (p->min_pts < 1) return fail(MAPPER_EINVAL, "min_pts must be >= 1");
    if (p->precision < 0 || p->precision > MAPPER_PREC_AUTO) return fail(MAPPER_EINVAL, "bad precision");
    int64_t ne = 1;
    for (int a = 0; a < p->n_axes; ++a) {
        const mapper_axis &ax = p->axis[a];
        if (ax.n_intervals < 1) return fail(MAPPER_EINVAL, "n_intervals must be >= 1");
        if (!(ax.overlap >= 0.0 && ax.overlap < 1.0)) return fail(MAPPER_EINVAL, "overlap must be in [0, 1)");
        if (ax.cover != MAPPER_COVER_UNIFORM && ax.cover != MAPPER_COVER_BALANCED)
            return fail(MAPPER_EINVAL, "cover must be MAPPER_COVER_UNIFORM or MAPPER_COVER_BALANCED");
        if (ax.kind < 0 || ax.kind > MAPPER_LENS_ECCENTRICITY) return fail(MAPPER_EINVAL, "bad lens kind");
        if (ax.kind == MAPPER_LENS_KNN_DISTANCE && (ax.column < 1 || ax.column > 16 || (int64_t)ax.column > c->n - 1))
            return fail(MAPPER_EINVAL, "k-NN distance lens: k (the column field) must be in [1, min(16, n - 1)]");
        if (ax.kind == MAPPER_LENS_ECCENTRICITY && c->n < 2)
            return fail(MAPPER_EINVAL, "eccentricity lens needs at least two points");
        if (ax.kind == MAPPER_LENS_COLUMN && (ax.column < 0 || ax.column >= c->d))
            return fail(MAPPER_EINVAL, "lens column out of range");
        if (ax.kind == MAPPER_LENS_PROJECTION) {
            if (!ax.direction) return fail(MAPPER_EINVAL, "projection lens needs a direction");
            for (int j = 0; j < c->d; ++j)
                if (!std::isfinite(ax.direction[j])) return fail(MAPPER_EINVAL, "non-finite direction");
        }
        if (ax.kind == MAPPER_LENS_VALUES) {
            if (!ax.values) return fail(MAPPER_EINVAL, "values lens needs values");
            for (int64_t i = 0; i < c->n; ++i)
                if (!std::isfinite(ax.values[i])) return fail(MAPPER_EINVAL, "non-finite lens value");
        }
        ne *= ax.n_intervals;
    }
    if (ne > (1 << 24)) return fail(MAPPER_EINVAL, "more than 2^24 cover elements");
    return MAPPER_OK;
}

void copy_params(const mapper_cloud *c, const mapper_params *p, ParamsCopy &out) {
    out.p = *p;
    for (int a = 0; a < p->n_axes; ++a) {
        const mapper_axis &ax = p->axis[a];
        if (ax.kind == MAPPER_LENS_PROJECTION) {
            out.dir[a].assign(ax.direction, ax.direction + c->d);
            out.p.axis[a].direction = out.dir[a].data();
        } else {
            out.p.axis[a].direction = nullptr;
        }
        if (ax.kind == MAPPER_LENS_VALUES) {
            out.val[a].assign(ax.values, ax.values + c->n);
            out.p.axis[a].values = out.val[a].data();
        } else {
            out.p.axis[a].values = nullptr;
        }
    }
}

// Interval endpoints (Background section: n intervals of one length with
// fractional overlap p covering [m, M]); evaluated exactly as written, in
// FP64, with contraction disabled for this translation unit.
void cover_endpoints(double m, double M, int n, double p, std::vector<double> &lo,
                     std::vector<double> &hi) {
    lo.resize(n);
    hi.resize(n);
    const double L = (M - m) / ((double)n - (double)(n - 1) * p);
    const double s = L * (1.0 - p);
    for (int k = 0; k < n; ++k) {
        lo[k] = m + (double)k * s;
        hi[k] = (k == n - 1) ? M : lo[k] + L;
    }
}

double key_to_double(unsigned long long k) {
    const unsigned long long b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
    double d;
    std::memcpy(&d, &b, 8);
    return d;
}

template <typename T>
void d2h(std::vector<T> &dst, const T *src, int64_t count, hipStream_t s) {
    dst.resize((size_t)std::max<int64_t>(count, 0));
    if (count > 0) HIPCHK(hipMemcpyAsync(dst.data(), src, (size_t)count * sizeof(T), hipMemcpyDeviceToHost, s));
}

template <typename T>
void h2d(T *dst, const T *src, int64_t count, hipStream_t s) {
    if (count > 0) HIPCHK(hipMemcpyAsync(dst, src, (size_t)count * sizeof(T), hipMemcpyHostToDevice, s));
}

// Events of one run.  An event goes back to the pool once the stream has
// passed it, so a reused event is never still pending.
struct Events {
    std::vector<hipEvent_t> ev;
    hipStream_t s;
    EventPool &pool;
    Events(hipStream_t st, EventPool &p) : s(st), pool(p) {}
    ~Events() {
        for (auto e : ev) {
            (void)hipEventSynchronize(e);
            pool.put(e);
        }
    }
    void mark() {
        hipEvent_t e = pool.get();
        ev.push_back(e);
        HIPCHK(hipEventRecord(e, s));
    }
    double ms(size_t a, size_t b) {
        if (b >= ev.size()) return 0.0;
        float t = 0;
        (void)hipEventElapsedTime(&t, ev[a], ev[b]);
        return t;
    }
};

// Balanced cover: the uniform cover of the rank axis [0, n-1], each rank
// interval [a, b] rounded outward to [floor a, ceil b] and read back as lens
// values from a device radix sort of the lens.
void balanced_endpoints(Arena &arena, const double *f, int64_t n, int nint, double p, std::vector<double> &lo,
                        std::vector<double> &hi, hipStream_t s) {
    std::vector<double> rl, rh;
    cover_endpoints(0.0, (double)(n - 1), nint, p, rl, rh);
    std::vector<int64_t> rank(2 * (size_t)nint);
    for (int k = 0; k < nint; ++k) {
        rank[k] = std::max<int64_t>(0, (int64_t)std::floor(rl[k]));
        rank[nint + k] = std::min<int64_t>(n - 1, (int64_t)std::ceil(rh[k]));
    }
    Scope mem(arena, s);                                    // released on return, after the sync
    uint64_t *k1 = mem.get<uint64_t>(n), *k2 = mem.get<uint64_t>(n);
    uint32_t *v1 = mem.get<uint32_t>(n), *v2 = mem.get<uint32_t>(n);
    void *tmp = mem.get<char>(sort_temp_bytes(n));
    int64_t *drank = mem.get<int64_t>(2 * nint);
    double *dval = mem.get<double>(2 * nint);
    HIPCHK(launch_lens_keys(f, n, k1, v1, s));
    bool alt = false;
    HIPCHK(radix_sort_pairs(k1, v1, k2, v2, n, 64, tmp, &alt, s));
    h2d(drank, rank.data(), 2 * nint, s);
    HIPCHK(launch_rank_values(alt ? k2 : k1, drank, 2 * nint, dval, s));
    std::vector<double> val;
    d2h(val, dval, 2 * nint, s);
    HIPCHK(hipStreamSynchronize(s));
    lo.assign(val.begin(), val.begin() + nint);
    hi.assign(val.begin() + nint, val.end());
}

// ----------------------------------------------------------------- autotuner
// Precision choice (MAPPER_PREC_AUTO), measured: on the first run of its
// kind, each of the five precisions packs the run's panels and runs the tile
// kernel on an evenly strided sample of up to 8192 of the run's own tile
// pairs (after screening), timed with HIP events; its band pairs are counted.
// Predicted time = sampled tile time x (tile pairs / sample) + band pairs x
// (tile pairs / sample) x the FP64 recheck's cost per pair (a gather of two
// FP32 rows at 7 TB/s, as the recheck kernel runs).  The fastest is cached
// per kind of run (tune_key) and used without sampling afterwards.
using TuneKey = std::tuple<int, int, int>;

// The autotuner's cache key: d, eps^2 against the cloud's median squared row
// norm (quarter octaves) and the pair count (octaves).
TuneKey tune_key(int d, double E, double med_norm2, double pairs) {
    const int eb = (int)std::floor(std::log2(std::max(E, 1e-300) / std::max(med_norm2, 1e-300)) * 4.0);
    const int nbk = (int)std::floor(std::log2(std::max(pairs, 1.0)));
    return TuneKey{d, eb, nbk};
}

// Median squared row norm of the cloud from 4096 evenly spaced rows, taken
// once per cloud.
double cloud_median_norm2(mapper_context *ctx, const mapper_cloud *cloud, hipStream_t s) {
    {
        std::lock_guard<std::mutex> lk(ctx->tune_mu);
        if (cloud->med_norm2 >= 0) return cloud->med_norm2;
    }
    const int64_t ns = std::min<int64_t>(cloud->n, 4096);
    std::vector<int32_t> rows((size_t)ns);
    for (int64_t q = 0; q < ns; ++q) rows[(size_t)q] = (int32_t)(q * cloud->n / ns);
    Scope tmp(ctx->arena, s);
    int32_t *dr = tmp.get<int32_t>(ns);
    double *dn = tmp.get<double>(ns);
    h2d(dr, rows.data(), ns, s);
    HIPCHK(launch_row_norm2(dr, ns, cloud->X, cloud->d, dn, s));
    std::vector<double> nn;
    d2h(nn, dn, ns, s);
    HIPCHK(hipStreamSynchronize(s));
    std::nth_element(nn.begin(), nn.begin() + nn.size() / 2, nn.end());
    std::lock_guard<std::mutex> lk(ctx->tune_mu);
    cloud->med_norm2 = nn[nn.size() / 2];
    return cloud->med_norm2;
}

// The cached choice for key, or -1.
int cached_precision(mapper_context *ctx, const TuneKey &key) {
    std::lock_guard<std::mutex> lk(ctx->tune_mu);
    auto it = ctx->tune.find(key);
    return it == ctx->tune.end() ? -1 : it->second;
}

int tune_precision(mapper_context *ctx, const mapper_cloud *cloud, const TileTable &tt, int64_t n_tiles,
                   const uint32_t *slot_point, int64_t S, double scale, double E, const TuneKey &key,
                   mapper_run_stats &st, hipStream_t s) {
    const int32_t d = cloud->d;
    const int64_t m = std::min<int64_t>(n_tiles, 8192);
    int best = P_BF16X3;
    if (m > 0 && S > 0) {
        Scope tmp(ctx->arena, s);
        TileItem *smp = tmp.get<TileItem>(m);
        HIPCHK(launch_sample_items(tt.items, n_tiles, m, smp, s));
        TileTable ts = tt;
        ts.items = smp;
        ts.n_items = m;
        float *thrA = tmp.get<float>(S), *thrB = tmp.get<float>(S);
        int32_t *cnt = tmp.get<int32_t>(S);
        uint32_t *bm = tmp.get<uint32_t>((uint64_t)m * TILE_WORDS);
        uint32_t *bmk = tmp.get<uint32_t>((uint64_t)m * TILE_WORDS);    // band masks
        const int nseg = 8;
        const int64_t cap = 256;                        // band pairs are counted; few are stored
        unsigned long long *bn = tmp.get<unsigned long long>(nseg);
        BandPair *band = tmp.get<BandPair>((uint64_t)nseg * cap);
        uint64_t most = 0;
        for (int p = 0; p < 5; ++p) most = std::max<uint64_t>(most, (uint64_t)panel_row_stride(p, panel_dp(p, d)));
        char *panel = tmp.get<char>((uint64_t)S * most);
        const double per_band_ms = 8.0 * d / 7.0e12 * 1e3;
        double bestt = 1e300;
        for (int p = 0; p < 5; ++p) {
            PackArgs pk{};
            pk.X = cloud->X;
            pk.d = d;
            pk.dp = panel_dp(p, d);
            pk.slot_point = slot_point;
            pk.n_slots = S;
            pk.prec = p;
            pk.scale = scale;
            pk.n_levels = 1;
            pk.E_scaled[0] = E * scale * scale;
            pk.panel = panel;
            pk.thrA = thrA;
            pk.thrB = thrB;
            HIPCHK(launch_pack(pk, s));
            HIPCHK(hipMemsetAsync(cnt, 0, (size_t)S * 4, s));
            HIPCHK(hipMemsetAsync(bn, 0, (size_t)nseg * 8, s));
            TileArgs ta{};
            ta.tt = ts;
            ta.panel = panel;
            ta.dp = pk.dp;
            ta.thrA = thrA;
            ta.thrB = thrB;
            ta.bitmask = bm;
            ta.count = cnt;
            ta.band = band;
            ta.band_n = bn;
            ta.band_cap = cap;
            ta.nseg = nseg;
            ta.n_levels = 1;
            ta.level_slots = S;
            ta.level_words = (uint64_t)m * TILE_WORDS;
            ta.bandmask = bmk;
            Events ev(s, ctx->events);
            ev.mark();
            HIPCHK(launch_tiles(p, ta, s));
            ev.mark();
            HIPCHK(launch_band_collect(ts, bmk, 1, ta.level_words, band, bn, cap, nseg, s));
            std::vector<unsigned long long> bh;
            d2h(bh, bn, nseg, s);
            HIPCHK(hipStreamSynchronize(s));
            uint64_t nb = 0;
            for (unsigned long long v : bh) nb += v;
            const double scale_up = (double)n_tiles / (double)m;
            const double t = ev.ms(0, 1) * scale_up + (double)nb * scale_up * per_band_ms;
            st.tune_pred_ms[p] = t;
            if (t < bestt) {
                bestt = t;
                best = p;
            }
        }
        st.tune_sampled = 1;
    }
    std::lock_guard<std::mutex> lk(ctx->tune_mu);
    ctx->tune[key] = best;
    return best;
}

// k-NN screening and FP64 step on the whole cloud (see k_knn): dout[i]
// (device) = the k-th smallest canonical D over j != i (mode 0) or the
// largest (mode 1, k = 1).  Synchronous; its work arrays are released on
// return.
void knn_device(mapper_context *ctx, const mapper_cloud *cloud, int32_t k, int32_t mode, int prec,
                double *dout, mapper_run_stats &st, hipStream_t s) {
    Scope mem(ctx->arena, s);
    const int64_t n = cloud->n;
    const int32_t d = cloud->d;
    const int32_t T = (int32_t)((n + TILE - 1) / TILE);
    // column-block chunks: enough workgroups to fill the chip twice over
    const int32_t C = (int32_t)std::max<int64_t>(1, std::min<int64_t>(T, (4 * ctx->cus + T - 1) / T));
    st.precision = prec;
    st.tile_m = st.tile_n = TILE;
    st.split_terms = prec_is_split(prec) ? 3 : 1;
    st.pairs = n * (n - 1);
    st.tiles = 2 * (int64_t)T * T;
    // screening by the cloud's cells: slots in cell order, per row block the
    // column blocks its rows may need (k_knn_lists)
    const bool screen = cloud->korder && cloud->cell && d <= BALL_DMAX && cloud->ncell >= 2 &&
                        (int64_t)T * T <= (1ll << 28);
    const uint32_t *slots = nullptr;
    if (screen) {
        slots = cloud->korder;
    } else {
        std::vector<uint32_t> iota((size_t)n);
        for (int64_t i = 0; i < n; ++i) iota[i] = (uint32_t)i;
        uint32_t *ident = mem.get<uint32_t>(n);
        h2d(ident, iota.data(), n, s);
        slots = ident;
    }
    double scale = 1.0;
    if (cloud->maxabs > 0) scale = std::ldexp(1.0, 10 - std::ilogb((double)cloud->maxabs));
    const int dp = panel_dp(prec, d);
    PackArgs pk{};
    pk.X = cloud->X;
    pk.d = d;
    pk.dp = dp;
    pk.slot_point = slots;
    pk.n_slots = n;
    pk.prec = prec;
    pk.scale = scale;
    pk.n_levels = 1;
    pk.E_scaled[0] = 0.0;                               // thresholds at eps = 0: |x|^2/2 +- e
    pk.panel = mem.get<char>((uint64_t)n * (uint64_t)panel_row_stride(prec, dp));
    float *hU = mem.get<float>(n), *hL = mem.get<float>(n);
    pk.thrA = hU;
    pk.thrB = hL;
    HIPCHK(launch_pack(pk, s));
    KnnArgs ka{};
    ka.t.panel = pk.panel;
    ka.t.dp = dp;
    ka.t.n_levels = 1;
    ka.mode = mode;
    ka.k = k;
    ka.n = n;
    ka.T = T;
    ka.C = C;
    ka.hU = hU;
    ka.hL = hL;
    ka.part = mem.get<float>((uint64_t)C * T * TILE * 4 * KNN_KMAX);
    float *thr = mem.get<float>(n);
    ka.thr = thr;
    unsigned long long *cmask = nullptr, *fmask = nullptr;
    double *dgap = nullptr;
    int32_t *jlist = nullptr, *jcount = nullptr;
    const double shrink = 1.0 - ((double)d + 8.0) * 0x1.0p-52;
    const int nall = cloud->ncell;
    auto list_sum = [&]() {
        std::vector<int32_t> jc;
        d2h(jc, jcount, T, s);
        HIPCHK(hipStreamSynchronize(s));
        int64_t t = 0;
        for (int32_t v : jc) t += v;
        return t;
    };
    int64_t tiles1 = (int64_t)T * T;
    if (screen) {
        // the cells of every row block (k_tile_cells on one element of all
        // slots; the near table is not used here)
        cmask = mem.get<unsigned long long>(T);
        unsigned long long *nmask = mem.get<unsigned long long>(T);
        unsigned long long *near0 = mem.get<unsigned long long>(CELL_MAX);
        int64_t *eo = mem.get<int64_t>(2), *rbo = mem.get<int64_t>(1);
        const int64_t eoh[2] = {0, n}, rboh[1] = {0};
        h2d(eo, eoh, 2, s);
        h2d(rbo, rboh, 1, s);
        HIPCHK(hipMemsetAsync(near0, 0, CELL_MAX * 8, s));
        HIPCHK(launch_tile_cells(slots, eo, rbo, 1, T, cloud->cell, nullptr, nall - 1, shrink, 0.0, near0, cmask,
                                 nmask, s));
        if (mode == 1 && cloud->farcell) {              // the cells of the rows' farthest landmarks
            fmask = mem.get<unsigned long long>(T);
            HIPCHK(launch_tile_cells(slots, eo, rbo, 1, T, cloud->farcell, nullptr, nall - 1, shrink, 0.0, near0,
                                     fmask, nmask, s));
        }
        dgap = mem.get<double>(2 * (uint64_t)nall * nall);      // the gap table, then the far table
        h2d(dgap, cloud->cell_gap.data(), (int64_t)nall * nall, s);
        h2d(dgap + (size_t)nall * nall, cloud->cell_far.data(), (int64_t)nall * nall, s);
        jlist = mem.get<int32_t>((uint64_t)T * T);
        jcount = mem.get<int32_t>(T);
        HIPCHK(launch_knn_lists(T, n, mode, cmask, fmask, dgap, dgap + (size_t)nall * nall, nall, nullptr, 0.0,
                                shrink, jlist, jcount, s));
        ka.jlist = jlist;
        ka.jcount = jcount;
        tiles1 = list_sum();
    }
    Events ev(s, ctx->events);
    ev.mark();
    HIPCHK(launch_knn_pass(prec, 1, ka, s));
    HIPCHK(launch_knn_merge(ka.part, C, T, n, k, thr, s));
    int64_t tiles2 = (int64_t)T * T;
    if (screen) {
        HIPCHK(launch_knn_lists(T, n, mode, cmask, nullptr, dgap, dgap + (size_t)nall * nall, nall, thr,
                                1.0 / (scale * scale), shrink, jlist, jcount, s));
    }
    ev.mark();
    if (screen) tiles2 = list_sum();
    st.tiles = tiles1 + tiles2;
    // candidate lists: up to 256 MiB at first (1024 entries at most); a row
    // with more candidates than that redoes pass 2 with lists as long as it
    int32_t cmax = (int32_t)std::max<int64_t>(64, std::min<int64_t>(1024, (int64_t)(256 << 20) / (4 * n)));
    int32_t *ccnt = mem.get<int32_t>(n);
    int64_t ncand = 0;
    for (;;) {
        ka.cand = mem.get<int32_t>((uint64_t)n * cmax);
        ka.ccnt = ccnt;
        ka.cmax = cmax;
        Events e2(s, ctx->events);
        e2.mark();
        HIPCHK(hipMemsetAsync(ccnt, 0, (size_t)n * 4, s));
        HIPCHK(launch_knn_pass(prec, 2, ka, s));
        e2.mark();
        std::vector<int32_t> cc;
        d2h(cc, ccnt, n, s);
        HIPCHK(hipStreamSynchronize(s));
        int64_t most = 0;
        ncand = 0;
        for (int64_t i = 0; i < n; ++i) {
            most = std::max<int64_t>(most, cc[i]);
            ncand += cc[i];
        }
        st.ms_tiles = ev.ms(0, 1) + e2.ms(0, 1);
        if (most <= cmax) break;
        if (most > (int64_t)0x7fffffff / std::max<int64_t>(n, 1)) throw NoMem{(uint64_t)most * (uint64_t)n * 4};
        mem.release(ka.cand);                           // the stream is idle: the lists go back at once
        cmax = (int32_t)most;
        ++st.tile_launches;
    }
    {
        Events e3(s, ctx->events);
        e3.mark();
        HIPCHK(launch_knn_final(cloud->X, d, n, k, ka.cand, ccnt, cmax, mode, screen ? slots : nullptr, dout, s));
        e3.mark();
        HIPCHK(hipStreamSynchronize(s));
        st.ms_recheck = e3.ms(0, 1);
    }
    st.tile_launches += 1;
    st.band_pairs = ncand;
    st.ms_total = st.ms_tiles + st.ms_recheck;
    st.arena_peak_bytes = mem.bytes();
}

// ------------------------------------------------------------- cloud cells
// The locality order of a cloud (cells.hip), built once when it is
// uploaded.  From an evenly strided sample of 4096 rows: each row's nearest
// other sample row (GPU), the inliers (no more than 4x the median of those
// squared distances away: isolated rows such as uniform background noise
// would otherwise be picked first), up to CELL_MAX - 2 landmarks among the
// inliers by farthest-point sampling (FP64, host), numbered along a
// nearest-neighbour chain.  Every point then goes to its nearest landmark,
// or to the outlier cell when it lies farther from it than 1.5x the largest
// distance of an inlier sample row in that cell.  Each landmark cell gets a
// ball (the landmark, the largest distance of a member); the outlier cell
// has none, and each of its points gets a lower bound of its distance to
// every landmark cell instead (the slot order sorts them by it).  Only
// clouds large enough to fill several tiles get cells, and only when the
// landmarks fit the kernel's LDS; otherwise slots stay in point order.
void build_cells(mapper_context *ctx, mapper_cloud *c, hipStream_t s) {
    const int64_t n = c->n;
    const int32_t d = c->d;
    const int ncell_max = std::min<int>(CELL_MAX - 2, CELL_LDS_FLOATS / std::max(d, 1));
    if (n < 8 * TILE || ncell_max < 8) return;
    const int64_t m = std::min<int64_t>(n, 4096), step = n / m;
    std::vector<float> sub((size_t)(m * d));
    std::vector<float> nn2((size_t)m);
    {
        Scope tmp(ctx->arena, s);
        float *dsub = tmp.get<float>((uint64_t)m * d);
        float *dnn = tmp.get<float>(m);
        HIPCHK(hipMemcpy2DAsync(dsub, (size_t)d * 4, c->X, (size_t)(step * d) * 4, (size_t)d * 4, (size_t)m,
                                hipMemcpyDeviceToDevice, s));
        HIPCHK(launch_sample_nn2(dsub, (int32_t)m, d, dnn, s));
        HIPCHK(hipMemcpyAsync(sub.data(), dsub, sub.size() * 4, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(nn2.data(), dnn, nn2.size() * 4, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
    }
    std::vector<float> sorted_nn = nn2;
    std::nth_element(sorted_nn.begin(), sorted_nn.begin() + m / 2, sorted_nn.end());
    const float inl = 4.0f * sorted_nn[(size_t)(m / 2)];
    std::vector<int64_t> rows;                                  // the inlier sample rows
    for (int64_t i = 0; i < m; ++i)
        if (nn2[(size_t)i] <= inl) rows.push_back(i);
    if ((int64_t)rows.size() < 2 * ncell_max) return;
    auto dist2 = [&](int64_t a, int64_t b) {
        const float *x = &sub[(size_t)(a * d)], *y = &sub[(size_t)(b * d)];
        double acc = 0.0;
        for (int j = 0; j < d; ++j) {
            const double t = (double)x[j] - (double)y[j];
            acc += t * t;
        }
        return acc;
    };
    std::vector<double> dmin(rows.size(), 1e300);
    std::vector<int64_t> pick;
    size_t cur = 0;
    for (int k = 0; k < ncell_max; ++k) {
        pick.push_back(rows[cur]);
        size_t far = 0;
        for (size_t q = 0; q < rows.size(); ++q) {
            dmin[q] = std::min(dmin[q], dist2(rows[q], rows[cur]));
            if (dmin[q] > dmin[far]) far = q;
        }
        if (dmin[far] <= 0.0) break;                            // fewer distinct rows than landmarks
        cur = far;
    }
    const int nc = (int)pick.size();
    if (nc < 2) return;
    // number the landmarks along a nearest-neighbour chain, so that the
    // cells of one cluster (farthest-point sampling splits a large cluster
    // among several landmarks) are consecutive in the slot order
    std::vector<int64_t> chain{pick[0]};
    std::vector<char> used((size_t)nc, 0);
    used[0] = 1;
    for (int k = 1; k < nc; ++k) {
        int best = -1;
        double bd = 0.0;
        for (int q = 0; q < nc; ++q) {
            if (used[(size_t)q]) continue;
            const double t = dist2(chain.back(), pick[(size_t)q]);
            if (best < 0 || t < bd) { best = q; bd = t; }
        }
        used[(size_t)best] = 1;
        chain.push_back(pick[(size_t)best]);
    }
    // each cell's limit: 1.5x the largest distance of an inlier sample row
    // whose nearest landmark it is
    std::vector<float> limit2((size_t)nc, 0.f);
    for (int64_t r : rows) {
        int best = 0;
        double bd = dist2(r, chain[0]);
        for (int k = 1; k < nc; ++k) {
            const double t = dist2(r, chain[(size_t)k]);
            if (t < bd) { bd = t; best = k; }
        }
        limit2[(size_t)best] = std::max(limit2[(size_t)best], (float)(2.25 * bd));
    }
    // landmarks row by row (nc x d), the cells' limits (nc), then the
    // landmarks transposed with CELL_MAX columns (d x CELL_MAX, zero past
    // nc) and their squared norms (CELL_MAX), for the assignment kernel
    const size_t lt_off = ((size_t)nc * d + nc + 63) / 64 * 64;      // 256-byte aligned
    std::vector<float> land(lt_off + (size_t)d * CELL_MAX + CELL_MAX, 0.0f);
    float *lt = land.data() + lt_off, *ln = lt + (size_t)d * CELL_MAX;
    for (int k = 0; k < nc; ++k) {
        const float *src = &sub[(size_t)(chain[k] * d)];
        std::memcpy(&land[(size_t)k * d], src, (size_t)d * 4);
        float nrm = 0.0f;
        for (int j = 0; j < d; ++j) {
            lt[(size_t)j * CELL_MAX + k] = src[j];
            nrm += src[j] * src[j];
        }
        ln[k] = nrm;
    }
    std::memcpy(land.data() + (size_t)nc * d, limit2.data(), (size_t)nc * 4);
    uint8_t *cell = (uint8_t *)ctx->arena.alloc((uint64_t)n);
    uint8_t *farc = (uint8_t *)ctx->arena.alloc((uint64_t)n);
    float *dl = (float *)ctx->arena.alloc((uint64_t)land.size() * 4);
    unsigned long long *r2 = (unsigned long long *)ctx->arena.alloc((uint64_t)CELL_MAX * 8);
    if (!cell || !farc || !dl || !r2) {                         // no room: keep point order
        ctx->arena.release(cell);
        ctx->arena.release(farc);
        ctx->arena.release(dl);
        ctx->arena.release(r2);
        return;
    }
    float *dlim = dl + (size_t)nc * d, *dlt = dl + lt_off, *dln = dlt + (size_t)d * CELL_MAX;
    std::vector<unsigned long long> r2h((size_t)CELL_MAX, 0);
    try {
        HIPCHK(hipMemcpyAsync(dl, land.data(), land.size() * 4, hipMemcpyHostToDevice, s));
        HIPCHK(launch_assign_cells(c->X, n, d, dlt, dln, nc, dlim, cell, farc, s));
        HIPCHK(hipMemsetAsync(r2, 0, (size_t)CELL_MAX * 8, s));
        HIPCHK(launch_cell_radius(c->X, n, d, dl, nc, cell, r2, s));
        HIPCHK(hipMemcpyAsync(r2h.data(), r2, (size_t)CELL_MAX * 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
    } catch (DevError &) {
        (void)hipStreamSynchronize(s);
        ctx->arena.release(cell);
        ctx->arena.release(farc);
        ctx->arena.release(dl);
        ctx->arena.release(r2);
        throw;
    }
    // cell balls: landmark l_c, radius r_c >= max |x - l_c| over its points
    // (relative margin 2^-40 for the FP64 sums, d <= BALL_DMAX); the gap of
    // two cells bounds every distance between their points from below.  Cell
    // nc (the outliers) has no ball: a gap of -1 keeps it near every cell;
    // each of its points gets its own gap to the landmark cells instead.
    const int nall = nc + 1;
    std::vector<double> rad((size_t)nc);
    for (int a = 0; a < nc; ++a) {
        double r2v;
        std::memcpy(&r2v, &r2h[(size_t)a], 8);
        rad[(size_t)a] = std::sqrt(r2v) * (1.0 + 0x1.0p-40);
    }
    float *ogap = (float *)ctx->arena.alloc((uint64_t)n * 4);
    if (ogap) {                                                 // no room: every outlier stays near every cell
        try {
            double *drad = (double *)r2;                            // the radius scratch, reused
            HIPCHK(hipMemcpyAsync(drad, rad.data(), (size_t)nc * 8, hipMemcpyHostToDevice, s));
            HIPCHK(launch_outlier_gap(c->X, n, d, dl, nc, drad, cell, ogap, s));
            HIPCHK(hipStreamSynchronize(s));
        } catch (DevError &) {
            (void)hipStreamSynchronize(s);
            ctx->arena.release(ogap);
            ctx->arena.release(cell);
            ctx->arena.release(farc);
            ctx->arena.release(dl);
            ctx->arena.release(r2);
            throw;
        }
    }
    ctx->arena.release(dl);
    ctx->arena.release(r2);
    c->cell_gap.assign((size_t)nall * nall, -1.0);
    c->cell_far.assign((size_t)nall * nall, std::numeric_limits<double>::infinity());
    for (int a = 0; a < nc; ++a)
        for (int b = 0; b < nc; ++b) {
            const double dc = std::sqrt(dist2(chain[(size_t)a], chain[(size_t)b]));
            if (a != b) c->cell_gap[(size_t)a * nall + b] = dc * (1.0 - 0x1.0p-40) - rad[(size_t)a] - rad[(size_t)b];
            c->cell_far[(size_t)a * nall + b] = dc * (1.0 + 0x1.0p-40) + rad[(size_t)a] + rad[(size_t)b];
        }
    // the slot order key: cell, then (outliers) the gap in 256 quantiles
    // ascending, so that for any eps the outliers within eps of a landmark
    // cell come first in their element and the far ones fill row blocks of
    // their own
    uint16_t *okey = (uint16_t *)ctx->arena.alloc((uint64_t)n * 2);
    uint32_t *korder = nullptr;
    if (okey) {
        std::vector<uint8_t> ch;
        std::vector<float> gh;
        std::vector<uint16_t> kh((size_t)n);
        try {
            d2h(ch, cell, n, s);
            if (ogap) d2h(gh, ogap, n, s);
            HIPCHK(hipStreamSynchronize(s));
            std::vector<float> og;
            if (ogap)
                for (int64_t i = 0; i < n; ++i)
                    if (ch[(size_t)i] == nc) og.push_back(gh[(size_t)i]);
            std::sort(og.begin(), og.end());
            std::vector<float> q;                                   // upper ends of quantiles 0 .. 254
            for (int k = 1; k < 256 && !og.empty(); ++k) q.push_back(og[(size_t)((og.size() - 1) * k / 256)]);
            for (int64_t i = 0; i < n; ++i) {
                const int cc = ch[(size_t)i];
                int gq = 0;
                if (cc == nc && !q.empty())
                    gq = (int)(std::lower_bound(q.begin(), q.end(), gh[(size_t)i]) - q.begin());
                kh[(size_t)i] = (uint16_t)(cc << 8 | gq);
            }
            HIPCHK(hipMemcpyAsync(okey, kh.data(), (size_t)n * 2, hipMemcpyHostToDevice, s));
            // the points in key order (a counting sort, stable), for the k-NN
            korder = (uint32_t *)ctx->arena.alloc((uint64_t)n * 4);
            if (korder) {
                std::vector<int64_t> start((size_t)65537, 0);
                for (int64_t i = 0; i < n; ++i) ++start[(size_t)kh[(size_t)i] + 1];
                for (size_t q = 1; q < start.size(); ++q) start[q] += start[q - 1];
                std::vector<uint32_t> ord((size_t)n);
                for (int64_t i = 0; i < n; ++i) ord[(size_t)start[kh[(size_t)i]]++] = (uint32_t)i;
                HIPCHK(hipMemcpyAsync(korder, ord.data(), (size_t)n * 4, hipMemcpyHostToDevice, s));
            }
            HIPCHK(hipStreamSynchronize(s));
        } catch (DevError &) {
            (void)hipStreamSynchronize(s);
            ctx->arena.release(korder);
            ctx->arena.release(okey);
            ctx->arena.release(ogap);
            ctx->arena.release(cell);
            ctx->arena.release(farc);
            throw;
        }
    }
    if (!okey) {                                                // no room: keep point order
        ctx->arena.release(ogap);
        ctx->arena.release(cell);
        ctx->arena.release(farc);
        return;
    }
    c->ncell = nall;
    c->cell = cell;
    c->farcell = farc;
    c->ogap = ogap;
    c->okey = okey;
    c->korder = korder;
    c->cell_bits = 8 + (32 - __builtin_clz((unsigned)(nall - 1)));
}

// ------------------------------------------------------------------ the run
enum class Phase { Ok, Retry };

// A serving request got its reservation: if it was the head-of-line
// request, other requests may start again.
void admitted(mapper_context *ctx, const void *req) {
    if (!req) return;
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (ctx->hol == req) {
        ctx->hol = nullptr;
        ctx->cv.notify_all();
    }
}


struct RunOut {
    std::vector<mapper_graph *> gs;    // one graph per eps value
    const void *req = nullptr;         // the serving request being run (head-of-line bookkeeping)
    bool tiles_done = false;           // the tile pass has run (a later shortage wastes it)
    ~RunOut() {
        for (mapper_graph *g : gs) delete g;
    }
};

// The graphs of one cloud and parameter set for n_levels eps values
// (eps_list, or P->eps when it is null): lens, cover, binning, panels and
// tiles are shared; every level has its own bitmask, counts and graph.
Phase run_pipeline(mapper_context *ctx, const mapper_cloud *cloud, const mapper_params *P,
                   hipStream_t s, bool may_retry, RunOut &out, const double *eps_list = nullptr,
                   int n_levels = 1, const int32_t *minpts_list = nullptr, int n_minpts = 1) {
    Scope mem(ctx->arena, s);
    Events ev(s, ctx->events);
    const int64_t n = cloud->n;
    const int32_t d = cloud->d;
    const int na = P->n_axes;
    mapper_run_stats st{};
    std::vector<double> Elev(n_levels);
    for (int lv = 0; lv < n_levels; ++lv) {
        const double e = eps_list ? eps_list[lv] : P->eps;
        Elev[lv] = e * e;
    }
    const bool dbg = (P->flags & MAPPER_FLAG_DEBUG_STAGES) != 0;
    std::vector<int> nint(2, 1);
    for (int a = 0; a < na; ++a) nint[a] = P->axis[a].n_intervals;
    const int64_t E_count = (int64_t)nint[0] * (na == 2 ? nint[1] : 1);
    const double E = Elev[0];

    ev.mark();                                                      // 0
    // ---- lens and range
    double *f[2] = {nullptr, nullptr};
    unsigned long long *rk = mem.get<unsigned long long>(4);
    {
        const unsigned long long init[4] = {~0ull, 0ull, ~0ull, 0ull};
        h2d(rk, init, 4, s);
    }
    for (int a = 0; a < na; ++a) {
        const mapper_axis &ax = P->axis[a];
        f[a] = mem.get<double>(n);
        float *dir = nullptr;
        double *vals = nullptr;
        if (ax.kind == MAPPER_LENS_PROJECTION) {
            dir = mem.get<float>(d);
            h2d(dir, ax.direction, d, s);
        }
        if (ax.kind == MAPPER_LENS_VALUES) {
            vals = mem.get<double>(n);
            h2d(vals, ax.values, n, s);
        }
        if (ax.kind == MAPPER_LENS_KNN_DISTANCE || ax.kind == MAPPER_LENS_ECCENTRICITY) {
            mapper_run_stats ks{};                          // whole-cloud lens: k-NN screening + FP64
            const bool ecc = ax.kind == MAPPER_LENS_ECCENTRICITY;
            knn_device(ctx, cloud, ecc ? 1 : ax.column, ecc ? 1 : 0, P_FP16, f[a], ks, s);
            HIPCHK(launch_sqrt(f[a], n, s));
        } else {
            HIPCHK(launch_lens(cloud->X, n, d, ax.kind, ax.column, dir, vals, f[a], s));
        }
        HIPCHK(launch_range(f[a], n, rk + 2 * a, s));
    }
    std::vector<unsigned long long> rkh;
    d2h(rkh, rk, 4, s);
    HIPCHK(hipStreamSynchronize(s));
    ev.mark();                                                      // 1
    std::vector<double> lo[2], hi[2], hc[2];
    double* dlo[2] = {nullptr, nullptr};
    double* dhc[2] = {nullptr, nullptr};
    for (int a = 0; a < na; ++a) {
        const double m = key_to_double(rkh[2 * a]), M = key_to_double(rkh[2 * a + 1]);
        if (P->axis[a].cover == MAPPER_COVER_BALANCED)
            balanced_endpoints(ctx->arena, f[a], n, nint[a], P->axis[a].overlap, lo[a], hi[a], s);
        else
            cover_endpoints(m, M, nint[a], P->axis[a].overlap, lo[a], hi[a]);
        hc[a].resize(nint[a]);
        for (int k = 0; k < nint[a]; ++k) {
            if (!std::isfinite(lo[a][k]) || !std::isfinite(hi[a][k]))
                throw std::runtime_error("lens range too wide for finite interval endpoints");
            hc[a][k] = std::min(hi[a][k], M);
        }
        for (int k = 1; k < nint[a]; ++k)
            if (lo[a][k] < lo[a][k - 1] || hc[a][k] < hc[a][k - 1])
                throw std::runtime_error("interval endpoints not monotone");
        dlo[a] = mem.get<double>(nint[a]);
        dhc[a] = mem.get<double>(nint[a]);
        h2d(dlo[a], lo[a].data(), nint[a], s);
        h2d(dhc[a], hc[a].data(), nint[a], s);
    }

    // ---- pullback sets: (element, point) pairs sorted stably by element
    int32_t *range4 = mem.get<int32_t>(4 * n);
    int32_t *mcount = mem.get<int32_t>(n);
    int64_t *mpos = mem.get<int64_t>(n + 1);
    void *stmp = mem.get<char>(scan_temp_bytes(n));
    unsigned long long *psum = mem.get<unsigned long long>(1);
    HIPCHK(hipMemsetAsync(psum, 0, 8, s));
    HIPCHK(launch_member_count(f[0], na == 2 ? f[1] : nullptr, n, dlo[0], dhc[0], nint[0],
                               na == 2 ? dlo[1] : nullptr, na == 2 ? dhc[1] : nullptr, nint[1],
                               range4, mcount, psum, s));
    HIPCHK(launch_scan_i32(mcount, mpos, n, stmp, s));
    int64_t S = 0;
    unsigned long long pair_bound = 0;       // sum over points of C(elements holding it, 2)
    HIPCHK(hipMemcpyAsync(&S, mpos + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&pair_bound, psum, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (S > (int64_t)0x7fffffff) throw std::runtime_error("more than 2^31 memberships");
    const int64_t Sa = std::max<int64_t>(S, 1);
    uint64_t *skey = mem.get<uint64_t>(Sa), *skey2 = mem.get<uint64_t>(Sa);
    uint32_t *sval = mem.get<uint32_t>(Sa), *sval2 = mem.get<uint32_t>(Sa);
    void *sortmp = mem.get<char>(sort_temp_bytes(Sa));
    // slots sorted by (element, cell, outlier gap rank): each element's
    // members in the cloud's locality order, point order within a cell (the
    // sort is stable)
    const int cbits = cloud->okey ? cloud->cell_bits : 0;
    HIPCHK(launch_member_emit(range4, mpos, n, nint[1], na == 2, cloud->okey, cbits, skey, sval, s));
    bool alt = false;
    HIPCHK(radix_sort_pairs(skey, sval, skey2, sval2, S, bits_for((uint64_t)E_count) + cbits, sortmp, &alt, s));
    uint64_t *slot_elem = alt ? skey2 : skey;
    uint32_t *slot_point = alt ? sval2 : sval;
    HIPCHK(launch_shift_keys(slot_elem, S, cbits, s));
    int64_t *elem_off = mem.get<int64_t>(E_count + 1);
    HIPCHK(launch_lower_bounds(slot_elem, S, E_count, elem_off, s));
    std::vector<int64_t> eoff;
    d2h(eoff, elem_off, E_count + 1, s);
    HIPCHK(hipStreamSynchronize(s));
    ev.mark();                                                      // 2
    // the binning temporaries are done (the stream is synchronized)
    for (void *q : {(void *)range4, (void *)mcount, (void *)mpos, stmp, (void *)psum, sortmp,
                    (void *)(alt ? skey : skey2), (void *)(alt ? sval : sval2)})
        mem.release(q);

    // ---- tiling (host): elements largest first
    std::vector<int32_t> order;
    std::vector<int64_t> T(E_count), P_e(E_count), blk_off(E_count);
    int64_t nblocks = 0, pairs = 0;
    for (int64_t e = 0; e < E_count; ++e) {
        const int64_t ne = eoff[e + 1] - eoff[e];
        T[e] = (ne + TILE - 1) / TILE;
        P_e[e] = T[e] * (T[e] + 1) / 2;
        blk_off[e] = nblocks;
        nblocks += P_e[e];
        pairs += ne * (ne + 1) / 2;
        if (ne > 0) order.push_back((int32_t)e);
    }
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return P_e[a] > P_e[b]; });
    std::vector<int64_t> item_off(order.size() + 1, 0);
    for (size_t k = 0; k < order.size(); ++k) item_off[k + 1] = item_off[k] + P_e[order[k]];
    st.n_slots = S;
    st.pairs = pairs;
    st.tiles = nblocks;

    // ---- panel scale and tile order (both independent of the precision)
    const float scale_src = cloud->maxabs;
    double scale = 1.0;
    if (scale_src > 0) scale = std::ldexp(1.0, 10 - std::ilogb((double)scale_src));
    // screening of tile pairs by their rows' cells: when the cloud has a
    // locality order (cells) and the cell balls' margins hold (d <= BALL_DMAX)
    const bool screen = cloud->cell != nullptr && d <= BALL_DMAX && nblocks > 0 &&
                        !(P->flags & (MAPPER_FLAG_NO_SCREEN | MAPPER_FLAG_TILE_MACRO));
    const int super = supertile_size(d);
    std::vector<int64_t> colpre, cp_off(E_count);
    build_supertile_columns(T, super, colpre, cp_off);
    int64_t nrb = 0;                                            // row blocks of all elements
    std::vector<int64_t> rb_off(std::max<int64_t>(E_count, 1), 0);
    for (int64_t e = 0; e < E_count; ++e) { rb_off[e] = nrb; nrb += T[e]; }

    // ---- device tile tables: every tile pair I <= J of every element
    int64_t *d_item_off = mem.get<int64_t>(item_off.size());
    int32_t *d_order = mem.get<int32_t>(std::max<size_t>(order.size(), 1));
    int64_t *d_blk_off = mem.get<int64_t>(std::max<int64_t>(E_count, 1));
    h2d(d_item_off, item_off.data(), (int64_t)item_off.size(), s);
    h2d(d_order, order.data(), (int64_t)order.size(), s);
    h2d(d_blk_off, blk_off.data(), E_count, s);
    TileTable tt;
    tt.item_off = d_item_off;
    tt.order = d_order;
    tt.elem_off = elem_off;
    tt.blk_off = d_blk_off;
    int64_t *d_colpre = mem.get<int64_t>(colpre.size());
    int64_t *d_cp_off = mem.get<int64_t>(std::max<int64_t>(E_count, 1));
    h2d(d_colpre, colpre.data(), (int64_t)colpre.size(), s);
    h2d(d_cp_off, cp_off.data(), E_count, s);
    tt.colpre = d_colpre;
    tt.cp_off = d_cp_off;
    tt.nord = (int32_t)order.size();
    tt.super = super;
    tt.n_items = nblocks;
    TileItem *d_items = mem.get<TileItem>(std::max<int64_t>(nblocks, 1));
    HIPCHK(launch_build_items(tt, d_items, s));
    tt.items = d_items;
    int64_t *d_rb_off = mem.get<int64_t>(rb_off.size());
    h2d(d_rb_off, rb_off.data(), (int64_t)rb_off.size(), s);

    // ---- screening: the tile pairs that can hold a neighbour pair, each
    // with its own bitmask block (their position in launch order)
    int64_t n_tiles = nblocks;                                  // tile pairs computed
    int64_t *diag_blk = nullptr, *next_blk = nullptr;
    st.pairs_computed = pairs;
    if (screen) {
        uint8_t *keep = mem.get<uint8_t>(nblocks);
        int64_t *kpos = mem.get<int64_t>(nblocks + 1);
        void *kst = mem.get<char>(scan_temp_bytes(nblocks));
        double Emax = 0.0;
        for (int lv = 0; lv < n_levels; ++lv) Emax = std::max(Emax, Elev[lv]);
        // cells eps may join: all but the pairs whose balls' gap g satisfies
        // g^2 (1 - (d + 8) 2^-52) > E (1 + 2^-40): the canonical FP64
        // distance of two points is at least (1 - (d + 1) 2^-53) times
        // their exact squared distance, which the gap bounds from below
        const int nc = cloud->ncell;
        std::vector<unsigned long long> nearh((size_t)CELL_MAX, 0);
        const double shrink = 1.0 - ((double)d + 8.0) * 0x1.0p-52;
        const double Eb = Emax * (1.0 + 0x1.0p-40);
        for (int a = 0; a < nc; ++a)
            for (int b = 0; b < nc; ++b) {
                const double g = cloud->cell_gap[(size_t)a * nc + b];
                if (!(a != b && g > 0.0 && g * g * shrink > Eb)) nearh[(size_t)a] |= 1ull << b;
            }
        // outliers farther than eps from every landmark cell (id nc, next to
        // the outlier cell nc - 1): near the outliers only
        const int out_id = nc - 1, far_id = nc;
        nearh[(size_t)out_id] |= 1ull << far_id;
        nearh[(size_t)far_id] = (1ull << out_id) | (1ull << far_id);
        unsigned long long *near = mem.get<unsigned long long>(CELL_MAX);
        unsigned long long *cmask = mem.get<unsigned long long>(nrb), *nmask = mem.get<unsigned long long>(nrb);
        h2d(near, nearh.data(), CELL_MAX, s);
        HIPCHK(launch_tile_cells(slot_point, elem_off, d_rb_off, (int32_t)E_count, nrb, cloud->cell, cloud->ogap,
                                 out_id, shrink, Eb, near, cmask, nmask, s));
        HIPCHK(launch_screen(d_items, nblocks, d_rb_off, cmask, nmask, keep, s));
        HIPCHK(launch_scan_u8(keep, kpos, nblocks, kst, s));
        TileItem *kept = mem.get<TileItem>(std::max<int64_t>(nblocks, 1));   // room for all: one read below
        diag_blk = mem.get<int64_t>(std::max<int64_t>(nrb, 1));
        next_blk = mem.get<int64_t>(std::max<int64_t>(nrb, 1));
        unsigned long long *pc = mem.get<unsigned long long>(PAIR_SLOTS);
        HIPCHK(hipMemsetAsync(pc, 0, PAIR_SLOTS * 8, s));
        HIPCHK(hipMemsetAsync(next_blk, 0xff, (size_t)std::max<int64_t>(nrb, 1) * 8, s));   // -1: no pair (I, I + 1)
        HIPCHK(launch_compact_items(d_items, nblocks, keep, kpos, d_rb_off, kept, diag_blk, next_blk, pc, s));
        unsigned long long pairs_c[PAIR_SLOTS];
        HIPCHK(hipMemcpyAsync(&n_tiles, kpos + nblocks, 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(pairs_c, pc, PAIR_SLOTS * 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        st.pairs_computed = 0;
        for (int q = 0; q < PAIR_SLOTS; ++q) st.pairs_computed += (int64_t)pairs_c[q];
        tt.items = kept;
        tt.n_items = n_tiles;
    }
    st.tiles_screened_out = nblocks - n_tiles;
    st.tiles = n_tiles;

    // ---- precision: as asked, or (AUTO) the cached choice for this kind of
    // run, or measured now on a sample of this run's tile pairs
    int prec = P->precision;
    if (prec == MAPPER_PREC_AUTO) {
        const TuneKey key = tune_key(d, E, cloud_median_norm2(ctx, cloud, s), (double)pairs);
        prec = cached_precision(ctx, key);
        if (prec < 0) prec = tune_precision(ctx, cloud, tt, n_tiles, slot_point, S, scale, E, key, st, s);
    }
    st.precision = prec;
    // launch form: macro tiles for single 16-bit products with one eps value
    // (screened runs keep scattered tile pairs: tile pairs then)
    const bool macro_ok = (prec == P_BF16 || prec == P_FP16) && n_levels == 1 && !screen &&
                          (uint64_t)panel_row_stride(prec, panel_dp(prec, d)) * MTILE < (1ull << 32);
    const bool use_macro = macro_ok && !(P->flags & MAPPER_FLAG_TILE_PAIRS);
    st.tile_m = st.tile_n = use_macro ? MTILE : TILE;
    st.split_terms = prec_is_split(prec) ? 3 : 1;

    // ---- host tables of the macro form
    const uint64_t level_words = (uint64_t)std::max<int64_t>(n_tiles, 1) * TILE_WORDS;
    int64_t n_mitems = 0;
    const int msuper = 4;          // 4 x 4 macro pairs: 1024 rows a side, as the tile pairs' 8 x 8
    std::vector<int64_t> T2, mitem_off, mcolpre, mcp_off, mblk_off;
    if (use_macro) {
        T2.resize(E_count);
        mblk_off.assign(E_count, 0);
        mcp_off.resize(E_count);
        for (int64_t e = 0; e < E_count; ++e) T2[e] = (eoff[e + 1] - eoff[e] + MTILE - 1) / MTILE;
        mitem_off.assign(order.size() + 1, 0);
        for (size_t k = 0; k < order.size(); ++k) {
            const int64_t t2 = T2[order[k]];
            mitem_off[k + 1] = mitem_off[k] + t2 * (t2 + 1) / 2;
        }
        n_mitems = mitem_off.back();
        build_supertile_columns(T2, msuper, mcolpre, mcp_off);
    }
    const int dp = panel_dp(prec, d);
    const uint64_t stride = (uint64_t)panel_row_stride(prec, dp);
    // band list: nseg segments (the tile pair form: 32 consecutive tile
    // pairs to a segment; the macro form: workgroup index mod nseg); grown
    // and collected again (macro: tiled again) if a segment overflows
    const int nseg = 8 * ((2 * ctx->cus + 7) / 8);          // two per CU, a multiple of the 8 XCDs
    int64_t band_cap = std::min<int64_t>(std::max<int64_t>(1 << 20, pairs / 256), 1ll << 28) / nseg;
    band_cap = std::max<int64_t>(band_cap, 1024);

    // ---- reservation: every later device array of the run, in one block
    // taken before the tile pass (a serving request that cannot have it
    // waits here, having run no tile pass).  Sizes are the allocations below
    // as the arena rounds them; a level's graph arrays at their upper bounds
    // (labelled slots <= S, nodes <= S, node pairs sharing a point <=
    // pair_bound), once: levels run one after another and free their arrays.
    auto r256 = [](uint64_t b) { return (b + 16 + 255) & ~(uint64_t)255; };
    const uint64_t E1 = (uint64_t)std::max<int64_t>(E_count, 1), U = (uint64_t)Sa;
    uint64_t fixed = 0;
    if (use_macro)
        fixed += r256(mitem_off.size() * 8) + r256(mcolpre.size() * 8) + 2 * r256(E1 * 8) +
                 r256((uint64_t)std::max<int64_t>(n_mitems, 1) * sizeof(MacroItem));
    fixed += r256(U * stride) + 2 * r256((uint64_t)n_levels * U * 4) + r256((uint64_t)n_levels * U * 4) +
             r256((uint64_t)n_levels * level_words * 4) + r256((uint64_t)nseg * 8);
    if (!use_macro) fixed += r256((uint64_t)n_levels * level_words * 4);     // band masks
    const uint64_t EPb = std::max<uint64_t>(pair_bound, 1);
    const uint64_t level = r256(U * 4) + r256(U) + r256((U + 1) * 8) + 2 * r256(U * 4) +
                           r256(scan_temp_bytes((int64_t)U + 1)) + r256((uint64_t)std::max<int64_t>(nrb, 1)) +
                           2 * r256(U * 8) + 2 * r256(U * 4) + r256(sort_temp_bytes((int64_t)U)) +
                           r256((U + 1) * 8) + r256(U * 4) + 2 * r256(U * 8) + 2 * r256(U * 4) + r256(U * 4) +
                           r256((U + 1) * 8) + r256(scan_temp_bytes((int64_t)U + 1)) + 2 * r256(EPb * 8) +
                           2 * r256(EPb * 4) + r256(sort_temp_bytes((int64_t)EPb)) + r256(EPb) +
                           r256((EPb + 1) * 8) + r256(scan_temp_bytes((int64_t)EPb + 1)) + r256(2 * EPb * 4) +
                           r256(EPb * 4) +
                           // canonical node order: minpt, root keys and values (two each), sort space, node_of_rank
                           r256(U * 4) + 2 * r256(U * 8) + 2 * r256(U * 4) + r256(sort_temp_bytes((int64_t)U)) +
                           r256(U * 4);
    uint64_t need = 0;
    void *res = nullptr;
    for (;;) {
        need = fixed + level + r256((uint64_t)nseg * band_cap * sizeof(BandPair));
        res = ctx->arena.alloc(need);
        if (res || band_cap <= 8) break;
        band_cap = std::max<int64_t>(band_cap / 4, 8);     // small arenas: a small list, grown on demand
    }
    if (!res) {
        // a serving request waits while others hold memory; a request that
        // runs alone (or a direct call) goes on without a reservation and
        // takes what the arena has as it goes (the sizes above are upper
        // bounds, so the run may still fit)
        bool others = false;
        if (may_retry) {
            std::lock_guard<std::mutex> lk(ctx->mu);
            others = ctx->active > 1;
            if (!others) ctx->hol = out.req;                    // unreserved: start nothing else meanwhile
        }
        if (others) throw AdmitWait{need};
    }
    mem.adopt(res, ctx->arena);
    Arena sub;                                                      // the reservation, sub-allocated
    sub.init((char *)res, res ? need : 0);
    Scope rm(sub, s, &ctx->arena);
    st.reserved_bytes = res ? need : 0;
    if (may_retry && res) admitted(ctx, out.req);

    MacroItem *d_mitems = nullptr;
    if (use_macro) {
        int64_t *d_mitem_off = rm.get<int64_t>(mitem_off.size());
        int64_t *d_mcolpre = rm.get<int64_t>(mcolpre.size());
        int64_t *d_mcp_off = rm.get<int64_t>(std::max<int64_t>(E_count, 1));
        int64_t *d_mblk_off = rm.get<int64_t>(std::max<int64_t>(E_count, 1));
        h2d(d_mitem_off, mitem_off.data(), (int64_t)mitem_off.size(), s);
        h2d(d_mcolpre, mcolpre.data(), (int64_t)mcolpre.size(), s);
        h2d(d_mcp_off, mcp_off.data(), E_count, s);
        h2d(d_mblk_off, mblk_off.data(), E_count, s);
        TileTable mt = tt;
        mt.item_off = d_mitem_off;
        mt.colpre = d_mcolpre;
        mt.cp_off = d_mcp_off;
        mt.blk_off = d_mblk_off;
        mt.super = msuper;
        mt.n_items = n_mitems;
        mt.items = nullptr;
        d_mitems = rm.get<MacroItem>(std::max<int64_t>(n_mitems, 1));
        HIPCHK(launch_build_macro_items(mt, tt, d_mitems, n_mitems, s));
    }

    void *panel = rm.get<char>((uint64_t)Sa * stride);
    float *thrA = rm.get<float>((uint64_t)n_levels * Sa), *thrB = rm.get<float>((uint64_t)n_levels * Sa);
    PackArgs pk;
    pk.X = cloud->X;
    pk.d = d;
    pk.dp = dp;
    pk.slot_point = slot_point;
    pk.n_slots = S;
    pk.prec = prec;
    pk.scale = scale;
    pk.n_levels = n_levels;
    for (int lv = 0; lv < n_levels; ++lv) pk.E_scaled[lv] = Elev[lv] * scale * scale;
    pk.panel = panel;
    pk.thrA = thrA;
    pk.thrB = thrB;
    pk.dbg_norm2 = nullptr;
    pk.dbg_e = nullptr;
    HIPCHK(launch_pack(pk, s));

    int32_t *count_all = rm.get<int32_t>((uint64_t)n_levels * Sa);
    uint32_t *bitmask_all = rm.get<uint32_t>((uint64_t)n_levels * level_words);
    st.bitmask_bytes = n_tiles * TILE_WORDS * 4;
    unsigned long long *band_n = rm.get<unsigned long long>(nseg);
    uint32_t *bandmask_all = use_macro ? nullptr : rm.get<uint32_t>((uint64_t)n_levels * level_words);
    BandPair *band = rm.get<BandPair>((uint64_t)nseg * band_cap);
    ev.mark();                                                      // 3
    std::vector<unsigned long long> segn(nseg);
    double ms_collect = 0.0;
    // the tile pass, then (tile pair form) the band records from its band
    // masks; when a band-list segment overflows the list grows and the
    // records are collected again (the macro form redoes its tiles)
    for (int launch = 0;; ++launch) {
        HIPCHK(hipMemsetAsync(band_n, 0, (size_t)nseg * 8, s));
        if (!use_macro && launch > 0) {
            Events ct(s, ctx->events);
            ct.mark();
            HIPCHK(launch_band_collect(tt, bandmask_all, n_levels, level_words, band, band_n, band_cap, nseg, s));
            ct.mark();
            HIPCHK(hipMemcpyAsync(segn.data(), band_n, (size_t)nseg * 8, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            st.tile_launches = launch + 1;
            ms_collect = ct.ms(0, 1);
            const int64_t most = (int64_t)*std::max_element(segn.begin(), segn.end());
            if (most <= band_cap) break;
            band_cap = most + most / 8 + 256;
            rm.release(band);                               // the stream is synchronized
            band = rm.get<BandPair>((uint64_t)nseg * band_cap);
            continue;
        }
        HIPCHK(hipMemsetAsync(count_all, 0, (size_t)n_levels * Sa * 4, s));
        TileArgs ta{};
        ta.tt = tt;
        ta.panel = panel;
        ta.dp = dp;
        ta.thrA = thrA;
        ta.thrB = thrB;
        ta.bitmask = bitmask_all;
        ta.count = count_all;
        ta.band = band;
        ta.band_n = band_n;
        ta.band_cap = band_cap;
        ta.nseg = nseg;
        ta.n_levels = n_levels;
        ta.level_slots = Sa;
        ta.level_words = level_words;
        ta.mitems = d_mitems;
        ta.n_mitems = n_mitems;
        ta.bandmask = bandmask_all;
        Events kt(s, ctx->events);
        kt.mark();
        if (use_macro) HIPCHK(launch_tiles_macro(prec, ta, s));
        else HIPCHK(launch_tiles(prec, ta, s));
        kt.mark();
        if (!use_macro)
            HIPCHK(launch_band_collect(tt, bandmask_all, n_levels, level_words, band, band_n, band_cap, nseg, s));
        kt.mark();
        HIPCHK(hipMemcpyAsync(segn.data(), band_n, (size_t)nseg * 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        st.tile_launches = launch + 1;
        st.ms_tiles = kt.ms(0, 1);
        ms_collect = kt.ms(1, 2);
        const int64_t most = (int64_t)*std::max_element(segn.begin(), segn.end());
        if (most <= band_cap) break;
        band_cap = most + most / 8 + 256;                   // grow, and collect (macro: tile) again
        rm.release(band);                                   // the stream is synchronized
        band = rm.get<BandPair>((uint64_t)nseg * band_cap);
    }
    out.tiles_done = true;
    int64_t nband = 0;
    for (int g = 0; g < nseg; ++g) nband += (int64_t)segn[g];
    st.band_pairs = nband;
    ev.mark();                                                      // 4
    {
        Levels lvs{};
        for (int lv = 0; lv < n_levels; ++lv) lvs.E[lv] = Elev[lv];
        lvs.level_slots = Sa;
        lvs.level_words = level_words;
        HIPCHK(launch_recheck(band, band_n, nseg, band_cap, nband, cloud->X, d, slot_point, lvs, bitmask_all,
                              count_all, s));
    }
    ev.mark();                                                      // 5

    // ---- one graph per level and minPts value (counts and bitmask do not
    // depend on minPts: only the clusters, border points and edges are redone)
    for (int lv = 0; lv < n_levels; ++lv)
    for (int mu = 0; mu < n_minpts; ++mu) {
    const int32_t min_pts = minpts_list ? minpts_list[mu] : P->min_pts;
    Scope lm(sub, s, &ctx->arena);                                  // this graph's work arrays
    Events lev(s, ctx->events);
    lev.mark();                                                     // 0
    int32_t *count = count_all + (int64_t)lv * Sa;
    uint32_t *bitmask = bitmask_all + (uint64_t)lv * level_words;
    auto g = std::make_unique<mapper_graph>();
    g->stats = st;

    // ---- clusters
    int32_t *parent = lm.get<int32_t>(Sa);
    uint8_t *isroot = lm.get<uint8_t>(Sa);
    int64_t *rank = lm.get<int64_t>(Sa + 1);
    int32_t *node = lm.get<int32_t>(Sa);
    int32_t *node_elem = lm.get<int32_t>(Sa);
    HIPCHK(launch_cc_init(parent, S, s));
    HIPCHK(launch_cc_hook(tt, d_rb_off, nrb, (int32_t)E_count, diag_blk, next_blk, bitmask, count, min_pts,
                          parent, s));
    HIPCHK(launch_cc_compress(parent, S, s));
    HIPCHK(launch_cc_tiles(tt, bitmask, count, min_pts, parent, s));
    HIPCHK(launch_cc_flatten(count, min_pts, parent, isroot, S, s));
    void *stmp2 = lm.get<char>(scan_temp_bytes(Sa + 1));
    HIPCHK(launch_scan_u8(isroot, rank, S, stmp2, s));
    // canonical node order: the roots sorted by (element, smallest core point id)
    int64_t N = 0;
    HIPCHK(hipMemcpyAsync(&N, rank + S, 8, hipMemcpyDeviceToHost, s));
    int32_t *minpt = lm.get<int32_t>(Sa);
    uint64_t *rk1 = lm.get<uint64_t>(Sa), *rk2 = lm.get<uint64_t>(Sa);
    uint32_t *rv1 = lm.get<uint32_t>(Sa), *rv2 = lm.get<uint32_t>(Sa);
    void *rsort = lm.get<char>(sort_temp_bytes(Sa));
    int32_t *node_of_rank = lm.get<int32_t>(Sa);
    HIPCHK(launch_root_keys(count, min_pts, parent, slot_point, isroot, rank, slot_elem, minpt, rk1, rv1, S, s));
    HIPCHK(hipStreamSynchronize(s));                                // N
    bool ralt = false;
    HIPCHK(radix_sort_pairs(rk1, rv1, rk2, rv2, N, 32 + bits_for((uint64_t)E_count), rsort, &ralt, s));
    HIPCHK(launch_node_ids(count, min_pts, parent, rank, ralt ? rk2 : rk1, ralt ? rv2 : rv1, N, node_of_rank,
                           node, node_elem, S, s));
    {
        uint8_t *ncflag = lm.get<uint8_t>(std::max<int64_t>(nrb, 1));
        HIPCHK(hipMemsetAsync(ncflag, 0, (size_t)std::max<int64_t>(nrb, 1), s));
        HIPCHK(launch_noncore_flags(count, min_pts, slot_elem, elem_off, d_rb_off, ncflag, S, s));
        HIPCHK(launch_border(tt, bitmask, count, min_pts, ncflag, d_rb_off, node, s));
    }
    lev.mark();                                                     // 1

    // ---- node CSR: (node, point) sorted stably by node
    uint8_t *lab = isroot;       // reuse
    HIPCHK(launch_flag_labelled(node, lab, S, s));
    int64_t *mp = rank;          // reuse (roots already consumed by launch_node_ids)
    HIPCHK(launch_scan_u8(lab, mp, S, stmp2, s));
    int64_t M = 0;
    HIPCHK(hipMemcpyAsync(&M, mp + S, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const int64_t Ma = std::max<int64_t>(M, 1);
    uint64_t *k1 = lm.get<uint64_t>(Ma), *k2 = lm.get<uint64_t>(Ma);
    uint32_t *v1 = lm.get<uint32_t>(Ma), *v2 = lm.get<uint32_t>(Ma);
    void *sortmp2 = lm.get<char>(sort_temp_bytes(Ma));
    // sorted by (node, point): members ascending in each node (slots are in
    // cell order, not point order); then keys back to node ids
    const int pbits = bits_for((uint64_t)std::max<int64_t>(n - 1, 0));
    HIPCHK(launch_member_pairs(node, slot_point, mp, S, pbits, k1, v1, s));
    HIPCHK(radix_sort_pairs(k1, v1, k2, v2, M, bits_for((uint64_t)std::max<int64_t>(N - 1, 0)) + pbits, sortmp2,
                            &alt, s));
    uint64_t *nk = alt ? k2 : k1;
    uint32_t *nv = alt ? v2 : v1;
    HIPCHK(launch_shift_keys(nk, M, pbits, s));
    int64_t *node_off = lm.get<int64_t>(N + 1);
    HIPCHK(launch_node_offsets_from_sorted(nk, M, N, node_off, s));
    int32_t *members = lm.get<int32_t>(Ma);
    HIPCHK(launch_u32_to_i32(nv, members, M, s));
    // ---- edges: regroup (point, node) by point; stable, so nodes stay ascending
    uint64_t *ptk = lm.get<uint64_t>(Ma), *ptk2 = lm.get<uint64_t>(Ma);
    uint32_t *ptn = lm.get<uint32_t>(Ma), *ptn2 = lm.get<uint32_t>(Ma);
    HIPCHK(launch_widen_u32(nv, ptk, M, s));
    HIPCHK(launch_narrow_u64(nk, ptn, M, s));
    HIPCHK(radix_sort_pairs(ptk, ptn, ptk2, ptn2, M, bits_for((uint64_t)std::max<int64_t>(n - 1, 0)), sortmp2, &alt, s));
    uint64_t *sp_k = alt ? ptk2 : ptk;
    uint32_t *sp_n = alt ? ptn2 : ptn;
    int32_t *ecnt = lm.get<int32_t>(Ma);
    int64_t *epos = lm.get<int64_t>(Ma + 1);
    void *stmp3 = lm.get<char>(scan_temp_bytes(Ma + 1));
    HIPCHK(launch_edge_counts(sp_k, M, ecnt, s));
    HIPCHK(launch_scan_i32(ecnt, epos, M, stmp3, s));
    int64_t EP = 0;
    HIPCHK(hipMemcpyAsync(&EP, epos + M, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const int64_t EPa = std::max<int64_t>(EP, 1);
    uint64_t *ek = lm.get<uint64_t>(EPa), *ek2 = lm.get<uint64_t>(EPa);
    uint32_t *ev1 = lm.get<uint32_t>(EPa), *ev2 = lm.get<uint32_t>(EPa);
    void *sortmp3 = lm.get<char>(sort_temp_bytes(EPa));
    HIPCHK(launch_edge_emit(sp_k, sp_n, M, epos, N, ek, s));
    HIPCHK(hipMemsetAsync(ev1, 0, (size_t)EPa * 4, s));
    HIPCHK(radix_sort_pairs(ek, ev1, ek2, ev2, EP, bits_for((uint64_t)N * (uint64_t)N), sortmp3, &alt, s));
    uint64_t *sek = alt ? ek2 : ek;
    uint8_t *rs = lm.get<uint8_t>(EPa);
    int64_t *rr = lm.get<int64_t>(EPa + 1);
    void *stmp4 = lm.get<char>(scan_temp_bytes(EPa + 1));
    HIPCHK(launch_run_starts(sek, EP, rs, s));
    HIPCHK(launch_scan_u8(rs, rr, EP, stmp4, s));
    int64_t NE = 0;
    HIPCHK(hipMemcpyAsync(&NE, rr + EP, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    int32_t *edges = lm.get<int32_t>(2 * std::max<int64_t>(NE, 1));
    int32_t *weights = lm.get<int32_t>(std::max<int64_t>(NE, 1));
    HIPCHK(launch_edge_compact(sek, EP, rr, N, edges, weights, s));
    lev.mark();                                                     // 2

    // ---- graph to the host
    d2h(g->node_element, node_elem, N, s);
    d2h(g->node_offsets, node_off, N + 1, s);
    d2h(g->node_members, members, M, s);
    d2h(g->edges, edges, 2 * NE, s);
    d2h(g->weights, weights, NE, s);
    if (dbg) {
        auto put = [&](const char *name, const void *src, int64_t cnt, size_t esz) {
            auto &slot = g->stages[name];
            slot.first.resize((size_t)std::max<int64_t>(cnt, 0) * esz + 1);
            slot.second = cnt;
            if (cnt > 0) HIPCHK(hipMemcpyAsync(slot.first.data(), src, (size_t)cnt * esz, hipMemcpyDeviceToHost, s));
        };
        std::vector<double> lensv;
        for (int a = 0; a < na; ++a) {
            std::vector<double> tmp;
            d2h(tmp, f[a], n, s);
            HIPCHK(hipStreamSynchronize(s));
            lensv.insert(lensv.end(), tmp.begin(), tmp.end());
        }
        auto &ls = g->stages["lens"];
        ls.first.assign((char *)lensv.data(), (char *)lensv.data() + lensv.size() * 8);
        ls.second = (int64_t)lensv.size();
        std::vector<double> lov, hiv;
        for (int a = 0; a < na; ++a) {
            lov.insert(lov.end(), lo[a].begin(), lo[a].end());
            hiv.insert(hiv.end(), hi[a].begin(), hi[a].end());
        }
        g->stages["lo"] = {std::vector<char>((char *)lov.data(), (char *)lov.data() + lov.size() * 8), (int64_t)lov.size()};
        g->stages["hi"] = {std::vector<char>((char *)hiv.data(), (char *)hiv.data() + hiv.size() * 8), (int64_t)hiv.size()};
        g->stages["elem_offsets"] = {std::vector<char>((char *)eoff.data(), (char *)eoff.data() + eoff.size() * 8), (int64_t)eoff.size()};
        put("elem_members", slot_point, S, 4);
        put("slot_count", count, S, 4);
        put("slot_node_raw", node, S, 4);
    }
    HIPCHK(hipStreamSynchronize(s));
    if (dbg && cbits > 0) {
        // slots are in cell order inside each element: report the per-slot
        // stage arrays in point order, as the stage contract states
        int32_t *mem_p = (int32_t *)g->stages["elem_members"].first.data();
        int32_t *cnt_p = (int32_t *)g->stages["slot_count"].first.data();
        int32_t *nod_p = (int32_t *)g->stages["slot_node_raw"].first.data();
        std::vector<int64_t> idx;
        std::vector<int32_t> tm, tc, tn;
        for (int64_t e = 0; e < E_count; ++e) {
            const int64_t a = eoff[e], b = eoff[e + 1];
            idx.resize((size_t)(b - a));
            for (int64_t k = 0; k < b - a; ++k) idx[(size_t)k] = a + k;
            std::sort(idx.begin(), idx.end(), [&](int64_t x, int64_t y) { return mem_p[x] < mem_p[y]; });
            tm.resize(idx.size());
            tc.resize(idx.size());
            tn.resize(idx.size());
            for (size_t k = 0; k < idx.size(); ++k) {
                tm[k] = mem_p[idx[k]];
                tc[k] = cnt_p[idx[k]];
                tn[k] = nod_p[idx[k]];
            }
            std::copy(tm.begin(), tm.end(), mem_p + a);
            std::copy(tc.begin(), tc.end(), cnt_p + a);
            std::copy(tn.begin(), tn.end(), nod_p + a);
        }
    }
    if (dbg) {
        auto &raw = g->stages["slot_node_raw"];
        std::vector<int32_t> nodev((size_t)S);
        if (S) std::memcpy(nodev.data(), raw.first.data(), (size_t)S * 4);
        std::vector<uint8_t> corev((size_t)S);
        const int32_t *cnt = (const int32_t *)g->stages["slot_count"].first.data();
        for (int64_t i = 0; i < S; ++i) {
            if (nodev[i] == 0x7fffffff) nodev[i] = -1;
            corev[i] = cnt[i] >= min_pts;
        }
        g->stages["slot_node"] = {std::vector<char>((char *)nodev.data(), (char *)nodev.data() + S * 4 + 1), S};
        g->stages["slot_core"] = {std::vector<char>((char *)corev.data(), (char *)corev.data() + S + 1), S};
        g->stages.erase("slot_node_raw");
    }
    g->stats.ms_lens = ev.ms(0, 1);                                 // the stream has passed every event
    g->stats.ms_bin = ev.ms(1, 2);
    g->stats.ms_recheck = ev.ms(4, 5) + ms_collect;                // band records and their FP64 re-decision
    g->stats.ms_cc = lev.ms(0, 1);
    g->stats.ms_edges = lev.ms(1, 2);
    g->stats.ms_total = ev.ms(0, 5) + lev.ms(0, 2);
    g->stats.arena_peak_bytes = mem.bytes() + rm.bytes() + lm.bytes();
    g->stats.reserve_overflow_bytes = rm.overflow() + lm.overflow();
    out.gs.push_back(g.release());
    }
    (void)may_retry;
    return Phase::Ok;
}

// Outcome of a serving attempt that could not finish for lack of arena.
struct Retry {
    bool again = false;        // requeue the request
    bool admission = false;    // it waited for its reservation (no tile pass run)
    bool redone = false;       // its tile pass was lost (a shortage after the reservation)
};

// out[0 .. n_levels) receive the graphs (n_levels eps values from eps_list,
// or P->eps when it is null).  req: the serving request (null otherwise).
mapper_status run_guarded(mapper_context *ctx, const mapper_cloud *cloud, const mapper_params *P,
                          hipStream_t s, bool may_retry, mapper_graph **out, Retry *retry,
                          const double *eps_list = nullptr, int n_levels = 1, const void *req = nullptr,
                          const int32_t *minpts_list = nullptr, int n_minpts = 1) {
    *retry = Retry{};
    RunOut ro;
    ro.req = req;
    // a serving request waits and retries only while another request holds
    // memory that it will return (checked when the shortage happens), and
    // fails only when it ran alone
    auto others_active = [&]() {
        if (!may_retry) return false;
        std::lock_guard<std::mutex> lk(ctx->mu);
        return ctx->active > 1;
    };
    try {
        HIPCHK(hipSetDevice(ctx->device));
        run_pipeline(ctx, cloud, P, s, may_retry, ro, eps_list, n_levels, minpts_list, n_minpts);
        for (int q = 0; q < n_levels * n_minpts; ++q) out[q] = ro.gs[(size_t)q];
        ro.gs.clear();
        return MAPPER_OK;
    } catch (AdmitWait &) {
        // thrown only while another request held memory: wait and try again
        // (a request that finds itself alone runs without a reservation)
        (void)hipStreamSynchronize(s);
        *retry = Retry{true, true, false};
        return MAPPER_ENOMEM;
    } catch (NoMem &nm) {
        (void)hipStreamSynchronize(s);
        if (others_active()) {
            // before its tile pass this is a wait for memory like a reservation
            *retry = Retry{true, !ro.tiles_done, ro.tiles_done};
            return MAPPER_ENOMEM;
        }
        return fail(MAPPER_ENOMEM, "arena too small for this run (needed " + std::to_string(nm.want) +
                                       " more bytes in one block)");
    } catch (DevError &de) {
        (void)hipStreamSynchronize(s);
        return fail(MAPPER_EDEVICE, std::string("HIP error: ") + hipGetErrorString(de.e) + " (runtime.cpp:" +
                                        std::to_string(de.line) + ")");
    } catch (std::exception &ex) {
        (void)hipStreamSynchronize(s);
        return fail(MAPPER_EINVAL, ex.what());
    }
}

void worker_main(mapper_context *ctx, hipStream_t s) {
    (void)hipSetDevice(ctx->device);
    while (true) {
        Request *r = nullptr;
        {
            std::unique_lock<std::mutex> lk(ctx->mu);
            // while a head-of-line request waits for its reservation, only it
            // may be taken
            ctx->cv.wait(lk, [&] {
                return (ctx->stop && ctx->pending.empty()) ||
                       (!ctx->pending.empty() && (!ctx->hol || ctx->pending.front() == ctx->hol));
            });
            if (ctx->stop && ctx->pending.empty()) return;
            r = ctx->pending.front();
            ctx->pending.pop_front();
            ++ctx->active;
        }
        mapper_graph *g = nullptr;
        Retry retry;
        const mapper_status st = run_guarded(ctx, r->cloud, &r->params.p, s, true, &g, &retry, nullptr, 1, r);
        std::unique_lock<std::mutex> lk(ctx->mu);
        --ctx->active;
        if (retry.again) {
            r->waits += retry.admission ? 1 : 0;
            r->redone += retry.redone ? 1 : 0;
            // the failed run has released its own memory by now: hold the
            // queue for it and wait for another request's release (or 50 ms)
            // before trying again
            ctx->hol = r;
            const uint64_t seen = ctx->arena.epoch();
            ctx->pending.push_front(r);
            lk.unlock();
            ctx->arena.wait_release(seen, 50);
            ctx->cv.notify_all();
            continue;
        }
        if (ctx->hol == r) ctx->hol = nullptr;              // done (or failed for good): release the queue
        if (g) {
            g->stats.admission_waits = r->waits;
            g->stats.tile_passes_redone = r->redone;
        }
        r->status = st;
        r->err = st == MAPPER_OK ? "" : g_last_error;
        r->graph = g;
        r->done = true;
        const_cast<mapper_cloud *>(r->cloud)->inflight--;
        ctx->cv.notify_all();
    }
}

}  // namespace

// ================================================================= C ABI

// ------------------------------------------------- the no-alloc k-NN scratch
// mapper_knn_d2_noalloc keeps all of its device work arrays in this array,
// one copy per GPU (it is part of the library's code object, so every device
// the library runs on holds it until the process ends).  In host code the
// name is only a stand-in: the device address of each GPU's copy comes from
// hipGetSymbolAddress with that GPU current, taken once per device when a
// context is created there, and only that address is handed to kernels and
// copies.
constexpr uint64_t NOALLOC_SCRATCH_BYTES = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;                      // guards g_scratch and serializes no-alloc calls per device
void *g_scratch[MAX_DEVICES] = {};
std::mutex g_noalloc_mu[MAX_DEVICES];

// Resolve (once) this device's copy of the scratch array.
hipError_t resolve_scratch(int device) {
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[device]) return hipSuccess;
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    e = hipSetDevice(device);
    if (e != hipSuccess) return e;
    void *ptr = nullptr;
    e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
    (void)hipSetDevice(cur);
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch[device] = ptr;
    return hipSuccess;
}

void *scratch_of(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return (device >= 0 && device < MAX_DEVICES) ? g_scratch[device] : nullptr;
}

// Carves 256-byte aligned pieces off the scratch array; no allocation.
struct ScratchCarve {
    char *base;
    uint64_t used, cap;
    template <class T> T *take(uint64_t count) {
        const uint64_t b = (count * sizeof(T) + 255) & ~(uint64_t)255;
        if (used + b > cap) return nullptr;
        T *p = (T *)(base + used);
        used += b;
        return p;
    }
};

// Scratch bytes of a k-NN call with C column chunks and candidate lists of
// cmax entries (the same arrays as knn_device).
uint64_t knn_scratch_bytes(int64_t n, int32_t d, int prec, int32_t T, int32_t C, int32_t cmax) {
    auto al = [](uint64_t b) { return (b + 255) & ~(uint64_t)255; };
    const uint64_t stride = (uint64_t)panel_row_stride(prec, panel_dp(prec, d));
    return al(256) + al((uint64_t)n * 4) + al((uint64_t)n * stride) + 2 * al((uint64_t)n * 4) +
           al((uint64_t)C * T * TILE * 4 * KNN_KMAX * 4) + al((uint64_t)n * 4) + al((uint64_t)n * 4) +
           al((uint64_t)n * cmax * 4);
}
}  // namespace

extern "C" {

const char *mapper_last_error(void) { return g_last_error.c_str(); }

mapper_status mapper_context_create(int device, void *arena, uint64_t arena_bytes, void *stream,
                                    mapper_context **out) {
    if (!out) return fail(MAPPER_EINVAL, "out is null");
    *out = nullptr;
    if (!arena || arena_bytes < (1u << 20)) return fail(MAPPER_EINVAL, "arena must be at least 1 MiB");
    if (((uintptr_t)arena & 255) != 0) return fail(MAPPER_EINVAL, "arena must be 256-byte aligned");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return fail(MAPPER_EDEVICE, "no such HIP device");
    if (device >= MAX_DEVICES) return fail(MAPPER_EDEVICE, "device ordinal beyond the library's table");
    if (hipError_t e = resolve_scratch(device); e != hipSuccess)
        return fail(MAPPER_EDEVICE, std::string("scratch array: ") + hipGetErrorString(e));
    auto *c = new mapper_context();
    c->device = device;
    if (hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || c->cus < 1)
        c->cus = 256;
    c->arena.init((char *)arena, arena_bytes);
    c->stream = (hipStream_t)stream;
    *out = c;
    return MAPPER_OK;
}

mapper_status mapper_context_set_streams(mapper_context *ctx, void *const *streams, int count) {
    if (!ctx || count < 0 || (count > 0 && !streams)) return fail(MAPPER_EINVAL, "bad streams");
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (!ctx->workers.empty()) return fail(MAPPER_EBUSY, "streams already in use by the request loop");
    ctx->slots.clear();
    for (int i = 0; i < count; ++i) ctx->slots.push_back((hipStream_t)streams[i]);
    return MAPPER_OK;
}

void mapper_context_destroy(mapper_context *ctx) {
    if (!ctx) return;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->stop = true;
    }
    ctx->cv.notify_all();
    for (auto &t : ctx->workers) t.join();
    for (auto &kv : ctx->tickets) {
        if (kv.second->graph) mapper_graph_destroy(kv.second->graph);
        delete kv.second;
    }
    delete ctx;
}

mapper_status mapper_context_memory(const mapper_context *ctx, uint64_t *in_use, uint64_t *peak) {
    if (!ctx) return fail(MAPPER_EINVAL, "null context");
    if (in_use) *in_use = ctx->arena.in_use();
    if (peak) *peak = ctx->arena.peak();
    return MAPPER_OK;
}

mapper_status mapper_cloud_create(mapper_context *ctx, const float *points, int64_t n, int32_t d,
                                  int32_t on_device, mapper_cloud **out) {
    if (!ctx || !points || !out) return fail(MAPPER_EINVAL, "null argument");
    *out = nullptr;
    if (n < 1 || n > 0x7fffffff || d < 1 || d > (1 << 16)) return fail(MAPPER_EINVAL, "need 1 <= n < 2^31, 1 <= d <= 65536");
    const uint64_t bytes = (uint64_t)n * (uint64_t)d * 4;
    float *X = (float *)ctx->arena.alloc(bytes);
    uint32_t *flags = (uint32_t *)ctx->arena.alloc(256);
    if (!X || !flags) {
        ctx->arena.release(X);
        ctx->arena.release(flags);
        return fail(MAPPER_ENOMEM, "arena cannot hold the cloud");
    }
    try {
        HIPCHK(hipSetDevice(ctx->device));
        hipStream_t s = ctx->stream;
        HIPCHK(hipMemcpyAsync(X, points, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
        HIPCHK(hipMemsetAsync(flags, 0, 8, s));
        HIPCHK(launch_check_cloud(X, (int64_t)n * d, flags, s));
        uint32_t h[2] = {0, 0};
        HIPCHK(hipMemcpyAsync(h, flags, 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        ctx->arena.release(flags);
        if (h[0]) {
            ctx->arena.release(X);
            return fail(MAPPER_EINVAL, "cloud has non-finite coordinates");
        }
        auto *c = new mapper_cloud();
        c->ctx = ctx;
        c->X = X;
        c->n = n;
        c->d = d;
        std::memcpy(&c->maxabs, &h[1], 4);
        build_cells(ctx, c, s);
        *out = c;
        return MAPPER_OK;
    } catch (DevError &de) {
        ctx->arena.release(X);
        ctx->arena.release(flags);
        return fail(MAPPER_EDEVICE, std::string("HIP error: ") + hipGetErrorString(de.e));
    }
}

mapper_status mapper_cloud_destroy(mapper_cloud *c) {
    if (!c) return fail(MAPPER_EINVAL, "null cloud");
    if (c->inflight.load() > 0) return fail(MAPPER_EBUSY, "cloud has requests in flight");
    c->ctx->arena.release(c->cell);
    c->ctx->arena.release(c->farcell);
    c->ctx->arena.release(c->ogap);
    c->ctx->arena.release(c->okey);
    c->ctx->arena.release(c->korder);
    c->ctx->arena.release(c->X);
    delete c;
    return MAPPER_OK;
}

mapper_status mapper_run(mapper_context *ctx, const mapper_cloud *cloud, const mapper_params *params,
                         mapper_graph **out) {
    if (!ctx || !out) return fail(MAPPER_EINVAL, "null argument");
    *out = nullptr;
    mapper_status v = validate(cloud, params);
    if (v != MAPPER_OK) return v;
    Retry retry;
    return run_guarded(ctx, cloud, params, ctx->stream, false, out, &retry);
}

static_assert(MAPPER_MAX_EPS_VALUES == mgpu::MAX_LEVELS, "eps values per pass");

mapper_status mapper_run_eps_sweep(mapper_context *ctx, const mapper_cloud *cloud, const mapper_params *params,
                                   const double *eps_list, int32_t n_eps, mapper_graph **out) {
    if (!ctx || !out || !eps_list) return fail(MAPPER_EINVAL, "null argument");
    if (n_eps < 1 || n_eps > MAPPER_MAX_EPS_VALUES) return fail(MAPPER_EINVAL, "n_eps must be in [1, MAPPER_MAX_EPS_VALUES]");
    for (int t = 0; t < n_eps; ++t) {
        out[t] = nullptr;
        if (!(eps_list[t] >= 0.0) || !std::isfinite(eps_list[t]))
            return fail(MAPPER_EINVAL, "eps values must be finite and >= 0");
    }
    mapper_status v = validate(cloud, params);
    if (v != MAPPER_OK) return v;
    Retry retry;
    return run_guarded(ctx, cloud, params, ctx->stream, false, out, &retry, eps_list, n_eps);
}

mapper_status mapper_run_sweep(mapper_context *ctx, const mapper_cloud *cloud, const mapper_params *params,
                               const double *eps_list, int32_t n_eps, const int32_t *minpts_list,
                               int32_t n_minpts, mapper_graph **out) {
    if (!ctx || !out || !eps_list || !minpts_list) return fail(MAPPER_EINVAL, "null argument");
    if (n_eps < 1 || n_eps > MAPPER_MAX_EPS_VALUES) return fail(MAPPER_EINVAL, "n_eps must be in [1, MAPPER_MAX_EPS_VALUES]");
    if (n_minpts < 1 || n_minpts > MAPPER_MAX_MINPTS_VALUES)
        return fail(MAPPER_EINVAL, "n_minpts must be in [1, MAPPER_MAX_MINPTS_VALUES]");
    for (int t = 0; t < n_eps * n_minpts; ++t) out[t] = nullptr;
    for (int t = 0; t < n_eps; ++t)
        if (!(eps_list[t] >= 0.0) || !std::isfinite(eps_list[t]))
            return fail(MAPPER_EINVAL, "eps values must be finite and >= 0");
    for (int u = 0; u < n_minpts; ++u)
        if (minpts_list[u] < 1) return fail(MAPPER_EINVAL, "minPts values must be >= 1");
    mapper_status v = validate(cloud, params);
    if (v != MAPPER_OK) return v;
    Retry retry;
    return run_guarded(ctx, cloud, params, ctx->stream, false, out, &retry, eps_list, n_eps, nullptr, minpts_list,
                       n_minpts);
}

mapper_status mapper_knn_d2(mapper_context *ctx, const mapper_cloud *cloud, int32_t k, int32_t precision,
                            double *out_d2, mapper_run_stats *stats) {
    if (!ctx || !cloud || !out_d2) return fail(MAPPER_EINVAL, "null argument");
    if (cloud->n < 2) return fail(MAPPER_EINVAL, "k-NN needs at least two points");
    if (k < 1 || k > KNN_KMAX || (int64_t)k > cloud->n - 1)
        return fail(MAPPER_EINVAL, "k must be in [1, min(16, n - 1)]");
    if (precision < 0 || precision > MAPPER_PREC_AUTO) return fail(MAPPER_EINVAL, "bad precision");
    // screening precision: the result is exact either way; FP16 (one product
    // per pair) was the fastest at 100k x 256 (35 ms against 56 for BF16x3,
    // with 1.8x the candidates)
    const int prec = precision == MAPPER_PREC_AUTO ? P_FP16 : precision;
    hipStream_t s = ctx->stream;
    try {
        HIPCHK(hipSetDevice(ctx->device));
        Scope mem(ctx->arena, s);
        double *dout = mem.get<double>(cloud->n);
        mapper_run_stats st{};
        knn_device(ctx, cloud, k, 0, prec, dout, st, s);
        HIPCHK(hipMemcpyAsync(out_d2, dout, (size_t)cloud->n * 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (stats) *stats = st;
        return MAPPER_OK;
    } catch (NoMem &) {
        (void)hipStreamSynchronize(s);
        return fail(MAPPER_ENOMEM, "arena too small for the k-NN tiles");
    } catch (DevError &de) {
        (void)hipStreamSynchronize(s);
        return fail(MAPPER_EDEVICE, std::string("HIP error: ") + hipGetErrorString(de.e));
    }
}

mapper_status mapper_submit(mapper_context *ctx, const mapper_cloud *cloud, const mapper_params *params,
                            uint64_t *ticket) {
    if (!ctx || !ticket) return fail(MAPPER_EINVAL, "null argument");
    mapper_status v = validate(cloud, params);
    if (v != MAPPER_OK) return v;
    auto *r = new Request();
    r->cloud = cloud;
    copy_params(cloud, params, r->params);
    const_cast<mapper_cloud *>(cloud)->inflight++;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (ctx->workers.empty()) {
            std::vector<hipStream_t> ss = ctx->slots;
            if (ss.empty()) ss.push_back(ctx->stream);
            for (hipStream_t s : ss) ctx->workers.emplace_back(worker_main, ctx, s);
        }
        r->ticket = ctx->next_ticket++;
        ctx->tickets[r->ticket] = r;
        ctx->pending.push_back(r);
        *ticket = r->ticket;
    }
    ctx->cv.notify_all();
    return MAPPER_OK;
}

mapper_status mapper_wait(mapper_context *ctx, uint64_t ticket, int64_t timeout_us, mapper_graph **out) {
    if (!ctx || !out) return fail(MAPPER_EINVAL, "null argument");
    *out = nullptr;
    std::unique_lock<std::mutex> lk(ctx->mu);
    auto it = ctx->tickets.find(ticket);
    if (it == ctx->tickets.end()) return fail(MAPPER_EINVAL, "unknown ticket");
    Request *r = it->second;
    if (timeout_us < 0) {
        ctx->cv.wait(lk, [&] { return r->done; });
    } else if (!ctx->cv.wait_for(lk, std::chrono::microseconds(timeout_us), [&] { return r->done; })) {
        return fail(MAPPER_ETIMEDOUT, "request still running");
    }
    ctx->tickets.erase(it);
    const mapper_status st = r->status;
    if (st != MAPPER_OK) g_last_error = r->err;
    *out = r->graph;
    delete r;
    return st;
}

int64_t mapper_graph_num_nodes(const mapper_graph *g) { return g ? (int64_t)g->node_element.size() : 0; }
int64_t mapper_graph_num_edges(const mapper_graph *g) { return g ? (int64_t)g->weights.size() : 0; }
const int32_t *mapper_graph_node_element(const mapper_graph *g) { return g ? g->node_element.data() : nullptr; }
const int64_t *mapper_graph_node_offsets(const mapper_graph *g) { return g ? g->node_offsets.data() : nullptr; }
const int32_t *mapper_graph_node_members(const mapper_graph *g) { return g ? g->node_members.data() : nullptr; }
const int32_t *mapper_graph_edges(const mapper_graph *g) { return g ? g->edges.data() : nullptr; }
const int32_t *mapper_graph_edge_weights(const mapper_graph *g) { return g ? g->weights.data() : nullptr; }

mapper_status mapper_graph_stats(const mapper_graph *g, mapper_run_stats *out) {
    if (!g || !out) return fail(MAPPER_EINVAL, "null argument");
    *out = g->stats;
    return MAPPER_OK;
}

const void *mapper_graph_stage(const mapper_graph *g, const char *name, int64_t *count) {
    if (!g || !name) return nullptr;
    auto it = g->stages.find(name);
    if (it == g->stages.end()) return nullptr;
    if (count) *count = it->second.second;
    return it->second.first.data();
}

void mapper_graph_destroy(mapper_graph *g) { delete g; }

}  // extern "C"

extern "C" mapper_status mapper_debug_tile_d2(mapper_context *ctx, const mapper_cloud *cloud,
                                              const int32_t *rows, int32_t nrows, int32_t precision,
                                              double eps, double *out_d2, double *out_band) {
    if (!ctx || !cloud || !rows || !out_d2 || !out_band || nrows < 1)
        return fail(MAPPER_EINVAL, "null argument or empty row set");
    if (precision < 0 || precision > P_FP16X3) return fail(MAPPER_EINVAL, "precision must be explicit");
    if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(MAPPER_EINVAL, "bad eps");
    for (int32_t i = 0; i < nrows; ++i)
        if (rows[i] < 0 || rows[i] >= cloud->n) return fail(MAPPER_EINVAL, "row id out of range");
    hipStream_t s = ctx->stream;
    try {
        HIPCHK(hipSetDevice(ctx->device));
        Scope mem(ctx->arena, s);
        const int32_t d = cloud->d;
        const int64_t T = (nrows + TILE - 1) / TILE, P = T * (T + 1) / 2;
        uint32_t *slot_point = mem.get<uint32_t>(nrows);
        h2d(slot_point, (const uint32_t *)rows, nrows, s);
        const int64_t eo[2] = {0, nrows};
        const int64_t io[2] = {0, P};
        const int64_t bo[1] = {0};
        const int32_t od[1] = {0};
        int64_t *d_eo = mem.get<int64_t>(2), *d_io = mem.get<int64_t>(2), *d_bo = mem.get<int64_t>(1);
        int32_t *d_od = mem.get<int32_t>(1);
        h2d(d_eo, eo, 2, s);
        h2d(d_io, io, 2, s);
        h2d(d_bo, bo, 1, s);
        h2d(d_od, od, 1, s);
        double scale = 1.0;
        if (cloud->maxabs > 0) scale = std::ldexp(1.0, 10 - std::ilogb((double)cloud->maxabs));
        const int dp = panel_dp(precision, d);
        PackArgs pk{};
        pk.X = cloud->X;
        pk.d = d;
        pk.dp = dp;
        pk.slot_point = slot_point;
        pk.n_slots = nrows;
        pk.prec = precision;
        pk.scale = scale;
        pk.n_levels = 1;
        pk.E_scaled[0] = eps * eps * scale * scale;
        pk.panel = mem.get<char>((uint64_t)nrows * (uint64_t)panel_row_stride(precision, dp));
        pk.thrA = mem.get<float>(nrows);
        pk.thrB = mem.get<float>(nrows);
        pk.dbg_norm2 = mem.get<double>(nrows);
        pk.dbg_e = mem.get<double>(nrows);
        HIPCHK(launch_pack(pk, s));
        TileArgs ta{};
        ta.tt.item_off = d_io;
        ta.tt.order = d_od;
        ta.tt.elem_off = d_eo;
        ta.tt.blk_off = d_bo;
        std::vector<int64_t> colpre, cp_off(1);
        const int super = supertile_size(d);
        build_supertile_columns(std::vector<int64_t>{T}, super, colpre, cp_off);
        int64_t *d_cp = mem.get<int64_t>(colpre.size()), *d_cpo = mem.get<int64_t>(1);
        h2d(d_cp, colpre.data(), (int64_t)colpre.size(), s);
        h2d(d_cpo, cp_off.data(), 1, s);
        ta.tt.colpre = d_cp;
        ta.tt.cp_off = d_cpo;
        ta.tt.nord = 1;
        ta.tt.super = super;
        ta.tt.n_items = P;
        TileItem *d_items = mem.get<TileItem>(std::max<int64_t>(P, 1));
        HIPCHK(launch_build_items(ta.tt, d_items, s));
        ta.tt.items = d_items;
        ta.panel = pk.panel;
        ta.dp = dp;
        ta.thrA = pk.thrA;
        ta.thrB = pk.thrB;
        ta.bitmask = mem.get<uint32_t>((uint64_t)P * TILE_WORDS);
        ta.bandmask = mem.get<uint32_t>((uint64_t)P * TILE_WORDS);
        ta.count = mem.get<int32_t>(nrows);
        ta.band_cap = 0;
        ta.band = nullptr;
        ta.band_n = mem.get<unsigned long long>(1);
        ta.nseg = 1;
        ta.n_levels = 1;
        ta.level_slots = nrows;
        ta.level_words = (uint64_t)P * TILE_WORDS;
        ta.debug_g = mem.get<float>((uint64_t)nrows * nrows);
        ta.debug_ld = nrows;
        HIPCHK(hipMemsetAsync(ta.count, 0, (size_t)nrows * 4, s));
        HIPCHK(hipMemsetAsync(ta.band_n, 0, 8, s));
        HIPCHK(launch_tiles(precision, ta, s));
        std::vector<float> g;
        std::vector<double> nn, ee;
        d2h(g, ta.debug_g, (int64_t)nrows * nrows, s);
        d2h(nn, pk.dbg_norm2, nrows, s);
        d2h(ee, pk.dbg_e, nrows, s);
        HIPCHK(hipStreamSynchronize(s));
        const double inv = 1.0 / (scale * scale);
        for (int64_t i = 0; i < nrows; ++i)
            for (int64_t j = 0; j < nrows; ++j) {
                out_d2[i * nrows + j] = (nn[i] + nn[j] - 2.0 * (double)g[i * nrows + j]) * inv;
                out_band[i * nrows + j] = 2.0 * (ee[i] + ee[j]) * inv;
            }
        return MAPPER_OK;
    } catch (NoMem &) {
        (void)hipStreamSynchronize(s);
        return fail(MAPPER_ENOMEM, "arena too small for the debug tiles");
    } catch (DevError &de) {
        (void)hipStreamSynchronize(s);
        return fail(MAPPER_EDEVICE, std::string("HIP error: ") + hipGetErrorString(de.e));
    }
}

extern "C" mapper_status mapper_debug_lens(mapper_context *ctx, const mapper_cloud *cloud,
                                           const mapper_axis *axis, double *out) {
    if (!ctx || !cloud || !axis || !out) return fail(MAPPER_EINVAL, "null argument");
    mapper_params p{};
    p.n_axes = 1;
    p.axis[0] = *axis;
    p.axis[0].n_intervals = 1;
    p.axis[0].overlap = 0.0;
    p.axis[0].cover = MAPPER_COVER_UNIFORM;
    p.eps = 0.0;
    p.min_pts = 1;
    p.precision = MAPPER_PREC_FP32;
    mapper_status v = validate(cloud, &p);
    if (v != MAPPER_OK) return v;
    hipStream_t s = ctx->stream;
    try {
        HIPCHK(hipSetDevice(ctx->device));
        Scope mem(ctx->arena, s);
        const int64_t n = cloud->n;
        const int32_t d = cloud->d;
        double *f = mem.get<double>(std::max<int64_t>(n, 1));
        const mapper_axis &ax = p.axis[0];
        float *dir = nullptr;
        double *vals = nullptr;
        if (ax.kind == MAPPER_LENS_PROJECTION) {
            dir = mem.get<float>(d);
            h2d(dir, ax.direction, d, s);
        }
        if (ax.kind == MAPPER_LENS_VALUES) {
            vals = mem.get<double>(n);
            h2d(vals, ax.values, n, s);
        }
        if (ax.kind == MAPPER_LENS_KNN_DISTANCE || ax.kind == MAPPER_LENS_ECCENTRICITY) {
            mapper_run_stats ks{};
            const bool ecc = ax.kind == MAPPER_LENS_ECCENTRICITY;
            knn_device(ctx, cloud, ecc ? 1 : ax.column, ecc ? 1 : 0, P_FP16, f, ks, s);
            HIPCHK(launch_sqrt(f, n, s));
        } else {
            HIPCHK(launch_lens(cloud->X, n, d, ax.kind, ax.column, dir, vals, f, s));
        }
        HIPCHK(hipMemcpyAsync(out, f, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        return MAPPER_OK;
    } catch (NoMem &) {
        (void)hipStreamSynchronize(s);
        return fail(MAPPER_ENOMEM, "arena too small for the lens");
    } catch (DevError &de) {
        (void)hipStreamSynchronize(s);
        return fail(MAPPER_EDEVICE, std::string("HIP error: ") + hipGetErrorString(de.e));
    }
}

extern "C" mapper_status mapper_debug_sqrt(mapper_context *ctx, const double *in, int64_t n, double *out) {
    if (!ctx || (n > 0 && (!in || !out)) || n < 0) return fail(MAPPER_EINVAL, "null argument or negative count");
    if (n == 0) return MAPPER_OK;
    hipStream_t s = ctx->stream;
    try {
        HIPCHK(hipSetDevice(ctx->device));
        Scope mem(ctx->arena, s);
        double *f = mem.get<double>(n);
        HIPCHK(hipMemcpyAsync(f, in, (size_t)n * sizeof(double), hipMemcpyHostToDevice, s));
        HIPCHK(launch_sqrt(f, n, s));
        HIPCHK(hipMemcpyAsync(out, f, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        return MAPPER_OK;
    } catch (NoMem &) {
        (void)hipStreamSynchronize(s);
        return fail(MAPPER_ENOMEM, "arena too small");
    } catch (DevError &de) {
        (void)hipStreamSynchronize(s);
        return fail(MAPPER_EDEVICE, std::string("HIP error: ") + hipGetErrorString(de.e));
    }
}

extern "C" mapper_status mapper_knn_d2_noalloc(mapper_context *ctx, const float *points, int64_t n, int32_t d,
                                               int32_t k, int32_t precision, double *out_d2) {
    if (!ctx || !points || !out_d2) return fail(MAPPER_EINVAL, "null argument");
    if (n < 2 || n > 0x7fffffff || d < 1 || d > (1 << 16))
        return fail(MAPPER_EINVAL, "need 2 <= n < 2^31 and 1 <= d <= 65536");
    if (k < 1 || k > KNN_KMAX || (int64_t)k > n - 1) return fail(MAPPER_EINVAL, "k must be in [1, min(16, n - 1)]");
    if (precision < 0 || precision > MAPPER_PREC_AUTO) return fail(MAPPER_EINVAL, "bad precision");
    const int prec = precision == MAPPER_PREC_AUTO ? P_FP16 : precision;
    const int32_t T = (int32_t)((n + TILE - 1) / TILE);
    int32_t C = (int32_t)std::max<int64_t>(1, std::min<int64_t>(T, (4 * ctx->cus + T - 1) / T));
    int32_t cmax = 64;
    while (C > 1 && knn_scratch_bytes(n, d, prec, T, C, cmax) > NOALLOC_SCRATCH_BYTES) --C;
    const uint64_t need = knn_scratch_bytes(n, d, prec, T, C, cmax);
    if (need <= NOALLOC_SCRATCH_BYTES) {
        // longer lists where the array has room (up to 1024 entries): a row
        // with more candidates than the lists hold redoes pass 2
        const uint64_t rest = NOALLOC_SCRATCH_BYTES - knn_scratch_bytes(n, d, prec, T, C, 0);
        const uint64_t fit = rest > 256 ? (rest - 256) / ((uint64_t)n * 4) : 0;
        cmax = (int32_t)std::max<uint64_t>(64, std::min<uint64_t>(1024, fit));
    }
    if (need > NOALLOC_SCRATCH_BYTES) {
        char msg[160];
        std::snprintf(msg, sizeof msg, "n x d too large for the no-alloc scratch: needs %llu bytes, the array holds %llu",
                      (unsigned long long)need, (unsigned long long)NOALLOC_SCRATCH_BYTES);
        return fail(MAPPER_EINVAL, msg);
    }
    char *base = (char *)scratch_of(ctx->device);
    if (!base) return fail(MAPPER_EDEVICE, "scratch array not resolved for this device");
    std::lock_guard<std::mutex> serial(g_noalloc_mu[ctx->device]);   // calls on one device share the array
    hipStream_t s = ctx->stream;
    try {
        HIPCHK(hipSetDevice(ctx->device));
        ScratchCarve sc{base, 0, NOALLOC_SCRATCH_BYTES};
        uint32_t *flags = sc.take<uint32_t>(64);              // [0] non-finite, [1] max |x| bits, [2] most candidates
        uint32_t *ident = sc.take<uint32_t>(n);
        const int dp = panel_dp(prec, d);
        char *panel = sc.take<char>((uint64_t)n * (uint64_t)panel_row_stride(prec, dp));
        float *hU = sc.take<float>(n), *hL = sc.take<float>(n);
        float *part = sc.take<float>((uint64_t)C * T * TILE * 4 * KNN_KMAX);
        float *thr = sc.take<float>(n);
        int32_t *ccnt = sc.take<int32_t>(n);
        const uint64_t cand_off = sc.used;
        int32_t *cand = sc.take<int32_t>((uint64_t)n * cmax);
        if (!flags || !ident || !panel || !hU || !hL || !part || !thr || !ccnt || !cand)
            return fail(MAPPER_EINVAL, "scratch layout does not fit");   // not reached: sized above
        // finiteness and the largest magnitude (the panels' power-of-two scale)
        HIPCHK(hipMemsetAsync(flags, 0, 16, s));
        HIPCHK(launch_check_cloud(points, n * (int64_t)d, flags, s));
        uint32_t h[2] = {0, 0};
        HIPCHK(hipMemcpyAsync(h, flags, 8, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (h[0]) return fail(MAPPER_EINVAL, "points have non-finite coordinates");
        float maxabs = 0.f;
        std::memcpy(&maxabs, &h[1], 4);
        double scale = 1.0;
        if (maxabs > 0) scale = std::ldexp(1.0, 10 - std::ilogb((double)maxabs));
        HIPCHK(launch_iota_u32(ident, n, s));
        PackArgs pk{};
        pk.X = points;
        pk.d = d;
        pk.dp = dp;
        pk.slot_point = ident;
        pk.n_slots = n;
        pk.prec = prec;
        pk.scale = scale;
        pk.n_levels = 1;
        pk.E_scaled[0] = 0.0;
        pk.panel = panel;
        pk.thrA = hU;
        pk.thrB = hL;
        HIPCHK(launch_pack(pk, s));
        KnnArgs ka{};
        ka.t.panel = panel;
        ka.t.dp = dp;
        ka.t.n_levels = 1;
        ka.mode = 0;
        ka.k = k;
        ka.n = n;
        ka.T = T;
        ka.C = C;
        ka.hU = hU;
        ka.hL = hL;
        ka.part = part;
        ka.thr = thr;
        HIPCHK(launch_knn_pass(prec, 1, ka, s));
        HIPCHK(launch_knn_merge(part, C, T, n, k, thr, s));
        for (;;) {
            ka.cand = cand;
            ka.ccnt = ccnt;
            ka.cmax = cmax;
            HIPCHK(hipMemsetAsync(ccnt, 0, (size_t)n * 4, s));
            HIPCHK(hipMemsetAsync(flags + 2, 0, 4, s));
            HIPCHK(launch_knn_pass(prec, 2, ka, s));
            HIPCHK(launch_max_i32(ccnt, n, (int32_t *)(flags + 2), s));
            int32_t most = 0;
            HIPCHK(hipMemcpyAsync(&most, flags + 2, 4, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            if (most <= cmax) {
                HIPCHK(launch_knn_final(points, d, n, k, cand, ccnt, cmax, 0, nullptr, out_d2, s));
                HIPCHK(hipStreamSynchronize(s));
                break;
            }
            // longer candidate lists: the rest of the array, or an error
            if ((uint64_t)most * (uint64_t)n * 4 > NOALLOC_SCRATCH_BYTES - cand_off)
                return fail(MAPPER_EINVAL, "candidate lists exceed the no-alloc scratch (many equal distances)");
            cmax = most;
        }
        return MAPPER_OK;
    } catch (DevError &de) {
        (void)hipStreamSynchronize(s);
        return fail(MAPPER_EDEVICE, std::string("HIP error: ") + hipGetErrorString(de.e));
    }
}
