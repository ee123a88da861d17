// Host side of the C ABI: validation, contexts, workspaces, dispatch.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "common.h"

#include <map>
#include <mutex>
#include <tuple>
#include <vector>

namespace corr {

static thread_local std::string g_last_error;

// Fixed device scratch of the no-allocation entry point: one copy per GPU,
// held until the process ends. Host code never passes `scratch` itself to a
// kernel (in host code the name is a host-side stand-in); it uses the device
// address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[CORR_SCRATCH_BYTES];

// The device address of `scratch` on `device` (the caller has made it
// current), looked up once per device.
static int scratch_address(int device, void** out) {
    static std::mutex mu;
    static std::map<int, void*> addr;
    std::lock_guard<std::mutex> lock(mu);
    auto it = addr.find(device);
    if (it == addr.end()) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr) {
            (void)hipGetLastError();
            return fail(CORR_EHIP, std::string("scratch symbol address: ") + hipGetErrorString(e));
        }
        it = addr.emplace(device, p).first;
    }
    *out = it->second;
    return CORR_OK;
}

void set_error(const std::string& msg) { g_last_error = msg; }

int fail(int status, const std::string& msg) {
    g_last_error = msg;
    return status;
}

int ctx_use_stream(corr_ctx* ctx, hipStream_t s) {
    if (ctx->used && ctx->last_stream != s) CORR_HIP(hipDeviceSynchronize());
    ctx->used = true;
    ctx->last_stream = s;
    return CORR_OK;
}

int ws_get(corr_ctx* ctx, int slot, size_t bytes, hipStream_t stream, void** out) {
    if (bytes == 0) bytes = 256;
    if (ctx->ws_size[slot] < bytes) {
        size_t others = 0;
        for (int i = 0; i < WS_COUNT; ++i)
            if (i != slot) others += ctx->ws_size[i];
        if (bytes > ctx->ws_limit || others > ctx->ws_limit - bytes)
            return fail(CORR_ENOMEM, "workspace limit: the call needs " + std::to_string(others + bytes) +
                                         " bytes of context workspace, the limit is " + std::to_string(ctx->ws_limit));
        if (ctx->ws[slot]) {
            CORR_HIP(hipStreamSynchronize(stream));
            CORR_HIP(hipFree(ctx->ws[slot]));
            ctx->ws[slot] = nullptr;
            ctx->ws_size[slot] = 0;
        }
        size_t want = bytes + bytes / 8;
        if (want > ctx->ws_limit - others) want = bytes;
        hipError_t e = hipMalloc(&ctx->ws[slot], want);
        if (e != hipSuccess) {
            ctx->ws[slot] = nullptr;
            (void)hipGetLastError();
            return fail(CORR_ENOMEM, "workspace allocation of " + std::to_string(want) + " bytes failed");
        }
        ctx->ws_size[slot] = want;
    }
    *out = ctx->ws[slot];
    return CORR_OK;
}

// Where a call's workspaces come from: the context's grow-only slots, or a
// fixed arena carved front to back in 256-byte steps (the no-allocation
// entry point), which fails with CORR_EINVAL when the call needs more.
struct Ws {
    corr_ctx* ctx = nullptr;
    char* arena = nullptr;
    size_t cap = 0;
    size_t used = 0;
    std::vector<void*>* owned = nullptr;  // set: every buffer is a new allocation recorded here
    int get(int slot, size_t bytes, hipStream_t s, void** out) {
        if (owned) {
            void* p = nullptr;
            hipError_t e = hipMalloc(&p, bytes ? bytes : 256);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                return fail(CORR_ENOMEM, "allocation of " + std::to_string(bytes) + " bytes failed");
            }
            owned->push_back(p);
            *out = p;
            return CORR_OK;
        }
        if (!arena) return ws_get(ctx, slot, bytes, s, out);
        const size_t off = (used + 255) & ~size_t(255);
        if (bytes > cap || off > cap - bytes)
            return fail(CORR_EINVAL, "the call needs more than the " + std::to_string(cap >> 20) +
                                         " MiB of fixed scratch (at least " + std::to_string(off + bytes) + " bytes)");
        *out = arena + off;
        used = off + bytes;
        return CORR_OK;
    }
};

int kernel_setup(const void* fn, size_t lds, int threads, int* per_cu) {
    struct Key {
        int device;
        const void* fn;
        size_t lds;
        int threads;
        bool operator<(const Key& o) const {
            return std::tie(device, fn, lds, threads) < std::tie(o.device, o.fn, o.lds, o.threads);
        }
    };
    static std::mutex mu;
    static std::map<Key, int> done;
    int dev = 0;
    CORR_HIP(hipGetDevice(&dev));
    const Key key{dev, fn, lds, threads};
    std::lock_guard<std::mutex> lock(mu);
    auto it = done.find(key);
    if (it == done.end()) {
        if (lds > 64 * 1024) CORR_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        int n = 0;
        CORR_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, threads, lds));
        it = done.emplace(key, n < 1 ? 1 : n).first;
    }
    if (per_cu) *per_cu = it->second;
    return CORR_OK;
}

__global__ void fill_u64_kernel(unsigned long long* p, int64_t n, unsigned long long v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

int launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s) {
    fill_u64_kernel<<<dim3((unsigned)((n + 255) / 256)), 256, 0, s>>>(p, n, v);
    CORR_LAUNCH_CHECK();
    return CORR_OK;
}

__global__ void self_col_kernel(Box a, Box b, int32_t* out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < a.count()) out[i] = (int32_t)b.local(a.global(i));
}

void timing_begin(corr_ctx* ctx, int which, hipStream_t s) {
    if (ctx->timing) (void)hipEventRecord(ctx->ev_start[which], s);
}

void timing_end(corr_ctx* ctx, int which, hipStream_t s) {
    if (ctx->timing) {
        (void)hipEventRecord(ctx->ev_stop[which], s);
        ctx->ev_valid[which] = true;
    }
}

// ---- validation -------------------------------------------------------------
static int64_t field_points(const corr_field& f) { return (int64_t)f.nx * f.ny * f.nz; }

static int check_field(const corr_field* f, const char* name) {
    if (!f) return fail(CORR_EINVAL, std::string(name) + ": null field");
    if (!f->data) return fail(CORR_EINVAL, std::string(name) + ": null data pointer");
    if (f->dtype != CORR_F32 && f->dtype != CORR_F16)
        return fail(CORR_EUNSUPPORTED, std::string(name) + ": unsupported dtype");
    if (f->M < 2) return fail(CORR_EINVAL, std::string(name) + ": M must be >= 2");
    if (f->nx < 1 || f->ny < 1 || f->nz < 1) return fail(CORR_EINVAL, std::string(name) + ": empty grid");
    if (field_points(*f) >= (int64_t(1) << 31))
        return fail(CORR_EUNSUPPORTED, std::string(name) + ": more than 2^31-1 grid points");
    if (f->member_stride != 0 && f->member_stride < field_points(*f))
        return fail(CORR_EINVAL, std::string(name) + ": member_stride smaller than the grid");
    return CORR_OK;
}

static int check_region(const corr_region* r, const corr_field& f, const char* name) {
    if (!r) return fail(CORR_EINVAL, std::string(name) + ": null region");
    if (r->dx < 1 || r->dy < 1 || r->dz < 1) return fail(CORR_EINVAL, std::string(name) + ": empty region");
    if (r->x0 < 0 || r->y0 < 0 || r->z0 < 0 || r->x0 + r->dx > f.nx || r->y0 + r->dy > f.ny ||
        r->z0 + r->dz > f.nz)
        return fail(CORR_EINVAL, std::string(name) + ": region outside the grid");
    return CORR_OK;
}

static bool same_field(const corr_field& a, const corr_field& b) {
    int64_t sa = a.member_stride ? a.member_stride : field_points(a);
    int64_t sb = b.member_stride ? b.member_stride : field_points(b);
    return a.data == b.data && a.dtype == b.dtype && a.M == b.M && a.nx == b.nx && a.ny == b.ny && a.nz == b.nz &&
           sa == sb;
}

static Box whole_box(const corr_field& f) { return Box{0, 0, 0, f.nx, f.ny, f.nz, f.nx, f.ny}; }
static Box region_box(const corr_region& r, const corr_field& f) {
    return Box{r.x0, r.y0, r.z0, r.dx, r.dy, r.dz, f.nx, f.ny};
}

static int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

static bool boxes_overlap(const Box& a, const Box& b) {
    return a.x0 < b.x0 + b.dx && b.x0 < a.x0 + a.dx && a.y0 < b.y0 + b.dy && b.y0 < a.y0 + a.dy &&
           a.z0 < b.z0 + b.dz && b.z0 < a.z0 + a.dz;
}
static int64_t overlap_count(const Box& a, const Box& b) {
    if (!boxes_overlap(a, b)) return 0;
    int64_t ox = std::min(a.x0 + a.dx, b.x0 + b.dx) - std::max(a.x0, b.x0);
    int64_t oy = std::min(a.y0 + a.dy, b.y0 + b.dy) - std::max(a.y0, b.y0);
    int64_t oz = std::min(a.z0 + a.dz, b.z0 + b.dz) - std::max(a.z0, b.z0);
    return ox * oy * oz;
}

// Statistics accumulate in FP64 for KSG (its integer counts must be exactly
// reproducible) and for large ensembles (cancellation); FP32 otherwise.
static bool stats_acc64(int measure, int M) { return measure == CORR_KSG || M > 256; }

// Standardise the points of `box` into (stats slot, hi slot, lo slot).
static int standardize_box(Ws& w, const corr_field& f, const Box& box, bool acc64, int fmt, int64_t rows_pad,
                           int64_t ld, int stats_slot, int hi_slot, int lo_slot, hipStream_t s, Stats* st_out,
                           void** hi, void** lo) {
    const int64_t n = box.count();
    void* sb = nullptr;
    int rc = w.get(stats_slot, sizeof(float) * 4 * (size_t)n, s, &sb);
    if (rc) return rc;
    Stats st = stats_view((float*)sb, n);
    if (fmt != ZF_RAW) {
        rc = launch_stats(f, box, acc64, st, s);
        if (rc) return rc;
    }
    size_t es = (fmt == ZF_KSG || fmt == ZF_RAW || fmt == ZF_F32) ? 4 : 2;
    rc = w.get(hi_slot, es * (size_t)(rows_pad * ld), s, hi);
    if (rc) return rc;
    *lo = nullptr;
    if (fmt == ZF_F16X2 || fmt == ZF_BF16X2) {
        rc = w.get(lo_slot, es * (size_t)(rows_pad * ld), s, lo);
        if (rc) return rc;
    }
    rc = launch_transpose(f, box, st, fmt, *hi, *lo, rows_pad, ld, s);
    if (rc) return rc;
    if (st_out) *st_out = st;
    return CORR_OK;
}

// Each standardised row sorted ascending (the marginals KSG counts on).
static int sorted_rows(Ws& w, const float* z, int64_t ld, int64_t nrows, int M, int slot, hipStream_t s,
                       void** out) {
    int rc = w.get(slot, sizeof(float) * (size_t)nrows * ksg_p2(M), s, out);
    if (rc) return rc;
    return launch_sort_rows(z, ld, nrows, M, (float*)*out, w.ctx->num_cus, s);
}

static int read_keys(corr_ctx* ctx, hipStream_t s, unsigned long long* k0, unsigned long long* k1) {
    CORR_HIP(hipMemcpyAsync(ctx->keys_host, ctx->keys, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    CORR_HIP(hipStreamSynchronize(s));
    *k0 = ctx->keys_host[0];
    *k1 = ctx->keys_host[1];
    return CORR_OK;
}

static void decode_key(unsigned long long key, const Box& ba, const Box& bb, bool is_abs, corr_max* out) {
    if (key == 0) {
        out->value = 0.0f;
        out->signed_value = 0.0f;
        out->pa = out->pb = -1;
        return;
    }
    float v = from_order_bits((uint32_t)(key >> 32));
    uint32_t lin = key_lin(key);
    int64_t nb = bb.count();
    int64_t la = lin / nb, lb = lin % nb;
    out->value = v;
    out->signed_value = (is_abs && (key & 1ull)) ? -v : v;
    out->pa = ba.global(la);
    out->pb = bb.global(lb);
}

// Default small-K tile configuration before any tuning: measured fastest on
// gfx950 for the 20480 x 20480 focus-view shape.
// Untuned default: the first usable configuration in order of measured
// preference for the precision class (split modes need one row block per
// wave; a configuration whose kernel would spill at this K is skipped).
static int default_smallk_cfg(int prec, int K) {
    static const int pref16[] = {6, 7, 5, 3, 2, 1, 4, 0};
    static const int pref32[] = {7, 6, 3, 1, 4, 5, 2, 0};
    static const int prefsplit[] = {3, 4, 6, 7, 1, 5};
    const int* p = prec_split(prec) ? prefsplit : (prec == CORR_PREC_F32 ? pref32 : pref16);
    const int n = prec_split(prec) ? 6 : 8;
    for (int i = 0; i < n; ++i)
        if (smallk_config_ok(prec, p[i], K)) return p[i];
    return 3;
}

static int tuned_smallk_cfg(corr_ctx* ctx, int K, int prec, int64_t na, int64_t nb) {
    for (const corr_tune_rec& r : ctx->tune)
        if (r.kind == 0 && r.K == K && r.prec == prec && r.na == na && r.nb == nb && smallk_config_ok(prec, r.cfg, K))
            return r.cfg;
    return default_smallk_cfg(prec, K);
}

static int tuned_ksg_pw(corr_ctx* ctx, int M, int k) {
    for (const corr_tune_rec& r : ctx->tune)
        if (r.kind == 1 && r.K == M && r.prec == k) return r.cfg;
    return 0;
}

static void tune_store(corr_ctx* ctx, const corr_tune_rec& rec) {
    for (corr_tune_rec& r : ctx->tune)
        if (r.kind == rec.kind && r.K == rec.K && r.prec == rec.prec && r.na == rec.na && r.nb == rec.nb) {
            r = rec;
            return;
        }
    ctx->tune.push_back(rec);
}

// Exhaustive Pearson region maximum: standardise both regions into the
// contraction layout, run the fused MFMA contraction, decode the key.
// cfg < 0 selects the tuned (or default) small-K configuration.
static int pearson_exhaustive(Ws& w, const corr_field& A, const Box& ba, const corr_field& B, const Box& bb,
                              bool sf, int prec, int cfg, corr_max* out, hipStream_t s) {
    corr_ctx* ctx = w.ctx;
    const int64_t na = ba.count(), nb = bb.count();
    const bool acc64 = stats_acc64(CORR_PEARSON, A.M);
    const int fmt = zfmt_for_prec(prec);
    const bool small = A.M <= 128;
    int64_t K, row_pad, col_pad;
    if (small) {
        K = smallk_pad_K(A.M);
        if (cfg < 0) cfg = tuned_smallk_cfg(ctx, (int)K, prec, na, nb);
        if (!smallk_config_ok(prec, cfg, (int)K)) return fail(CORR_EINVAL, "tile configuration not valid for this precision");
        row_pad = smallk_row_pad(cfg);
        col_pad = smallk_col_pad(cfg);
    } else {
        K = round_up(A.M, gemm_k_pad(prec));
        row_pad = gemm_row_pad();
        col_pad = gemm_col_pad();
    }
    const int64_t na_pad = round_up(na, row_pad), nb_pad = round_up(nb, col_pad);
    void *ah, *al, *bh, *bl;
    int rc = launch_fill_u64(ctx->keys, 2, 0ull, s);
    if (rc) return rc;
    rc = standardize_box(w, A, ba, acc64, fmt, na_pad, K, WS_STATS_A, WS_ZH_A, WS_ZL_A, s, nullptr, &ah, &al);
    if (rc) return rc;
    rc = standardize_box(w, B, bb, acc64, fmt, nb_pad, K, WS_STATS_B, WS_ZH_B, WS_ZL_B, s, nullptr, &bh, &bl);
    if (rc) return rc;
    const int32_t* self_col = nullptr;
    int64_t n_self = 0;
    if (sf && boxes_overlap(ba, bb)) {
        void* m = nullptr;
        rc = w.get(WS_MISC, sizeof(int32_t) * (size_t)na, s, &m);
        if (rc) return rc;
        self_col_kernel<<<dim3((unsigned)((na + 255) / 256)), 256, 0, s>>>(ba, bb, (int32_t*)m);
        CORR_LAUNCH_CHECK();
        self_col = (const int32_t*)m;
        n_self = overlap_count(ba, bb);
    }
    GemmArgs g{};
    g.prec = prec;
    g.a_hi = ah; g.a_lo = al; g.b_hi = bh; g.b_lo = bl;
    g.K = K;
    g.na = na; g.nb = nb; g.na_pad = na_pad; g.nb_pad = nb_pad;
    g.self_col = self_col;
    g.key = ctx->keys;
    timing_begin(ctx, TK_GEMM, s);
    rc = small ? launch_gemm_smallk(g, cfg, ctx->num_cus, s) : launch_gemm_max(g, ctx->num_cus, s);
    timing_end(ctx, TK_GEMM, s);
    if (rc) return rc;
    unsigned long long k0, k1;
    if ((rc = read_keys(ctx, s, &k0, &k1))) return rc;
    decode_key(k0, ba, bb, true, out);
    out->n_evaluated = na * nb - n_self;
    return CORR_OK;
}

}  // namespace corr

using namespace corr;

extern "C" {

const char* corr_version(void) { return "libcorr 0.1 (gfx950)"; }

const char* corr_status_str(int status) {
    switch (status) {
        case CORR_OK: return "ok";
        case CORR_EINVAL: return "invalid argument";
        case CORR_EUNSUPPORTED: return "unsupported";
        case CORR_ENOMEM: return "out of memory";
        case CORR_EHIP: return "HIP error";
        case CORR_ESTATE: return "invalid state";
    }
    return "unknown status";
}

const char* corr_last_error(void) { return g_last_error.c_str(); }

int corr_create(int device, corr_ctx** out) {
    if (!out) return fail(CORR_EINVAL, "corr_create: null out");
    *out = nullptr;
    int ndev = 0;
    CORR_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(CORR_EINVAL, "corr_create: no such device");
    CORR_HIP(hipSetDevice(device));
    corr_ctx* c = new (std::nothrow) corr_ctx();
    if (!c) return fail(CORR_ENOMEM, "corr_create: host allocation failed");
    c->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) c->num_cus = prop.multiProcessorCount;
    // digamma at integers (the log-derivative of Gamma): psi(1) = -gamma,
    // psi(n + 1) = psi(n) + 1/n.
    c->psi_max = 4100;
    double* h = new double[c->psi_max + 1];
    h[0] = 0.0;
    h[1] = -0.57721566490153286060651209008240243;
    for (int n = 1; n < c->psi_max; ++n) h[n + 1] = h[n] + 1.0 / (double)n;
    hipError_t e = hipMalloc(&c->psi, sizeof(double) * (c->psi_max + 1));
    if (e == hipSuccess) e = hipMemcpy(c->psi, h, sizeof(double) * (c->psi_max + 1), hipMemcpyHostToDevice);
    delete[] h;
    if (e == hipSuccess) e = hipMalloc(&c->keys, 64 * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipHostMalloc(&c->keys_host, 64 * sizeof(unsigned long long), hipHostMallocDefault);
    for (int i = 0; i < TK_COUNT && e == hipSuccess; ++i) {
        e = hipEventCreate(&c->ev_start[i]);
        if (e == hipSuccess) e = hipEventCreate(&c->ev_stop[i]);
    }
    if (e != hipSuccess) {
        corr_destroy(c);
        return fail(CORR_EHIP, std::string("corr_create: ") + hipGetErrorString(e));
    }
    if (scratch_address(device, &c->scratch) != CORR_OK) {
        const std::string msg = "corr_create: " + g_last_error;
        corr_destroy(c);
        return fail(CORR_EHIP, msg);
    }
    *out = c;
    return CORR_OK;
}

void corr_destroy(corr_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    for (int i = 0; i < WS_COUNT; ++i)
        if (c->ws[i]) (void)hipFree(c->ws[i]);
    if (c->psi) (void)hipFree(c->psi);
    if (c->keys) (void)hipFree(c->keys);
    if (c->keys_host) (void)hipHostFree(c->keys_host);
    for (int i = 0; i < TK_COUNT; ++i) {
        if (c->ev_start[i]) (void)hipEventDestroy(c->ev_start[i]);
        if (c->ev_stop[i]) (void)hipEventDestroy(c->ev_stop[i]);
    }
    delete c;
}

int corr_set_workspace_limit(corr_ctx* ctx, size_t bytes) {
    if (!ctx) return fail(CORR_EINVAL, "null context");
    ctx->ws_limit = bytes == 0 ? (size_t)-1 : bytes;
    return CORR_OK;
}

int corr_set_timing(corr_ctx* ctx, int on) {
    if (!ctx) return fail(CORR_EINVAL, "null context");
    ctx->timing = on != 0;
    return CORR_OK;
}

int corr_kernel_time_ms(corr_ctx* ctx, int which, float* ms) {
    if (!ctx || !ms) return fail(CORR_EINVAL, "null argument");
    if (which < 0 || which >= TK_COUNT) return fail(CORR_EINVAL, "unknown kernel class");
    *ms = -1.0f;
    if (!ctx->ev_valid[which]) return CORR_OK;
    CORR_HIP(hipEventSynchronize(ctx->ev_stop[which]));
    CORR_HIP(hipEventElapsedTime(ms, ctx->ev_start[which], ctx->ev_stop[which]));
    return CORR_OK;
}

int corr_autotune(corr_ctx* ctx, const corr_field* A, const corr_region* ra, const corr_field* B,
                  const corr_region* rb, int prec, int reps, int* best_cfg, float* best_ms, corr_stream_t stream) {
    if (!ctx) return fail(CORR_EINVAL, "null context");
    int rc = check_field(A, "A");
    if (rc) return rc;
    if ((rc = check_field(B, "B"))) return rc;
    if (A->M != B->M) return fail(CORR_EINVAL, "fields differ in M");
    if ((rc = check_region(ra, *A, "ra"))) return rc;
    if ((rc = check_region(rb, *B, "rb"))) return rc;
    if (prec < CORR_PREC_F32 || prec > CORR_PREC_BF16X3) return fail(CORR_EUNSUPPORTED, "unknown precision");
    if (reps < 1) return fail(CORR_EINVAL, "reps < 1");
    if (best_cfg) *best_cfg = -1;
    if (best_ms) *best_ms = -1.0f;
    if (A->M > 128) return CORR_OK;  // the chunked contraction has a single configuration
    hipStream_t s = (hipStream_t)stream;
    if ((rc = ctx_use_stream(ctx, s))) return rc;
    Box ba = region_box(*ra, *A), bb = region_box(*rb, *B);
    if (ba.count() * bb.count() >= (int64_t(1) << 31))
        return fail(CORR_EUNSUPPORTED, "region pair has 2^31 or more point pairs");
    const bool sf = same_field(*A, *B);
    const bool saved_timing = ctx->timing;
    ctx->timing = true;
    int best = -1;
    float best_t = 0.0f;
    std::vector<float> t(reps);
    Ws w{ctx};
    for (int cfg = 0; cfg < smallk_num_configs(); ++cfg) {
        if (!smallk_config_ok(prec, cfg, smallk_pad_K(A->M))) continue;
        corr_max tmp;
        rc = pearson_exhaustive(w, *A, ba, *B, bb, sf, prec, cfg, &tmp, s);  // warm-up
        for (int r = 0; r < reps && rc == CORR_OK; ++r) {
            rc = pearson_exhaustive(w, *A, ba, *B, bb, sf, prec, cfg, &tmp, s);
            if (rc == CORR_OK) rc = corr_kernel_time_ms(ctx, TK_GEMM, &t[r]);
        }
        if (rc) {
            ctx->timing = saved_timing;
            return rc;
        }
        std::sort(t.begin(), t.end());
        float med = t[reps / 2];
        if (best < 0 || med < best_t) {
            best = cfg;
            best_t = med;
        }
    }
    ctx->timing = saved_timing;
    tune_store(ctx, {0, smallk_pad_K(A->M), prec, ba.count(), bb.count(), best, best_t});
    if (best_cfg) *best_cfg = best;
    if (best_ms) *best_ms = best_t;
    return CORR_OK;
}

int corr_ksg_autotune(corr_ctx* ctx, const corr_field* A, const corr_field* B, const int32_t* pairs, int64_t n,
                      int32_t k, int reps, int* best_pw, float* best_ms, corr_stream_t stream) {
    if (!ctx) return fail(CORR_EINVAL, "null context");
    if (reps < 1) return fail(CORR_EINVAL, "reps < 1");
    if (best_pw) *best_pw = -1;
    if (best_ms) *best_ms = -1.0f;
    if (n <= 0) return fail(CORR_EINVAL, "autotuning needs a non-empty pair list");
    if (!A) return fail(CORR_EINVAL, "A: null field");
    std::vector<float> out_host;  // unused; results go to a workspace
    void* mi = nullptr;
    hipStream_t s = (hipStream_t)stream;
    if (int rc_ = ctx_use_stream(ctx, s)) return rc_;
    int rc = ws_get(ctx, WS_PAIRS, sizeof(float) * (size_t)n, s, &mi);
    if (rc) return rc;
    const bool saved_timing = ctx->timing;
    ctx->timing = true;
    int best = -1;
    float best_t = 0.0f;
    std::vector<float> t(reps);
    Ws w{ctx};
    static const int cands[] = {1, 2, 4, 8, 16};
    // remove any previous choice so each candidate runs as given
    for (size_t i = 0; i < ctx->tune.size(); ++i)
        if (ctx->tune[i].kind == 1 && ctx->tune[i].K == A->M && ctx->tune[i].prec == k) {
            ctx->tune.erase(ctx->tune.begin() + i);
            break;
        }
    for (int pw : cands) {
        if (ksg_lds_bytes(A->M, pw) > 160 * 1024) continue;
        tune_store(ctx, {1, A->M, k, 0, 0, pw, 0.0f});
        rc = corr_ksg_mi_pairs(ctx, A, B, pairs, n, k, 0, (float*)mi, nullptr, stream);  // warm-up
        for (int r = 0; r < reps && rc == CORR_OK; ++r) {
            rc = corr_ksg_mi_pairs(ctx, A, B, pairs, n, k, 0, (float*)mi, nullptr, stream);
            if (rc == CORR_OK) rc = corr_kernel_time_ms(ctx, TK_KSG, &t[r]);
        }
        if (rc) break;
        std::sort(t.begin(), t.end());
        if (best < 0 || t[reps / 2] < best_t) {
            best = pw;
            best_t = t[reps / 2];
        }
    }
    ctx->timing = saved_timing;
    if (rc) return rc;
    tune_store(ctx, {1, A->M, k, 0, 0, best, best_t});
    CORR_HIP(hipStreamSynchronize(s));
    if (best_pw) *best_pw = best;
    if (best_ms) *best_ms = best_t;
    return CORR_OK;
}

int corr_tune_save(corr_ctx* ctx, const char* path) {
    if (!ctx || !path) return fail(CORR_EINVAL, "null argument");
    FILE* f = fopen(path, "w");
    if (!f) return fail(CORR_EINVAL, std::string("cannot write ") + path);
    for (const corr_tune_rec& r : ctx->tune)
        fprintf(f,
                "{\"arch\": \"gfx950\", \"kind\": %d, \"K\": %d, \"prec\": %d, \"na\": %lld, \"nb\": %lld, "
                "\"cfg\": %d, \"ms\": %.6f}\n",
                r.kind, r.K, r.prec, (long long)r.na, (long long)r.nb, r.cfg, r.ms);
    fclose(f);
    return CORR_OK;
}

int corr_tune_load(corr_ctx* ctx, const char* path) {
    if (!ctx || !path) return fail(CORR_EINVAL, "null argument");
    FILE* f = fopen(path, "r");
    if (!f) return fail(CORR_EINVAL, std::string("cannot read ") + path);
    char line[512];
    int n = 0;
    while (fgets(line, sizeof line, f)) {
        corr_tune_rec r{};
        long long na = 0, nb = 0;
        if (sscanf(line,
                   " {\"arch\": \"gfx950\", \"kind\": %d, \"K\": %d, \"prec\": %d, \"na\": %lld, \"nb\": %lld, "
                   "\"cfg\": %d, \"ms\": %f}",
                   &r.kind, &r.K, &r.prec, &na, &nb, &r.cfg, &r.ms) != 7)
            continue;
        r.na = na;
        r.nb = nb;
        if (r.kind == 0 && !smallk_config_ok(r.prec, r.cfg, r.K)) continue;
        if (r.kind == 1 && (r.cfg < 1 || r.cfg > 16 || r.K < 2 || ksg_lds_bytes(r.K, r.cfg) > 160 * 1024)) continue;
        if (r.kind != 0 && r.kind != 1) continue;
        tune_store(ctx, r);
        ++n;
    }
    fclose(f);
    return CORR_OK;
}

int corr_standardize(corr_ctx* ctx, const corr_field* A, float* mu32, float* inv32, float* sigma,
                     corr_stream_t stream) {
    if (!ctx) return fail(CORR_EINVAL, "null context");
    int rc = check_field(A, "A");
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    if ((rc = ctx_use_stream(ctx, s))) return rc;
    Box box = whole_box(*A);
    const int64_t n = box.count();
    void* sb = nullptr;
    rc = ws_get(ctx, WS_STATS_A, sizeof(float) * 4 * (size_t)n, s, &sb);
    if (rc) return rc;
    Stats st = stats_view((float*)sb, n);
    rc = launch_stats(*A, box, true, st, s);
    if (rc) return rc;
    if (mu32) CORR_HIP(hipMemcpyAsync(mu32, st.mu32, sizeof(float) * n, hipMemcpyDeviceToDevice, s));
    if (inv32) CORR_HIP(hipMemcpyAsync(inv32, st.inv32, sizeof(float) * n, hipMemcpyDeviceToDevice, s));
    if (sigma) CORR_HIP(hipMemcpyAsync(sigma, st.sigma, sizeof(float) * n, hipMemcpyDeviceToDevice, s));
    return CORR_OK;
}

int corr_pearson_pairs(corr_ctx* ctx, const corr_field* A, const corr_field* B, const int32_t* pairs, int64_t n,
                       int prec, float* r_out, corr_stream_t stream) {
    if (!ctx) return fail(CORR_EINVAL, "null context");
    int rc = check_field(A, "A");
    if (rc) return rc;
    if ((rc = check_field(B, "B"))) return rc;
    if (A->M != B->M) return fail(CORR_EINVAL, "fields differ in M");
    if (n < 0) return fail(CORR_EINVAL, "n < 0");
    if (prec < CORR_PREC_F32 || prec > CORR_PREC_BF16X3) return fail(CORR_EUNSUPPORTED, "unknown precision");
    if (n == 0) return CORR_OK;
    if (!pairs || !r_out) return fail(CORR_EINVAL, "null pairs or output");
    hipStream_t s = (hipStream_t)stream;
    if ((rc = ctx_use_stream(ctx, s))) return rc;
    const int64_t ld = round_up(A->M, 16);
    const bool acc64 = stats_acc64(CORR_PEARSON, A->M);
    Box ba = whole_box(*A), bb = whole_box(*B);
    void *ah, *al, *bh, *bl;
    Ws w{ctx};
    rc = standardize_box(w, *A, ba, acc64, zfmt_for_prec(prec), ba.count(), ld, WS_STATS_A, WS_ZH_A, WS_ZL_A, s,
                         nullptr, &ah, &al);
    if (rc) return rc;
    if (same_field(*A, *B)) {
        bh = ah;
        bl = al;
    } else {
        rc = standardize_box(w, *B, bb, acc64, zfmt_for_prec(prec), bb.count(), ld, WS_STATS_B, WS_ZH_B, WS_ZL_B, s,
                             nullptr, &bh, &bl);
        if (rc) return rc;
    }
    timing_begin(ctx, TK_PAIRS, s);
    rc = launch_pearson_pairs(prec, ah, al, bh, bl, ld, pairs, n, r_out, ba, bb, 0, nullptr, s);
    timing_end(ctx, TK_PAIRS, s);
    return rc;
}

int corr_ksg_mi_pairs(corr_ctx* ctx, const corr_field* A, const corr_field* B, const int32_t* pairs, int64_t n,
                      int32_t k, uint32_t flags, float* mi_out, int32_t* counts_out, corr_stream_t stream) {
    if (!ctx) return fail(CORR_EINVAL, "null context");
    int rc = check_field(A, "A");
    if (rc) return rc;
    if ((rc = check_field(B, "B"))) return rc;
    if (A->M != B->M) return fail(CORR_EINVAL, "fields differ in M");
    if (n < 0) return fail(CORR_EINVAL, "n < 0");
    if (k < 1 || k > A->M - 1) return fail(CORR_EINVAL, "k must be in [1, M-1]");
    if (k > 31) return fail(CORR_EUNSUPPORTED, "k > 31");
    if (A->M > 2048) return fail(CORR_EUNSUPPORTED, "M > 2048");
    if (flags & ~CORR_KSG_RAW) return fail(CORR_EINVAL, "unknown flags");
    if (n == 0) return CORR_OK;
    if (!pairs || (!mi_out && !counts_out)) return fail(CORR_EINVAL, "null pairs or outputs");
    hipStream_t s = (hipStream_t)stream;
    if ((rc = ctx_use_stream(ctx, s))) return rc;
    const bool raw = flags & CORR_KSG_RAW;
    const int fmt = raw ? ZF_RAW : ZF_KSG;
    const int64_t ld = round_up(A->M, 4);
    Box ba = whole_box(*A), bb = whole_box(*B);
    Stats sa{}, sb{};
    void *za, *zb, *unused;
    Ws w{ctx};
    rc = standardize_box(w, *A, ba, true, fmt, ba.count(), ld, WS_STATS_A, WS_Z_A, WS_ZL_A, s, &sa, &za, &unused);
    if (rc) return rc;
    if (same_field(*A, *B)) {
        zb = za;
        sb = sa;
    } else {
        rc = standardize_box(w, *B, bb, true, fmt, bb.count(), ld, WS_STATS_B, WS_Z_B, WS_ZL_B, s, &sb, &zb,
                             &unused);
        if (rc) return rc;
    }
    void *sra, *srb;
    rc = sorted_rows(w, (const float*)za, ld, ba.count(), A->M, WS_SORT_A, s, &sra);
    if (rc) return rc;
    if (zb == za) {
        srb = sra;
    } else {
        rc = sorted_rows(w, (const float*)zb, ld, bb.count(), A->M, WS_SORT_B, s, &srb);
        if (rc) return rc;
    }
    KsgArgs a{};
    a.za = (const float*)za;
    a.zb = (const float*)zb;
    a.sa = (const float*)sra;
    a.sb = (const float*)srb;
    a.pw = tuned_ksg_pw(ctx, A->M, k);
    a.ld = ld;
    a.inv_a = raw ? nullptr : sa.inv32;
    a.inv_b = raw ? nullptr : sb.inv32;
    a.pairs = pairs;
    a.n = n;
    a.M = A->M;
    a.k = k;
    a.psi = ctx->psi;
    a.mi_out = mi_out;
    a.counts_out = counts_out;
    a.key = nullptr;
    a.work = ctx->keys + 8;
    a.ba = ba;
    a.bb = bb;
    a.whole_a = 1;
    a.whole_b = 1;
    a.same_field = 0;
    timing_begin(ctx, TK_KSG, s);
    rc = launch_ksg(a, ctx->num_cus, s);
    timing_end(ctx, TK_KSG, s);
    return rc;
}

}  // extern "C"

// A whole field standardised once (corr_prepare).
struct corr_prepared {
    int device = 0;
    int measure = 0, prec = 0, M = 0;
    int nx = 0, ny = 0, nz = 0;
    int64_t ld = 0;
    Stats st{};
    void* hi = nullptr;
    void* lo = nullptr;
    void* sorted = nullptr;
    std::vector<void*> bufs;
};

extern "C" {

void corr_prepared_destroy(corr_prepared* p) {
    if (!p) return;
    (void)hipSetDevice(p->device);
    (void)hipDeviceSynchronize();
    for (void* b : p->bufs) (void)hipFree(b);
    delete p;
}

int corr_prepare(corr_ctx* ctx, const corr_field* A, int measure, int prec, corr_prepared** out,
                 corr_stream_t stream) {
    if (!out) return fail(CORR_EINVAL, "corr_prepare: null out");
    *out = nullptr;
    if (!ctx) return fail(CORR_EINVAL, "null context");
    int rc = check_field(A, "A");
    if (rc) return rc;
    if (measure != CORR_PEARSON && measure != CORR_KSG) return fail(CORR_EINVAL, "unknown measure");
    if (measure == CORR_PEARSON && (prec < CORR_PREC_F32 || prec > CORR_PREC_BF16X3))
        return fail(CORR_EUNSUPPORTED, "unknown precision");
    if (measure == CORR_KSG && A->M > 2048) return fail(CORR_EUNSUPPORTED, "M > 2048");
    hipStream_t s = (hipStream_t)stream;
    if ((rc = ctx_use_stream(ctx, s))) return rc;
    corr_prepared* p = new (std::nothrow) corr_prepared();
    if (!p) return fail(CORR_ENOMEM, "corr_prepare: host allocation failed");
    p->device = ctx->device;
    p->measure = measure;
    p->prec = measure == CORR_PEARSON ? prec : 0;
    p->M = A->M;
    p->nx = A->nx;
    p->ny = A->ny;
    p->nz = A->nz;
    Ws w{ctx};
    w.owned = &p->bufs;
    const Box box = whole_box(*A);
    if (measure == CORR_PEARSON) {
        p->ld = round_up(A->M, 16);
        rc = standardize_box(w, *A, box, stats_acc64(CORR_PEARSON, A->M), zfmt_for_prec(prec), box.count(), p->ld,
                             WS_STATS_A, WS_ZH_A, WS_ZL_A, s, &p->st, &p->hi, &p->lo);
    } else {
        p->ld = round_up(A->M, 4);
        rc = standardize_box(w, *A, box, true, ZF_KSG, box.count(), p->ld, WS_STATS_A, WS_Z_A, WS_ZL_A, s, &p->st,
                             &p->hi, &p->lo);
        if (!rc) rc = sorted_rows(w, (const float*)p->hi, p->ld, box.count(), A->M, WS_SORT_A, s, &p->sorted);
    }
    if (rc) {
        corr_prepared_destroy(p);
        return rc;
    }
    *out = p;
    return CORR_OK;
}

static Box prepared_box(const corr_prepared* p) { return Box{0, 0, 0, p->nx, p->ny, p->nz, p->nx, p->ny}; }

int corr_pearson_pairs_prepared(corr_ctx* ctx, const corr_prepared* A, const corr_prepared* B,
                                const int32_t* pairs, int64_t n, float* r_out, corr_stream_t stream) {
    if (!ctx) return fail(CORR_EINVAL, "null context");
    if (!A || !B) return fail(CORR_EINVAL, "null prepared field");
    if (A->measure != CORR_PEARSON || B->measure != CORR_PEARSON)
        return fail(CORR_EINVAL, "fields not prepared for Pearson");
    if (A->M != B->M) return fail(CORR_EINVAL, "fields differ in M");
    if (A->prec != B->prec) return fail(CORR_EINVAL, "fields prepared with different precisions");
    if (n < 0) return fail(CORR_EINVAL, "n < 0");
    if (n == 0) return CORR_OK;
    if (!pairs || !r_out) return fail(CORR_EINVAL, "null pairs or output");
    hipStream_t s = (hipStream_t)stream;
    if (int rc_ = ctx_use_stream(ctx, s)) return rc_;
    timing_begin(ctx, TK_PAIRS, s);
    int rc = launch_pearson_pairs(A->prec, A->hi, A->lo, B->hi, B->lo, A->ld, pairs, n, r_out, prepared_box(A),
                                  prepared_box(B), 0, nullptr, s);
    timing_end(ctx, TK_PAIRS, s);
    return rc;
}

int corr_ksg_mi_pairs_prepared(corr_ctx* ctx, const corr_prepared* A, const corr_prepared* B,
                               const int32_t* pairs, int64_t n, int32_t k, float* mi_out, int32_t* counts_out,
                               corr_stream_t stream) {
    if (!ctx) return fail(CORR_EINVAL, "null context");
    if (!A || !B) return fail(CORR_EINVAL, "null prepared field");
    if (A->measure != CORR_KSG || B->measure != CORR_KSG) return fail(CORR_EINVAL, "fields not prepared for KSG");
    if (A->M != B->M) return fail(CORR_EINVAL, "fields differ in M");
    if (n < 0) return fail(CORR_EINVAL, "n < 0");
    if (k < 1 || k > A->M - 1) return fail(CORR_EINVAL, "k must be in [1, M-1]");
    if (k > 31) return fail(CORR_EUNSUPPORTED, "k > 31");
    if (n == 0) return CORR_OK;
    if (!pairs || (!mi_out && !counts_out)) return fail(CORR_EINVAL, "null pairs or outputs");
    hipStream_t s = (hipStream_t)stream;
    if (int rc_ = ctx_use_stream(ctx, s)) return rc_;
    KsgArgs a{};
    a.za = (const float*)A->hi;
    a.zb = (const float*)B->hi;
    a.sa = (const float*)A->sorted;
    a.sb = (const float*)B->sorted;
    a.pw = tuned_ksg_pw(ctx, A->M, k);
    a.ld = A->ld;
    a.inv_a = A->st.inv32;
    a.inv_b = B->st.inv32;
    a.pairs = pairs;
    a.n = n;
    a.M = A->M;
    a.k = k;
    a.psi = ctx->psi;
    a.mi_out = mi_out;
    a.counts_out = counts_out;
    a.key = nullptr;
    a.work = ctx->keys + 8;
    a.ba = prepared_box(A);
    a.bb = prepared_box(B);
    a.whole_a = 1;
    a.whole_b = 1;
    a.same_field = 0;
    timing_begin(ctx, TK_KSG, s);
    int rc = launch_ksg(a, ctx->num_cus, s);
    timing_end(ctx, TK_KSG, s);
    return rc;
}

int corr_box_pairs_max(corr_ctx* ctx, const corr_prepared* A, const corr_prepared* B, const corr_region* boxes_a,
                       const corr_region* boxes_b, int32_t n, corr_max* out, corr_stream_t stream) {
    if (!ctx) return fail(CORR_EINVAL, "null context");
    if (!A || !B) return fail(CORR_EINVAL, "null prepared field");
    if (n < 0) return fail(CORR_EINVAL, "n < 0");
    if (n == 0) return CORR_OK;
    if (!boxes_a || !boxes_b || !out) return fail(CORR_EINVAL, "null boxes or output");
    if (A->measure != CORR_PEARSON || B->measure != CORR_PEARSON || A->prec != CORR_PREC_F32 ||
        B->prec != CORR_PREC_F32)
        return fail(CORR_EUNSUPPORTED, "box maxima need fields prepared for Pearson with CORR_PREC_F32");
    if (A->M != B->M) return fail(CORR_EINVAL, "fields differ in M");
    std::vector<Box> hb(2 * (size_t)n);
    int64_t max_pts = 1;
    for (int32_t t = 0; t < n; ++t) {
        const corr_region* rs[2] = {&boxes_a[t], &boxes_b[t]};
        const corr_prepared* fs[2] = {A, B};
        for (int q = 0; q < 2; ++q) {
            const corr_region& r = *rs[q];
            const corr_prepared& f = *fs[q];
            if (r.dx < 1 || r.dy < 1 || r.dz < 1 || r.x0 < 0 || r.y0 < 0 || r.z0 < 0 || r.x0 + r.dx > f.nx ||
                r.y0 + r.dy > f.ny || r.z0 + r.dz > f.nz)
                return fail(CORR_EINVAL, "box " + std::to_string(t) + " empty or outside the grid");
            const int64_t c = (int64_t)r.dx * r.dy * r.dz;
            if (c > 4096) return fail(CORR_EUNSUPPORTED, "box maxima: a box holds more than 4096 points");
            max_pts = std::max(max_pts, c);
            hb[(size_t)q * n + t] = Box{r.x0, r.y0, r.z0, r.dx, r.dy, r.dz, f.nx, f.ny};
        }
    }
    hipStream_t s = (hipStream_t)stream;
    int rc = ctx_use_stream(ctx, s);
    if (rc) return rc;
    void *dbox = nullptr, *dkeys = nullptr;
    if ((rc = ws_get(ctx, WS_BOXES, sizeof(Box) * hb.size(), s, &dbox))) return rc;
    if ((rc = ws_get(ctx, WS_BOX_KEYS, sizeof(unsigned long long) * (size_t)n, s, &dkeys))) return rc;
    CORR_HIP(hipMemcpyAsync(dbox, hb.data(), sizeof(Box) * hb.size(), hipMemcpyHostToDevice, s));
    const bool same = A == B;
    timing_begin(ctx, TK_PAIRS, s);
    rc = launch_box_pairs_max((const float*)A->hi, (const float*)B->hi, A->ld, (const Box*)dbox, n, same ? 1 : 0,
                              (int)max_pts, (unsigned long long*)dkeys, ctx->num_cus, s);
    timing_end(ctx, TK_PAIRS, s);
    if (rc) return rc;
    std::vector<unsigned long long> keys((size_t)n);
    CORR_HIP(hipMemcpyAsync(keys.data(), dkeys, sizeof(unsigned long long) * (size_t)n, hipMemcpyDeviceToHost, s));
    CORR_HIP(hipStreamSynchronize(s));
    for (int32_t t = 0; t < n; ++t) {
        const Box& ba = hb[t];
        const Box& bb = hb[(size_t)n + t];
        decode_key(keys[t], ba, bb, true, &out[t]);
        out[t].n_evaluated = ba.count() * bb.count() - (same ? overlap_count(ba, bb) : 0);
    }
    return CORR_OK;
}

}  // extern "C"

// Region maximum (exhaustive Pearson, or Pearson / KSG over a sample list)
// with its workspaces taken from `w`.
static int region_max_impl(Ws& w, const corr_field* A, const corr_region* ra, const corr_field* B,
                           const corr_region* rb, int measure, int prec, int32_t k, const int32_t* sample_pairs,
                           int64_t n_samples, corr_max* out, hipStream_t s);

// Exhaustive maximum over 2^31 or more point pairs (Sec. 3: the maximum over
// every pA in A and pB in B): region A is cut into consecutive pieces of its
// local x-fastest order -- z slabs, or y rows of one z layer, or x runs of
// one row when a layer or a row alone is too large -- each small enough for
// the 31-bit pair index, and each piece runs as an ordinary exhaustive call.
// Pieces cover increasing ranges of A's local index, so keeping the first
// piece among equal maxima keeps the smallest local pair index, the same
// tie-break as one call; n_evaluated adds up.
static int region_max_split(Ws& w, const corr_field* A, const corr_region* ra, const corr_field* B,
                            const corr_region* rb, int measure, int prec, int32_t k, corr_max* out,
                            hipStream_t s) {
    const int64_t nb = (int64_t)rb->dx * rb->dy * rb->dz;
    const int64_t cap = ((int64_t(1) << 31) - 1) / nb;  // points of A per piece (>= 1: nb < 2^31)
    const int64_t layer = (int64_t)ra->dx * ra->dy;
    corr_max best{};
    best.pa = best.pb = -1;
    bool have = false;
    int64_t evaluated = 0;
    auto piece = [&](const corr_region& sub) -> int {
        corr_max part{};
        const int rc = region_max_impl(w, A, &sub, B, rb, measure, prec, k, nullptr, 0, &part, s);
        if (rc) return rc;
        evaluated += part.n_evaluated;
        if (part.pa >= 0 && (!have || part.value > best.value)) {
            best = part;
            have = true;
        }
        return CORR_OK;
    };
    int rc = CORR_OK;
    if (layer <= cap) {
        const int32_t tz = (int32_t)(cap / layer);
        for (int32_t z = 0; z < ra->dz && !rc; z += tz)
            rc = piece(corr_region{ra->x0, ra->y0, ra->z0 + z, ra->dx, ra->dy, std::min(tz, ra->dz - z)});
    } else if ((int64_t)ra->dx <= cap) {
        const int32_t ty = (int32_t)(cap / ra->dx);
        for (int32_t z = 0; z < ra->dz && !rc; ++z)
            for (int32_t y = 0; y < ra->dy && !rc; y += ty)
                rc = piece(corr_region{ra->x0, ra->y0 + y, ra->z0 + z, ra->dx, std::min(ty, ra->dy - y), 1});
    } else {
        const int32_t tx = (int32_t)cap;
        for (int32_t z = 0; z < ra->dz && !rc; ++z)
            for (int32_t y = 0; y < ra->dy && !rc; ++y)
                for (int32_t x = 0; x < ra->dx && !rc; x += tx)
                    rc = piece(corr_region{ra->x0 + x, ra->y0 + y, ra->z0 + z, std::min(tx, ra->dx - x), 1, 1});
    }
    if (rc) return rc;
    *out = best;
    out->n_evaluated = evaluated;
    return CORR_OK;
}

static int region_max_impl(Ws& w, const corr_field* A, const corr_region* ra, const corr_field* B,
                           const corr_region* rb, int measure, int prec, int32_t k, const int32_t* sample_pairs,
                           int64_t n_samples, corr_max* out, hipStream_t s) {
    corr_ctx* ctx = w.ctx;
    if (!ctx) return fail(CORR_EINVAL, "null context");
    if (!out) return fail(CORR_EINVAL, "null output");
    int rc = check_field(A, "A");
    if (rc) return rc;
    if ((rc = check_field(B, "B"))) return rc;
    if (A->M != B->M) return fail(CORR_EINVAL, "fields differ in M");
    if ((rc = check_region(ra, *A, "ra"))) return rc;
    if ((rc = check_region(rb, *B, "rb"))) return rc;
    if (measure != CORR_PEARSON && measure != CORR_KSG) return fail(CORR_EINVAL, "unknown measure");
    if (measure == CORR_PEARSON && (prec < CORR_PREC_F32 || prec > CORR_PREC_BF16X3))
        return fail(CORR_EUNSUPPORTED, "unknown precision");
    if (measure == CORR_KSG) {
        if (k < 1 || k > A->M - 1) return fail(CORR_EINVAL, "k must be in [1, M-1]");
        if (k > 31) return fail(CORR_EUNSUPPORTED, "k > 31");
        if (A->M > 2048) return fail(CORR_EUNSUPPORTED, "M > 2048");
    }
    if (n_samples < 0) return fail(CORR_EINVAL, "n_samples < 0");
    if (sample_pairs == nullptr && n_samples != 0)
        return fail(CORR_EINVAL, "n_samples given without sample_pairs");
    Box ba = region_box(*ra, *A), bb = region_box(*rb, *B);
    const int64_t na = ba.count(), nb = bb.count();
    if (na * nb >= (int64_t(1) << 31)) {
        // the result key carries a 31-bit local pair index: an exhaustive
        // call over more pairs runs as consecutive pieces of region A
        if (sample_pairs != nullptr) return fail(CORR_EUNSUPPORTED, "region pair has 2^31 or more point pairs");
        return region_max_split(w, A, ra, B, rb, measure, prec, k, out, s);
    }
    if ((rc = ctx_use_stream(ctx, s))) return rc;
    const bool sf = same_field(*A, *B);
    memset(out, 0, sizeof(*out));
    out->pa = out->pb = -1;
    rc = launch_fill_u64(ctx->keys, 2, 0ull, s);
    if (rc) return rc;
    const bool exhaustive = sample_pairs == nullptr;
    if (!exhaustive && n_samples == 0) return CORR_OK;

    if (measure == CORR_PEARSON) {
        const bool acc64 = stats_acc64(CORR_PEARSON, A->M);
        const int fmt = zfmt_for_prec(prec);
        void *ah, *al, *bh, *bl;
        if (exhaustive) return pearson_exhaustive(w, *A, ba, *B, bb, sf, prec, -1, out, s);
        const int64_t ld = round_up(A->M, 16);
        rc = standardize_box(w, *A, ba, acc64, fmt, na, ld, WS_STATS_A, WS_ZH_A, WS_ZL_A, s, nullptr, &ah, &al);
        if (rc) return rc;
        rc = standardize_box(w, *B, bb, acc64, fmt, nb, ld, WS_STATS_B, WS_ZH_B, WS_ZL_B, s, nullptr, &bh, &bl);
        if (rc) return rc;
        timing_begin(ctx, TK_PAIRS, s);
        rc = launch_pearson_pairs(prec, ah, al, bh, bl, ld, sample_pairs, n_samples, nullptr, ba, bb, sf ? 1 : 0,
                                  ctx->keys, s);
        timing_end(ctx, TK_PAIRS, s);
        if (rc) return rc;
        unsigned long long k0, k1;
        if ((rc = read_keys(ctx, s, &k0, &k1))) return rc;
        decode_key(k0, ba, bb, true, out);
        out->n_evaluated = (int64_t)k1;
        return CORR_OK;
    }

    // KSG
    const int64_t ld = round_up(A->M, 4);
    Stats sa{}, sb{};
    void *za, *zb, *unused;
    rc = standardize_box(w, *A, ba, true, ZF_KSG, na, ld, WS_STATS_A, WS_Z_A, WS_ZL_A, s, &sa, &za, &unused);
    if (rc) return rc;
    rc = standardize_box(w, *B, bb, true, ZF_KSG, nb, ld, WS_STATS_B, WS_Z_B, WS_ZL_B, s, &sb, &zb, &unused);
    if (rc) return rc;
    void *sra, *srb;
    rc = sorted_rows(w, (const float*)za, ld, na, A->M, WS_SORT_A, s, &sra);
    if (rc) return rc;
    rc = sorted_rows(w, (const float*)zb, ld, nb, A->M, WS_SORT_B, s, &srb);
    if (rc) return rc;
    KsgArgs a{};
    a.za = (const float*)za;
    a.zb = (const float*)zb;
    a.sa = (const float*)sra;
    a.sb = (const float*)srb;
    a.pw = tuned_ksg_pw(ctx, A->M, k);
    a.ld = ld;
    a.inv_a = sa.inv32;
    a.inv_b = sb.inv32;
    a.pairs = sample_pairs;
    a.n = n_samples;
    a.M = A->M;
    a.k = k;
    a.psi = ctx->psi;
    a.key = ctx->keys;
    a.work = ctx->keys + 8;
    a.ba = ba;
    a.bb = bb;
    a.whole_a = (ba.count() == (int64_t)A->nx * A->ny * A->nz) ? 1 : 0;
    a.whole_b = (bb.count() == (int64_t)B->nx * B->ny * B->nz) ? 1 : 0;
    a.same_field = sf ? 1 : 0;
    timing_begin(ctx, TK_KSG, s);
    rc = launch_ksg(a, ctx->num_cus, s);
    timing_end(ctx, TK_KSG, s);
    if (rc) return rc;
    unsigned long long k0, k1;
    if ((rc = read_keys(ctx, s, &k0, &k1))) return rc;
    decode_key(k0, ba, bb, false, out);
    out->n_evaluated = (int64_t)k1;
    return CORR_OK;
}

extern "C" {

int corr_region_max(corr_ctx* ctx, const corr_field* A, const corr_region* ra, const corr_field* B,
                    const corr_region* rb, int measure, int prec, int32_t k, const int32_t* sample_pairs,
                    int64_t n_samples, corr_max* out, corr_stream_t stream) {
    Ws w{ctx};
    return region_max_impl(w, A, ra, B, rb, measure, prec, k, sample_pairs, n_samples, out, (hipStream_t)stream);
}

int corr_region_max_noalloc(corr_ctx* ctx, const corr_field* A, const corr_region* ra, const corr_field* B,
                            const corr_region* rb, int measure, int prec, int32_t k, const int32_t* sample_pairs,
                            int64_t n_samples, corr_max* out, corr_stream_t stream) {
    if (!ctx) return fail(CORR_EINVAL, "null context");
    if (!ctx->scratch) return fail(CORR_ESTATE, "corr_region_max_noalloc: the context has no fixed scratch");
    Ws w{ctx, (char*)ctx->scratch, CORR_SCRATCH_BYTES};
    return region_max_impl(w, A, ra, B, rb, measure, prec, k, sample_pairs, n_samples, out, (hipStream_t)stream);
}

int corr_block_means(corr_ctx* ctx, const corr_field* A, int f, int out_dtype, void* out, int64_t out_stride,
                     corr_stream_t stream) {
    if (!ctx) return fail(CORR_EINVAL, "null context");
    int rc = check_field(A, "A");
    if (rc) return rc;
    if (f < 1 || f > 64 || (f & (f - 1)) != 0) return fail(CORR_EINVAL, "f must be a power of two in [1, 64]");
    if (out_dtype != CORR_F32 && out_dtype != CORR_F16) return fail(CORR_EUNSUPPORTED, "unsupported output dtype");
    if (!out) return fail(CORR_EINVAL, "null output");
    const int64_t nout = (int64_t)((A->nx + f - 1) / f) * ((A->ny + f - 1) / f) * ((A->nz + f - 1) / f);
    if (out_stride != 0 && out_stride < nout) return fail(CORR_EINVAL, "out_stride smaller than the level's grid");
    hipStream_t s = (hipStream_t)stream;
    if ((rc = ctx_use_stream(ctx, s))) return rc;
    timing_begin(ctx, TK_AGG, s);
    rc = launch_block_means(*A, f, out_dtype, out, out_stride, s);
    timing_end(ctx, TK_AGG, s);
    return rc;
}

// ---- sampling (Sec. 3.1) and strategy (Sec. 5) ------------------------------
static int check_sampling_args(const corr_field* A, const corr_field* B, const corr_region* regions,
                               int32_t n_regions, const int32_t* region_pairs, int32_t n_pairs, int sampler,
                               int32_t n_samples) {
    int rc = check_field(A, "A");
    if (rc) return rc;
    if ((rc = check_field(B, "B"))) return rc;
    if (A->M != B->M) return fail(CORR_EINVAL, "fields differ in M");
    if (n_pairs < 0 || n_samples < 0) return fail(CORR_EINVAL, "negative pair or sample count");
    if ((int64_t)n_pairs * n_samples >= (int64_t(1) << 31)) return fail(CORR_EINVAL, "too many samples");
    if (sampler < CORR_SAMPLE_UNIFORM || sampler > CORR_SAMPLE_PLASTIC) return fail(CORR_EUNSUPPORTED, "sampler");
    if (n_pairs > 0 && (!regions || !region_pairs || n_regions < 1)) return fail(CORR_EINVAL, "null regions");
    for (int32_t p = 0; p < n_pairs; ++p) {
        const int32_t ia = region_pairs[2 * p], ib = region_pairs[2 * p + 1];
        if (ia < 0 || ia >= n_regions || ib < 0 || ib >= n_regions) return fail(CORR_EINVAL, "region index");
        if ((rc = check_region(&regions[ia], *A, "region of A"))) return rc;
        if ((rc = check_region(&regions[ib], *B, "region of B"))) return rc;
    }
    return CORR_OK;
}

static int stage_samples(corr_ctx* ctx, const corr_field* A, const corr_field* B, const corr_region* regions,
                         const int32_t* region_pairs, int32_t n_pairs, int sampler, int32_t n_samples, uint64_t seed,
                         int32_t* out, hipStream_t s) {
    const size_t bb = sample_boxes_bytes(n_pairs);
    void* dbox = nullptr;
    int rc = ctx_use_stream(ctx, s);
    if (rc) return rc;
    rc = ws_get(ctx, WS_SBOXES, bb + sizeof(corr_max) * (size_t)n_pairs, s, &dbox);
    if (rc) return rc;
    std::vector<unsigned char> hbox(bb);
    fill_sample_boxes(hbox.data(), regions, region_pairs, n_pairs, *A, *B);
    CORR_HIP(hipMemcpyAsync(dbox, hbox.data(), bb, hipMemcpyHostToDevice, s));
    rc = launch_sample_pairs(dbox, n_pairs, n_samples, sampler, seed, out, s);
    if (rc) return rc;
    CORR_HIP(hipStreamSynchronize(s));  // hbox is released on return
    return CORR_OK;
}

int corr_sample_pairs(corr_ctx* ctx, const corr_field* A, const corr_field* B, const corr_region* regions,
                      int32_t n_regions, const int32_t* region_pairs, int32_t n_pairs, int sampler,
                      int32_t n_samples, uint64_t seed, int32_t* out, corr_stream_t stream) {
    if (!ctx) return fail(CORR_EINVAL, "null context");
    int rc = check_sampling_args(A, B, regions, n_regions, region_pairs, n_pairs, sampler, n_samples);
    if (rc) return rc;
    if ((int64_t)n_pairs * n_samples == 0) return CORR_OK;
    if (!out) return fail(CORR_EINVAL, "null output");
    return stage_samples(ctx, A, B, regions, region_pairs, n_pairs, sampler, n_samples, seed, out,
                         (hipStream_t)stream);
}

int corr_sampled_max(corr_ctx* ctx, const corr_field* A, const corr_field* B, const corr_region* regions,
                     int32_t n_regions, const int32_t* region_pairs, int32_t n_pairs, int measure, int prec,
                     int32_t k, int sampler, int32_t n_samples, uint64_t seed, corr_max* out,
                     corr_stream_t stream) {
    if (!ctx) return fail(CORR_EINVAL, "null context");
    int rc = check_sampling_args(A, B, regions, n_regions, region_pairs, n_pairs, sampler, n_samples);
    if (rc) return rc;
    if (measure != CORR_PEARSON && measure != CORR_KSG) return fail(CORR_EINVAL, "unknown measure");
    if (measure == CORR_KSG && (k < 1 || k > A->M - 1)) return fail(CORR_EINVAL, "k outside [1, M-1]");
    if (n_pairs == 0) return CORR_OK;
    if (!out) return fail(CORR_EINVAL, "null output");
    hipStream_t s = (hipStream_t)stream;
    if ((rc = ctx_use_stream(ctx, s))) return rc;
    const int64_t n = (int64_t)n_pairs * n_samples;
    void *dpairs = nullptr, *dvals = nullptr, *dbox = nullptr;
    if ((rc = ws_get(ctx, WS_SAMPLES, sizeof(int32_t) * 2 * (size_t)(n > 0 ? n : 1), s, &dpairs))) return rc;
    if ((rc = ws_get(ctx, WS_SVALUES, sizeof(float) * (size_t)(n > 0 ? n : 1), s, &dvals))) return rc;
    if (n > 0) {
        rc = stage_samples(ctx, A, B, regions, region_pairs, n_pairs, sampler, n_samples, seed, (int32_t*)dpairs, s);
        if (rc) return rc;
        if (measure == CORR_PEARSON)
            rc = corr_pearson_pairs(ctx, A, B, (const int32_t*)dpairs, n, prec, (float*)dvals, stream);
        else
            rc = corr_ksg_mi_pairs(ctx, A, B, (const int32_t*)dpairs, n, k, 0, (float*)dvals, nullptr, stream);
        if (rc) return rc;
    }
    if ((rc = ws_get(ctx, WS_SBOXES, sample_boxes_bytes(n_pairs) + sizeof(corr_max) * (size_t)n_pairs, s, &dbox)))
        return rc;
    corr_max* dres = (corr_max*)((unsigned char*)dbox + sample_boxes_bytes(n_pairs));
    rc = launch_segment_max((const float*)dvals, (const int32_t*)dpairs, n_pairs, n_samples,
                            measure == CORR_PEARSON ? 1 : 0, same_field(*A, *B) ? 1 : 0, dres, s);
    if (rc) return rc;
    CORR_HIP(hipMemcpyAsync(out, dres, sizeof(corr_max) * (size_t)n_pairs, hipMemcpyDeviceToHost, s));
    CORR_HIP(hipStreamSynchronize(s));
    return CORR_OK;
}

int corr_choose_strategy(int64_t na, int64_t nb, double pairs_per_s, double budget_s, int32_t* strategy) {
    if (!strategy) return fail(CORR_EINVAL, "null output");
    if (na < 1 || nb < 1 || !(pairs_per_s > 0.0) || !(budget_s >= 0.0))
        return fail(CORR_EINVAL, "bad brick sizes, rate or budget");
    const int64_t bos_min = 16 * 16 * 16;
    if (na >= bos_min && nb >= bos_min)
        *strategy = CORR_STRATEGY_BOS;
    else if ((double)na * (double)nb <= budget_s * pairs_per_s)
        *strategy = CORR_STRATEGY_EXHAUSTIVE;
    else
        *strategy = CORR_STRATEGY_RANDOM;
    return CORR_OK;
}

// ---- sub-brick maxima (one refinement level of a brick pair) ---------------
static int split_box(const corr_region& r, const int32_t* splits, const corr_field& f, std::vector<Box>& out) {
    const int32_t o[3] = {r.x0, r.y0, r.z0}, d[3] = {r.dx, r.dy, r.dz};
    std::vector<int32_t> st[3], len[3];
    for (int a = 0; a < 3; ++a) {
        if (splits[a] < 1 || splits[a] > d[a]) return fail(CORR_EINVAL, "split count outside [1, axis extent]");
        int32_t start = o[a];
        for (int i = 0; i < splits[a]; ++i) {
            const int32_t n = d[a] / splits[a] + (i < d[a] % splits[a] ? 1 : 0);
            st[a].push_back(start);
            len[a].push_back(n);
            start += n;
        }
    }
    out.clear();
    for (size_t z = 0; z < st[2].size(); ++z)
        for (size_t y = 0; y < st[1].size(); ++y)
            for (size_t x = 0; x < st[0].size(); ++x)
                out.push_back(Box{st[0][x], st[1][y], st[2][z], len[0][x], len[1][y], len[2][z], f.nx, f.ny});
    return CORR_OK;
}

int corr_region_submax(corr_ctx* ctx, const corr_field* A, const corr_region* ra, const int32_t* splits_a,
                       const corr_field* B, const corr_region* rb, const int32_t* splits_b, int prec,
                       corr_max* out, corr_stream_t stream) {
    if (!ctx) return fail(CORR_EINVAL, "null context");
    int rc = check_field(A, "A");
    if (rc) return rc;
    if ((rc = check_field(B, "B"))) return rc;
    if (A->M != B->M) return fail(CORR_EINVAL, "fields differ in M");
    if ((rc = check_region(ra, *A, "ra"))) return rc;
    if ((rc = check_region(rb, *B, "rb"))) return rc;
    if (!splits_a || !splits_b || !out) return fail(CORR_EINVAL, "null splits or output");
    if (prec < CORR_PREC_F32 || prec > CORR_PREC_BF16X3) return fail(CORR_EUNSUPPORTED, "unknown precision");
    std::vector<Box> sa, sb;
    if ((rc = split_box(*ra, splits_a, *A, sa))) return rc;
    if ((rc = split_box(*rb, splits_b, *B, sb))) return rc;
    if (sa[0].count() * sb[0].count() >= (int64_t(1) << 31))  // the first sub-bricks are the largest
        return fail(CORR_EUNSUPPORTED, "a sub-brick pair has 2^31 or more point pairs");
    hipStream_t s = (hipStream_t)stream;
    if ((rc = ctx_use_stream(ctx, s))) return rc;
    const bool sf = same_field(*A, *B);
    const bool acc64 = stats_acc64(CORR_PEARSON, A->M);
    const int fmt = zfmt_for_prec(prec);
    const bool small = A->M <= 128;
    int64_t K, row_pad, col_pad;
    int cfg = -1;
    if (small) {
        K = smallk_pad_K(A->M);
        cfg = default_smallk_cfg(prec, (int)K);
        row_pad = smallk_row_pad(cfg);
        col_pad = smallk_col_pad(cfg);
    } else {
        K = round_up(A->M, gemm_k_pad(prec));
        row_pad = gemm_row_pad();
        col_pad = gemm_col_pad();
    }
    const size_t es = prec == CORR_PREC_F32 ? 4 : 2;
    const bool split = prec_split(prec);
    // rows of every sub-brick, each block padded for the contraction
    auto layout = [&](const std::vector<Box>& boxes, int64_t pad, std::vector<int64_t>& off, int64_t& total,
                      int64_t& largest) {
        off.clear();
        total = 0;
        largest = 0;
        for (const Box& b : boxes) {
            off.push_back(total);
            total += round_up(b.count(), pad);
            largest = std::max(largest, b.count());
        }
    };
    std::vector<int64_t> offa, offb;
    int64_t tot_a, tot_b, big_a, big_b;
    layout(sa, row_pad, offa, tot_a, big_a);
    layout(sb, col_pad, offb, tot_b, big_b);
    void *ah = nullptr, *al = nullptr, *bh = nullptr, *bl = nullptr, *sta = nullptr, *keys = nullptr;
    if ((rc = ws_get(ctx, WS_SUB_AH, es * (size_t)(tot_a * K), s, &ah))) return rc;
    if ((rc = ws_get(ctx, WS_SUB_BH, es * (size_t)(tot_b * K), s, &bh))) return rc;
    if (split) {
        if ((rc = ws_get(ctx, WS_SUB_AL, es * (size_t)(tot_a * K), s, &al))) return rc;
        if ((rc = ws_get(ctx, WS_SUB_BL, es * (size_t)(tot_b * K), s, &bl))) return rc;
    }
    if ((rc = ws_get(ctx, WS_STATS_A, sizeof(float) * 4 * (size_t)std::max(big_a, big_b), s, &sta))) return rc;
    const size_t n_out = sa.size() * sb.size();
    if ((rc = ws_get(ctx, WS_SUB_KEYS, sizeof(unsigned long long) * 2 * n_out, s, &keys))) return rc;
    if ((rc = launch_fill_u64((unsigned long long*)keys, 2 * (int64_t)n_out, 0ull, s))) return rc;
    auto stage = [&](const corr_field& f, const std::vector<Box>& boxes, const std::vector<int64_t>& off, int64_t pad,
                     void* hi, void* lo) {
        for (size_t i = 0; i < boxes.size(); ++i) {
            const int64_t n = boxes[i].count();
            Stats st = stats_view((float*)sta, n);
            int r = launch_stats(f, boxes[i], acc64, st, s);
            if (r) return r;
            unsigned char* h = (unsigned char*)hi + es * (size_t)(off[i] * K);
            unsigned char* l = lo ? (unsigned char*)lo + es * (size_t)(off[i] * K) : nullptr;
            r = launch_transpose(f, boxes[i], st, fmt, h, l, round_up(n, pad), K, s);
            if (r) return r;
        }
        return (int)CORR_OK;
    };
    if ((rc = stage(*A, sa, offa, row_pad, ah, al))) return rc;
    if ((rc = stage(*B, sb, offb, col_pad, bh, bl))) return rc;
    // self columns of overlapping sub-brick pairs (one field only)
    void* selfbuf = nullptr;
    if (sf && boxes_overlap(region_box(*ra, *A), region_box(*rb, *B)))
        if ((rc = ws_get(ctx, WS_MISC, sizeof(int32_t) * (size_t)big_a, s, &selfbuf))) return rc;
    for (size_t i = 0; i < sa.size(); ++i) {
        for (size_t j = 0; j < sb.size(); ++j) {
            const int64_t na = sa[i].count(), nb = sb[j].count();
            GemmArgs g{};
            g.prec = prec;
            g.a_hi = (unsigned char*)ah + es * (size_t)(offa[i] * K);
            g.a_lo = al ? (unsigned char*)al + es * (size_t)(offa[i] * K) : nullptr;
            g.b_hi = (unsigned char*)bh + es * (size_t)(offb[j] * K);
            g.b_lo = bl ? (unsigned char*)bl + es * (size_t)(offb[j] * K) : nullptr;
            g.K = K;
            g.na = na;
            g.nb = nb;
            g.na_pad = round_up(na, row_pad);
            g.nb_pad = round_up(nb, col_pad);
            g.self_col = nullptr;
            if (selfbuf && boxes_overlap(sa[i], sb[j])) {
                // the buffer is reused by the next overlapping pair only after
                // this pair's contraction (stream order)
                self_col_kernel<<<dim3((unsigned)((na + 255) / 256)), 256, 0, s>>>(sa[i], sb[j], (int32_t*)selfbuf);
                CORR_LAUNCH_CHECK();
                g.self_col = (const int32_t*)selfbuf;
            }
            g.key = (unsigned long long*)keys + 2 * (i * sb.size() + j);
            rc = small ? launch_gemm_smallk(g, cfg, ctx->num_cus, s) : launch_gemm_max(g, ctx->num_cus, s);
            if (rc) return rc;
        }
    }
    std::vector<unsigned long long> hk(2 * n_out);
    CORR_HIP(hipMemcpyAsync(hk.data(), keys, sizeof(unsigned long long) * hk.size(), hipMemcpyDeviceToHost, s));
    CORR_HIP(hipStreamSynchronize(s));
    for (size_t i = 0; i < sa.size(); ++i)
        for (size_t j = 0; j < sb.size(); ++j) {
            corr_max& o = out[i * sb.size() + j];
            decode_key(hk[2 * (i * sb.size() + j)], sa[i], sb[j], true, &o);
            o.n_evaluated = sa[i].count() * sb[j].count() - (sf ? overlap_count(sa[i], sb[j]) : 0);
        }
    return CORR_OK;
}

}  // extern "C"
