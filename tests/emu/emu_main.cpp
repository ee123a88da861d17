// Host-emulation driver of the batched BOS entry points -- TEST
// INFRASTRUCTURE ONLY. Reads a field, regions and region pairs, runs
// bos_create / bos_sample_step / bos_results / bos_history of the library's
// own BOS source (rewritten by transform.py, compiled for the host with the
// primitives of hip/hip_runtime.h) and writes every pair's history. The
// statistics, standardised rows and sorted rows that the library computes on
// the GPU are formed here with the same arithmetic.
#include "hip/hip_runtime.h"
#include <algorithm>
#include <cstdio>
#include <string>
#include <vector>
#include "bos.h"
#include "common.h"

thread_local dim3 threadIdx, blockIdx;
dim3 blockDim, gridDim;
void* emu_dyn_lds = nullptr;
std::barrier<>* emu_block_bar = nullptr;
std::barrier<>* emu_wave_bar[16] = {};
unsigned long long emu_xchg[16][64];
hipStream_t emu_capturing = nullptr;
EmuGraph* emu_graph = nullptr;
long emu_launches = 0;

void emu_run(dim3 g, dim3 b, size_t lds, std::function<void()> body) {
    ++emu_launches;
    blockDim = b;
    gridDim = g;
    for (unsigned bx = 0; bx < g.x; ++bx) {
        void* mem = std::malloc(lds ? lds : 1);
        std::memset(mem, 0xcd, lds ? lds : 1);
        emu_dyn_lds = mem;
        std::barrier<> bar(b.x);
        emu_block_bar = &bar;
        std::vector<std::unique_ptr<std::barrier<>>> wb;
        for (unsigned w = 0; w < (b.x + 63) / 64; ++w) {
            wb.emplace_back(new std::barrier<>(std::min(64u, b.x - 64 * w)));
            emu_wave_bar[w] = wb.back().get();
        }
        std::vector<std::thread> th;
        for (unsigned t = 0; t < b.x; ++t)
            th.emplace_back([&, t, bx]() {
                threadIdx = dim3(t);
                blockIdx = dim3(bx);
                body();
            });
        for (auto& t : th) t.join();
        std::free(mem);
    }
}

namespace corr {
static std::string g_err;
void set_error(const std::string& m) { g_err = m; }
int fail(int status, const std::string& m) {
    g_err = m;
    std::fprintf(stderr, "fail %d: %s\n", status, m.c_str());
    return status;
}
int ksg_p2(int M) {
    int p = 1;
    while (p < M + 1) p <<= 1;
    return p;
}
int launch_stats(const corr_field& f, const Box& box, bool, Stats st, hipStream_t) {
    const float* x = (const float*)f.data;
    int64_t stride = f.member_stride ? f.member_stride : (int64_t)f.nx * f.ny * f.nz;
    for (int64_t i = 0; i < box.count(); ++i) {
        int64_t p = box.global(i);
        double s = 0;
        for (int m = 0; m < f.M; ++m) s += x[m * stride + p];
        double mean = s / f.M, q = 0;
        for (int m = 0; m < f.M; ++m) {
            double d = x[m * stride + p] - mean;
            q += d * d;
        }
        bool pos = q > 0;
        st.mu32[i] = (float)mean;
        st.inv32[i] = pos ? (float)(1.0 / std::sqrt(q / f.M)) : 0.0f;
        st.rs32[i] = pos ? (float)(1.0 / std::sqrt(q)) : 0.0f;
        st.sigma[i] = (float)std::sqrt(q / f.M);
    }
    return 0;
}
int launch_transpose(const corr_field& f, const Box& box, Stats st, int fmt, void* hi, void*, int64_t rows_pad,
                     int64_t ld, hipStream_t) {
    const float* x = (const float*)f.data;
    int64_t stride = f.member_stride ? f.member_stride : (int64_t)f.nx * f.ny * f.nz;
    float* out = (float*)hi;
    for (int64_t i = 0; i < rows_pad; ++i)
        for (int64_t m = 0; m < ld; ++m) {
            float v = 0.0f;
            if (i < box.count() && m < f.M) {
                int64_t p = box.global(i);
                float mu = st.mu32[i], sc = fmt == ZF_KSG ? st.inv32[i] : st.rs32[i];
                float d = x[m * stride + p] - mu;
                v = d * sc;
            }
            out[i * ld + m] = v;
        }
    return 0;
}
int kernel_setup(const void*, size_t, int, int* per_cu) {
    if (per_cu) *per_cu = 1;
    return 0;
}
int launch_sort_rows(const float* z, int64_t ld, int64_t nrows, int M, float* out, int, hipStream_t) {
    int p2 = ksg_p2(M);
    for (int64_t r = 0; r < nrows; ++r) {
        std::vector<float> v(z + r * ld, z + r * ld + M);
        std::sort(v.begin(), v.end());
        for (int j = 0; j < p2; ++j) out[r * p2 + j] = j < M ? v[j] : INFINITY;
    }
    return 0;
}
}  // namespace corr

static std::vector<char> slurp(const char* path) {
    FILE* f = std::fopen(path, "rb");
    if (!f) { std::perror(path); std::exit(1); }
    std::fseek(f, 0, SEEK_END);
    long n = std::ftell(f);
    std::fseek(f, 0, SEEK_SET);
    std::vector<char> b(n);
    if (std::fread(b.data(), 1, n, f) != (size_t)n) std::exit(1);
    std::fclose(f);
    return b;
}

int main(int argc, char** argv) {
    // input: header int32 M, nx, ny, nz, n_regions, n_pairs, measure, seed; float data[M][P];
    // int32 regions[n][6]; int32 pairs[n_pairs][2]
    auto b = slurp(argv[1]);
    const int32_t* h = (const int32_t*)b.data();
    int M = h[0], nx = h[1], ny = h[2], nz = h[3], nr = h[4], np = h[5], measure = h[6], seed = h[7];
    int64_t P = (int64_t)nx * ny * nz;
    const float* data = (const float*)(h + 8);
    const int32_t* regs = (const int32_t*)(data + (int64_t)M * P);
    const int32_t* pairs = regs + 6 * nr;
    corr_ctx ctx;
    ctx.num_cus = 2;
    std::vector<double> psi(4101);
    psi[1] = -0.57721566490153286061;
    for (int n = 2; n <= 4100; ++n) psi[n] = psi[n - 1] + 1.0 / (n - 1);
    ctx.psi = psi.data();
    ctx.psi_max = 4100;
    corr_field f{data, CORR_F32, M, nx, ny, nz, 0};
    std::vector<corr_region> rr(nr);
    for (int r = 0; r < nr; ++r) rr[r] = corr_region{regs[6 * r], regs[6 * r + 1], regs[6 * r + 2], regs[6 * r + 3], regs[6 * r + 4], regs[6 * r + 5]};
    bos_config cfg;
    bos_config_default(&cfg);
    cfg.measure = measure;
    cfg.seed = (uint64_t)seed;
    bos_state* st = nullptr;
    int rc = bos_create(&ctx, &f, &f, rr.data(), nr, pairs, np, &cfg, &st, nullptr);
    std::fprintf(stderr, "bos_create rc=%d launches=%ld\n", rc, emu_launches);
    if (rc) return 1;
    if (argc > 3 && std::string(argv[3]) == "plain") rc = bos_set_launch(st, BOS_LAUNCH_PLAIN, 60.0);
    if (rc) return 1;
    for (int s = 0; s < 64; ++s) {
        int32_t act = -1;
        rc = bos_sample_step(st, nullptr, &act);
        std::fprintf(stderr, "step %d rc=%d active=%d launches=%ld\n", s + 1, rc, act, emu_launches);
        if (rc || act == 0) break;
    }
    std::vector<corr_max> res(np);
    rc = bos_results(st, res.data(), nullptr);
    FILE* o = std::fopen(argv[2], "w");
    for (int p = 0; p < np; ++p) {
        std::vector<int32_t> cells(6 * 128);
        std::vector<float> vals(128);
        int32_t n = 0;
        bos_history(st, p, cells.data(), vals.data(), &n, nullptr);
        std::fprintf(o, "pair %d value %.9g n %d\n", p, res[p].value, n);
        for (int i = 0; i < n; ++i)
            std::fprintf(o, "%d %d %d %d %d %d %.9g\n", cells[6 * i], cells[6 * i + 1], cells[6 * i + 2], cells[6 * i + 3],
                         cells[6 * i + 4], cells[6 * i + 5], vals[i]);
    }
    std::fclose(o);
    bos_destroy(st);
    return 0;
}
