// Host side of the batched T-product: autotuner, work-list construction,
// plans with hipGraph capture, and the batched C-ABI entry points.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "batched.h"
#include "facewise_impl.h"
#include "workspace.h"
#include "../../include/qtprod.h"

namespace qt {
namespace {

using detail::NUM_TILE_CFGS;
using detail::tile_mt;
using detail::tile_nt;

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// ------------------------------------------------------------------ tuner
// Cost model of one output tile of shape cfg with k-depth n, in seconds of
// whole-GPU throughput (elapsed time of a launch with many tiles / tiles):
//   t(cfg, n) = alpha[cfg] + beta[cfg] * ceil(n / 16).
// A problem's facewise phase then costs p ceil(m/MT) ceil(s/NT) t(cfg, n),
// padding waste included, and the tuner picks the cheapest shape per problem.
// The FFT radix order (detail::pick_radix policy 0 or 1) is picked per p by
// timing the batched FFT kernel of that length with both.
struct TuneTable {
    bool done = false;
    double alpha[NUM_TILE_CFGS] = {};
    double beta[NUM_TILE_CFGS] = {};
    int fft_pol[65] = {0};
};

std::mutex g_tune_mutex;
std::map<std::pair<int, int>, TuneTable> g_tune;   // (device, precision) -> table

int current_device() {
    int d = 0;
    return hipGetDevice(&d) == hipSuccess ? d : -1;
}

// The split-fp16 tiles run the same instruction mix as the split-bf16 ones
// (f16 instead of bf16 MFMA, same rate), so they share its cost model.
int tune_precision(int prec) { return prec == QT_SPLIT_FP16 ? QT_SPLIT_BF16 : prec; }

bool tuned(int prec, TuneTable* out) {
    prec = tune_precision(prec);
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    auto it = g_tune.find({current_device(), prec});
    if (it == g_tune.end() || !it->second.done) return false;
    if (out) *out = it->second;
    return true;
}

double tile_cost(const TuneTable& t, int cfg, int n) {
    return t.alpha[cfg] + t.beta[cfg] * (double)((n + 15) / 16);
}

// allowed: bit mask of tile shapes to choose from
int pick_tile(const TuneTable* t, int m, int n, int s, unsigned allowed = 0xffu) {
    int best = detail::TILE_128x64;
    double best_cost = 1e300;
    for (int cfg = 0; cfg < NUM_TILE_CFGS; ++cfg) {
        if (!((allowed >> cfg) & 1u)) continue;
        const double tiles = (double)((m + tile_mt(cfg) - 1) / tile_mt(cfg)) *
                             (double)((s + tile_nt(cfg) - 1) / tile_nt(cfg));
        // untuned: padded area as the cost (prefers the least waste)
        const double per = t ? tile_cost(*t, cfg, n) : (double)tile_mt(cfg) * tile_nt(cfg);
        const double c = tiles * per;
        if (c < best_cost * (1.0 - 1e-9)) {
            best_cost = c;
            best = cfg;
        }
    }
    return best;
}

std::string cache_path() {
    const char* p = std::getenv("QT_TUNE_CACHE");
    return p ? std::string(p) : std::string();
}

// Cache file: one line per (device name, precision):
//   <name>|<prec>|a0 a1 a2|b0 b1 b2|pol1 ... pol64
bool load_cache(const std::string& dev_name, int prec, TuneTable* t) {
    const std::string path = cache_path();
    if (path.empty()) return false;
    FILE* fp = std::fopen(path.c_str(), "r");
    if (!fp) return false;
    char line[4096];
    bool found = false;
    while (std::fgets(line, sizeof line, fp)) {
        std::string l(line);
        const size_t b1 = l.find('|'), b2 = l.find('|', b1 + 1);
        if (b1 == std::string::npos || b2 == std::string::npos) continue;
        if (l.substr(0, b1) != dev_name || std::atoi(l.substr(b1 + 1, b2 - b1 - 1).c_str()) != prec) continue;
        TuneTable r;
        const char* q = l.c_str() + b2 + 1;
        char* end = nullptr;
        bool ok = true;
        for (int c = 0; c < NUM_TILE_CFGS && ok; ++c) { r.alpha[c] = std::strtod(q, &end); ok = end != q; q = end; }
        if (ok && *q == '|') ++q; else ok = false;
        for (int c = 0; c < NUM_TILE_CFGS && ok; ++c) { r.beta[c] = std::strtod(q, &end); ok = end != q; q = end; }
        if (ok && *q == '|') ++q; else ok = false;
        for (int p = 1; p <= 64 && ok; ++p) { r.fft_pol[p] = (int)std::strtol(q, &end, 10) & 1; ok = end != q; q = end; }
        if (ok) {
            r.done = true;
            *t = r;
            found = true;
        }
    }
    std::fclose(fp);
    return found;
}

void save_cache(const std::string& dev_name, int prec, const TuneTable& t) {
    const std::string path = cache_path();
    if (path.empty()) return;
    FILE* fp = std::fopen(path.c_str(), "a");
    if (!fp) return;
    std::fprintf(fp, "%s|%d|", dev_name.c_str(), prec);
    for (int c = 0; c < NUM_TILE_CFGS; ++c) std::fprintf(fp, "%.6e ", t.alpha[c]);
    std::fprintf(fp, "|");
    for (int c = 0; c < NUM_TILE_CFGS; ++c) std::fprintf(fp, "%.6e ", t.beta[c]);
    std::fprintf(fp, "|");
    for (int p = 1; p <= 64; ++p) std::fprintf(fp, "%d ", t.fft_pol[p]);
    std::fprintf(fp, "\n");
    std::fclose(fp);
}

// Time `launch` (already warmed) with HIP events: median of reps, seconds.
template <typename F>
double time_launch(F launch, hipStream_t stream, int reps = 3) {
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    launch();
    std::vector<double> ts;
    for (int r = 0; r < reps; ++r) {
        (void)hipEventRecord(e0, stream);
        launch();
        (void)hipEventRecord(e1, stream);
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        ts.push_back(ms * 1e-3);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    std::sort(ts.begin(), ts.end());
    return ts[ts.size() / 2];
}

int run_tuner(int prec, hipStream_t stream, TuneTable* out) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, current_device()) != hipSuccess) return QT_ERR_HIP;
    const std::string dev_name = prop.gcnArchName;
    TuneTable t;
    if (load_cache(dev_name, prec, &t)) {
        *out = t;
        return QT_OK;
    }
    // calibration problem: m = s = 1024, p = 8, k-depth 64 and 256 (zeros:
    // MFMA timing does not depend on the values)
    const int M = 1024, S = 1024, P = 8, NMAX = 256;
    const int lda = NMAX, ldb = S, ldc = S;
    const size_t ea = 4ull * P * M * lda, eb = 4ull * P * NMAX * ldb, ec = 4ull * P * M * ldc;
    float* buf = nullptr;
    if (hipMalloc((void**)&buf, (ea + eb + ec) * sizeof(float)) != hipSuccess) return QT_ERR_ALLOC;
    if (hipMemsetAsync(buf, 0, (ea + eb + ec) * sizeof(float), stream) != hipSuccess) {
        (void)hipFree(buf);
        return QT_ERR_HIP;
    }
    const int ns[2] = {64, NMAX};
    bool fail = false;
    for (int cfg = 0; cfg < NUM_TILE_CFGS && !fail; ++cfg) {
        double tt[2];
        for (int q = 0; q < 2; ++q) {
            FacewiseArgs<float> fa{buf, buf + ea, buf + ea + eb, M, ns[q], S, P, lda, ldb, ldc};
            hipError_t err = hipSuccess;
            const double sec = time_launch([&] { err = launch_facewise_f32(fa, prec, stream, cfg); }, stream);
            if (err != hipSuccess) fail = true;
            const double tiles = (double)P * (M / tile_mt(cfg)) * (S / tile_nt(cfg));
            tt[q] = sec / tiles;
        }
        const double c0 = ns[0] / 16.0, c1 = ns[1] / 16.0;
        t.beta[cfg] = std::max(0.0, (tt[1] - tt[0]) / (c1 - c0));
        t.alpha[cfg] = std::max(0.0, tt[0] - t.beta[cfg] * c0);
    }
    // FFT radix order per p: one tensor of 65536 positions per p, both policies
    const int POS = 65536;
    float *src = nullptr, *dst = nullptr;
    BatchFftJob* djob = nullptr;
    BatchFftItem* ditems = nullptr;
    const int nitems = 2 * POS / 256;
    if (!fail && (hipMalloc((void**)&src, 4ull * 64 * POS * sizeof(float)) != hipSuccess ||
                  hipMalloc((void**)&dst, 4ull * 64 * POS * sizeof(float)) != hipSuccess ||
                  hipMalloc((void**)&djob, sizeof(BatchFftJob)) != hipSuccess ||
                  hipMalloc((void**)&ditems, nitems * sizeof(BatchFftItem)) != hipSuccess))
        fail = true;
    if (!fail) {
        std::vector<BatchFftItem> items(nitems);
        for (int i = 0; i < nitems; ++i) items[i] = BatchFftItem{0, i / (POS / 256), (i % (POS / 256)) * 256, 0};
        fail |= hipMemcpy(ditems, items.data(), nitems * sizeof(BatchFftItem), hipMemcpyHostToDevice) != hipSuccess;
        fail |= hipMemsetAsync(src, 0, 4ull * 64 * POS * sizeof(float), stream) != hipSuccess;
    }
    for (int p = 1; p <= 64 && !fail; ++p) {
        if (!batched_fft_supported(p)) continue;
        Twiddles tw;
        if (get_twiddles(p, stream, &tw) != QT_OK) { fail = true; break; }
        double best = 1e300;
        for (int pol = 0; pol < 2; ++pol) {
            BatchFftJob job{src, dst, tw.f32, 256, POS / 256, POS / 256, POS / 256, p, pol, 0, 0};
            if (hipMemcpy(djob, &job, sizeof job, hipMemcpyHostToDevice) != hipSuccess) { fail = true; break; }
            hipError_t err = hipSuccess;
            const double sec = time_launch(
                [&] { err = launch_batched_fft(false, p, pol, djob, ditems, nitems, stream); }, stream);
            if (err != hipSuccess) { fail = true; break; }
            if (sec < best * 0.98) {   // switch only on a clear win
                best = sec;
                t.fft_pol[p] = pol;
            }
        }
    }
    (void)hipStreamSynchronize(stream);
    (void)hipFree(buf);
    if (src) (void)hipFree(src);
    if (dst) (void)hipFree(dst);
    if (djob) (void)hipFree(djob);
    if (ditems) (void)hipFree(ditems);
    if (fail) return QT_ERR_HIP;
    t.done = true;
    save_cache(dev_name, prec, t);
    *out = t;
    return QT_OK;
}

int ensure_tuned(int prec, hipStream_t stream, TuneTable* out) {
    prec = tune_precision(prec);
    if (tuned(prec, out)) return QT_OK;
    TuneTable t;
    const int st = run_tuner(prec, stream, &t);
    if (st != QT_OK) return st;
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    g_tune[{current_device(), prec}] = t;
    *out = t;
    return QT_OK;
}

// ------------------------------------------------------------ validation
size_t tensor_bytes(long rows, long cols, long p) { return 16ull * p * rows * cols; }
size_t fourier_bytes(long rows, long cols, long p) { return align_up(16ull * p * rows * fourier_ld(cols)); }
bool aligned16(const void* ptr) { return ((uintptr_t)ptr & 15u) == 0; }
bool overlaps(const void* a, size_t abytes, const void* b, size_t bbytes) {
    const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    return a0 < b0 + bbytes && b0 < a0 + abytes;
}

bool problem_ok(const qt_problem& q) {
    if (q.m < 1 || q.n < 1 || q.s < 1 || q.p < 1) return false;
    if ((double)q.p * q.m * q.n > 1e10 || (double)q.p * q.n * q.s > 1e10 || (double)q.p * q.m * q.s > 1e10)
        return false;
    if (!q.A || !q.B || !q.C || !aligned16(q.A) || !aligned16(q.B) || !aligned16(q.C)) return false;
    const size_t cb = tensor_bytes(q.m, q.s, q.p);
    if (overlaps(q.C, cb, q.A, tensor_bytes(q.m, q.n, q.p)) || overlaps(q.C, cb, q.B, tensor_bytes(q.n, q.s, q.p)))
        return false;
    return true;
}

// ------------------------------------------------------- work-list layout
struct DescLayout {
    size_t fwd_jobs, fwd_items, probs, gitems, inv_jobs, inv_items, h_jobs, h_items, h_floats, tensors, total;
    long n_fwd_items_max, n_gitems_max, n_inv_items_max, n_h_items;
};

DescLayout desc_layout(int count, const qt_problem* probs) {
    DescLayout L{};
    long nfi = 0, ngi = 0, nii = 0, nfaces = 0;
    size_t tens = 0;
    for (int i = 0; i < count; ++i) {
        const qt_problem& q = probs[i];
        nfaces += 2L * q.p;                                     // split fp16: faces of A^ and B^
        // forward positions run over the padded rows (BatchFftJob::fill)
        nfi += 2 * (((long)q.m * fourier_ld(q.n) + 255) / 256) + 2 * (((long)q.n * fourier_ld(q.s) + 255) / 256);
        ngi += (long)q.p * ((q.m + 31) / 32) * ((q.s + 63) / 64);   // 32 x 64 is the smallest tile
        nii += 2 * (((long)q.m * q.s + 255) / 256);
        tens += fourier_bytes(q.m, q.n, q.p) + fourier_bytes(q.n, q.s, q.p) + fourier_bytes(q.m, q.s, q.p);
    }
    size_t off = 0;
    auto take = [&](size_t b) { size_t o = off; off += align_up(b); return o; };
    L.fwd_jobs = take(sizeof(BatchFftJob) * 2 * count);
    L.fwd_items = take(sizeof(BatchFftItem) * nfi);
    L.probs = take(sizeof(BatchGemmProb) * count);
    L.gitems = take(sizeof(BatchGemmItem) * ngi);
    L.inv_jobs = take(sizeof(BatchFftJob) * count);
    L.inv_items = take(sizeof(BatchFftItem) * nii);
    // split fp16: operand jobs, face items, and per face a maximum and a scale
    L.h_jobs = take(sizeof(BatchFp16Job) * 2 * count);
    L.h_items = take(sizeof(BatchFp16Item) * nfaces);
    L.h_floats = take(sizeof(float) * 2 * nfaces);
    L.tensors = off;
    L.total = off + tens;
    L.n_fwd_items_max = nfi;
    L.n_gitems_max = ngi;
    L.n_inv_items_max = nii;
    L.n_h_items = nfaces;
    return L;
}

// A run of FFT items with one tube length (and so one radix-order policy).
struct FftBucket {
    int p, pol, first, count;
};

// A problem whose tube length has no batched FFT kernel (not 7-smooth, or
// p > 64): its transforms are launched on their own (register-resident or
// Bluestein kernels of the single-problem path); its products still go into
// the shared persistent launches.
struct SingleFft {
    int p;
    Twiddles tw;
    FftJob<float> fwd[2], inv;
};

struct HostLists {
    std::vector<SingleFft> single;
    std::vector<BatchFftJob> fwd_jobs, inv_jobs;
    std::vector<BatchFftItem> fwd_items, inv_items;
    std::vector<FftBucket> fwd_buckets, inv_buckets;
    std::vector<BatchGemmProb> probs;
    std::vector<BatchGemmItem> gitems;      // grouped by tile shape, longest first in each group
    std::vector<BatchFp16Job> h_jobs;       // split fp16 only: A^, B^ of every problem
    std::vector<BatchFp16Item> h_items;
    int gfirst[detail::NUM_TILE_CFGS] = {}, gcount[detail::NUM_TILE_CFGS] = {};
};

void add_fft_items(std::vector<BatchFftItem>& items, int job, long positions) {
    for (int part = 0; part < 2; ++part)
        for (long e0 = 0; e0 < positions; e0 += 256) items.push_back(BatchFftItem{job, part, (int)e0, 0});
}

// Build the three work lists; longest items first so that the grid-stride
// walk approximates longest-processing-time scheduling.
int build_lists(int count, const qt_problem* probs, int prec, char* ws, const DescLayout& L,
                const TuneTable& tune, hipStream_t stream, HostLists* H) {
    size_t off = L.tensors;
    long hface = 0;                          // split fp16: faces placed so far (2 p per problem)
    for (int i = 0; i < count; ++i) {
        const qt_problem& q = probs[i];
        Twiddles tw;
        const int st = get_twiddles(q.p, stream, &tw);
        if (st != QT_OK) return st;
        const int lda = (int)fourier_ld(q.n), ldb = (int)fourier_ld(q.s), ldc = ldb;
        float* Ah = reinterpret_cast<float*>(ws + off); off += fourier_bytes(q.m, q.n, q.p);
        float* Bh = reinterpret_cast<float*>(ws + off); off += fourier_bytes(q.n, q.s, q.p);
        float* Ch = reinterpret_cast<float*>(ws + off); off += fourier_bytes(q.m, q.s, q.p);
        const int pol = q.p <= 64 ? tune.fft_pol[q.p] : 0;
        const int pack = prec == QT_SPLIT_BF16 ? 1 : 0;
        if (!batched_fft_supported(q.p)) {
            SingleFft sf{q.p, tw, {}, {}};
            sf.fwd[0] = FftJob<float>{(const float*)q.A, Ah, q.m, q.n, q.n, lda, pack, 2, 0, 1};
            sf.fwd[1] = FftJob<float>{(const float*)q.B, Bh, q.n, q.s, q.s, ldb, pack, 2, 0, 1};
            sf.inv = FftJob<float>{Ch, (float*)q.C, q.m, q.s, ldc, q.s};
            H->single.push_back(sf);
        }
        H->fwd_jobs.push_back(BatchFftJob{(const float*)q.A, Ah, tw.f32, q.m, q.n, q.n, lda, q.p, pol, pack, lda > q.n});
        H->fwd_jobs.push_back(BatchFftJob{(const float*)q.B, Bh, tw.f32, q.n, q.s, q.s, ldb, q.p, pol, pack, ldb > q.s});
        H->inv_jobs.push_back(BatchFftJob{Ch, (float*)q.C, tw.f32, q.m, q.s, ldc, q.s, q.p, pol, 0, 0});
        const int cfg = pick_tile(&tune, q.m, q.n, q.s);
        const float* scales = nullptr;
        if (prec == QT_SPLIT_FP16) {
            // faces of A^ then of B^: a maximum each, then the scales (A^ at f,
            // the B^ pair {f, -f}) in the same order
            float* fmax = reinterpret_cast<float*>(ws + L.h_floats) + 2 * hface;
            float* sc = fmax + 2 * q.p;
            H->h_jobs.push_back(BatchFp16Job{Ah, fmax, sc, q.m, q.n, lda, q.p});
            H->h_jobs.push_back(BatchFp16Job{Bh, fmax + q.p, sc + q.p, q.n, q.s, ldb, q.p});
            for (int part = 0; part < 2; ++part)
                for (int f = 0; f < q.p; ++f) H->h_items.push_back(BatchFp16Item{2 * i + part, f});
            hface += 2 * q.p;
            scales = sc;
        }
        H->probs.push_back(BatchGemmProb{FacewiseArgs<float>{Ah, Bh, Ch, q.m, q.n, q.s, q.p, lda, ldb, ldc},
                                         scales, cfg, 0});
    }
    // batched FFT items only for the lengths the batched kernel has
    for (int j = 0; j < (int)H->fwd_jobs.size(); ++j)
        if (batched_fft_supported(H->fwd_jobs[j].p))
            add_fft_items(H->fwd_items, j,
                          (long)H->fwd_jobs[j].rows * (H->fwd_jobs[j].fill ? H->fwd_jobs[j].dst_ld : H->fwd_jobs[j].cols));
    for (int j = 0; j < (int)H->inv_jobs.size(); ++j)
        if (batched_fft_supported(H->inv_jobs[j].p))
            add_fft_items(H->inv_items, j, (long)H->inv_jobs[j].rows * H->inv_jobs[j].cols);
    auto by_p = [](const std::vector<BatchFftJob>& jobs) {
        return [&jobs](const BatchFftItem& x, const BatchFftItem& y) { return jobs[x.job].p > jobs[y.job].p; };
    };
    std::stable_sort(H->fwd_items.begin(), H->fwd_items.end(), by_p(H->fwd_jobs));
    std::stable_sort(H->inv_items.begin(), H->inv_items.end(), by_p(H->inv_jobs));
    auto buckets = [](const std::vector<BatchFftJob>& jobs, const std::vector<BatchFftItem>& items,
                      std::vector<FftBucket>& out) {
        for (int i = 0; i < (int)items.size(); ++i) {
            const BatchFftJob& j = jobs[items[i].job];
            if (out.empty() || out.back().p != j.p) out.push_back(FftBucket{j.p, j.pol, i, 0});
            ++out.back().count;
        }
    };
    buckets(H->fwd_jobs, H->fwd_items, H->fwd_buckets);
    buckets(H->inv_jobs, H->inv_items, H->inv_buckets);

    std::vector<std::pair<double, BatchGemmItem>> g;
    for (int i = 0; i < count; ++i) {
        const BatchGemmProb& pr = H->probs[i];
        const int MT = tile_mt(pr.cfg), NT = tile_nt(pr.cfg);
        const int tm_n = (pr.a.m + MT - 1) / MT, tn_n = (pr.a.s + NT - 1) / NT;
        const double c = tile_cost(tune, pr.cfg, pr.a.n) + 1e-12 * MT * NT * ((pr.a.n + 15) / 16);
        for (int f = 0; f < pr.a.p; ++f)
            for (int tm = 0; tm < tm_n; ++tm)
                for (int tn = 0; tn < tn_n; ++tn) g.push_back({c, BatchGemmItem{i, f, tm, tn}});
    }
    std::stable_sort(g.begin(), g.end(), [](const auto& x, const auto& y) { return x.first > y.first; });
    H->gitems.reserve(g.size());
    // one persistent launch per tile shape: group the (sorted) items by shape
    for (int cfg = 0; cfg < detail::NUM_TILE_CFGS; ++cfg) {
        H->gfirst[cfg] = (int)H->gitems.size();
        for (auto& e : g)
            if (H->probs[e.second.prob].cfg == cfg) H->gitems.push_back(e.second);
        H->gcount[cfg] = (int)H->gitems.size() - H->gfirst[cfg];
    }
    if ((long)H->fwd_items.size() > L.n_fwd_items_max || (long)H->gitems.size() > L.n_gitems_max ||
        (long)H->inv_items.size() > L.n_inv_items_max || (long)H->h_items.size() > L.n_h_items ||
        (long)H->h_jobs.size() > 2L * count)
        return QT_ERR_INVALID_ARG;   // cannot happen: the layout is an upper bound
    return QT_OK;
}

int upload(const HostLists& H, char* ws, const DescLayout& L, hipStream_t stream) {
    struct Part { size_t off; const void* src; size_t bytes; };
    const Part parts[8] = {
        {L.fwd_jobs, H.fwd_jobs.data(), H.fwd_jobs.size() * sizeof(BatchFftJob)},
        {L.fwd_items, H.fwd_items.data(), H.fwd_items.size() * sizeof(BatchFftItem)},
        {L.probs, H.probs.data(), H.probs.size() * sizeof(BatchGemmProb)},
        {L.gitems, H.gitems.data(), H.gitems.size() * sizeof(BatchGemmItem)},
        {L.inv_jobs, H.inv_jobs.data(), H.inv_jobs.size() * sizeof(BatchFftJob)},
        {L.inv_items, H.inv_items.data(), H.inv_items.size() * sizeof(BatchFftItem)},
        {L.h_jobs, H.h_jobs.data(), H.h_jobs.size() * sizeof(BatchFp16Job)},
        {L.h_items, H.h_items.data(), H.h_items.size() * sizeof(BatchFp16Item)},
    };
    for (const Part& pt : parts) {
        if (!pt.bytes) continue;
        // pageable source: the call returns once the bytes are staged, so the
        // host vectors may be released afterwards
        if (hipMemcpyAsync(ws + pt.off, pt.src, pt.bytes, hipMemcpyHostToDevice, stream) != hipSuccess)
            return QT_ERR_HIP;
    }
    return QT_OK;
}

// Persistent product grid of a tile shape: exactly the workgroups that can be
// resident at once.
int gemm_grid(int prec, int cfg) {
    int dev = current_device(), cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return cus * batched_gemm_blocks_per_cu(prec, cfg);
}

int enqueue(const HostLists& H, char* ws, const DescLayout& L, int prec, hipStream_t stream) {
    const auto* fj = reinterpret_cast<const BatchFftJob*>(ws + L.fwd_jobs);
    const auto* fi = reinterpret_cast<const BatchFftItem*>(ws + L.fwd_items);
    const auto* pj = reinterpret_cast<const BatchGemmProb*>(ws + L.probs);
    const auto* gi = reinterpret_cast<const BatchGemmItem*>(ws + L.gitems);
    const auto* ij = reinterpret_cast<const BatchFftJob*>(ws + L.inv_jobs);
    const auto* ii = reinterpret_cast<const BatchFftItem*>(ws + L.inv_items);
    for (const FftBucket& b : H.fwd_buckets)
        if (launch_batched_fft(false, b.p, b.pol, fj, fi + b.first, b.count, stream) != hipSuccess)
            return QT_ERR_HIP;
    for (const SingleFft& sf : H.single)
        if (launch_tube_fft<float>(sf.p, false, sf.fwd, 2, sf.tw, stream) != hipSuccess) return QT_ERR_HIP;
    if (!H.h_items.empty() &&
        launch_batched_fp16_prep(reinterpret_cast<const BatchFp16Job*>(ws + L.h_jobs),
                                 reinterpret_cast<const BatchFp16Item*>(ws + L.h_items), (int)H.h_items.size(), pj,
                                 (int)H.probs.size(), stream) != hipSuccess)
        return QT_ERR_HIP;
    for (int cfg = 0; cfg < detail::NUM_TILE_CFGS; ++cfg) {
        const int n = H.gcount[cfg];
        if (n && launch_batched_gemm(prec, cfg, pj, gi + H.gfirst[cfg], n, std::min(n, gemm_grid(prec, cfg)),
                                     stream) != hipSuccess)
            return QT_ERR_HIP;
    }
    for (const FftBucket& b : H.inv_buckets)
        if (launch_batched_fft(true, b.p, b.pol, ij, ii + b.first, b.count, stream) != hipSuccess)
            return QT_ERR_HIP;
    for (const SingleFft& sf : H.single)
        if (launch_tube_fft<float>(sf.p, true, &sf.inv, 1, sf.tw, stream) != hipSuccess) return QT_ERR_HIP;
    return QT_OK;
}

int validate(int count, const qt_problem* probs, int prec, void* ws, size_t ws_bytes, DescLayout* L) {
    if (count < 1 || !probs || !ws || !aligned16(ws)) return QT_ERR_INVALID_ARG;
    if (prec != QT_FP32 && prec != QT_SPLIT_BF16 && prec != QT_SPLIT_FP16 && prec != QT_FP64)
        return QT_ERR_INVALID_ARG;
    for (int i = 0; i < count; ++i)
        if (!problem_ok(probs[i])) return QT_ERR_INVALID_ARG;
    *L = desc_layout(count, probs);
    if (ws_bytes < L->total) return QT_ERR_INVALID_ARG;
    for (int i = 0; i < count; ++i) {
        const qt_problem& q = probs[i];
        const size_t cb = tensor_bytes(q.m, q.s, q.p);
        if (overlaps(q.C, cb, ws, L->total) || overlaps(q.A, tensor_bytes(q.m, q.n, q.p), ws, L->total) ||
            overlaps(q.B, tensor_bytes(q.n, q.s, q.p), ws, L->total))
            return QT_ERR_INVALID_ARG;
    }
    // outputs must not overlap any other problem's input or output
    std::vector<std::pair<uintptr_t, uintptr_t>> outs;
    for (int i = 0; i < count; ++i) {
        const uintptr_t c0 = (uintptr_t)probs[i].C;
        outs.push_back({c0, c0 + tensor_bytes(probs[i].m, probs[i].s, probs[i].p)});
    }
    std::vector<std::pair<uintptr_t, uintptr_t>> sorted = outs;
    std::sort(sorted.begin(), sorted.end());
    for (size_t i = 1; i < sorted.size(); ++i)
        if (sorted[i].first < sorted[i - 1].second) return QT_ERR_INVALID_ARG;
    for (int i = 0; i < count; ++i) {
        const void* in[2] = {probs[i].A, probs[i].B};
        const size_t inb[2] = {tensor_bytes(probs[i].m, probs[i].n, probs[i].p),
                               tensor_bytes(probs[i].n, probs[i].s, probs[i].p)};
        for (int k = 0; k < 2; ++k) {
            const uintptr_t a0 = (uintptr_t)in[k], a1 = a0 + inb[k];
            auto it = std::lower_bound(sorted.begin(), sorted.end(), std::make_pair(a1, (uintptr_t)0));
            if (it != sorted.begin()) {
                --it;
                if (it->second > a0) return QT_ERR_INVALID_ARG;
            }
        }
    }
    if (prec == QT_FP64) return QT_ERR_UNSUPPORTED;
    for (int i = 0; i < count; ++i)
        if (probs[i].p > QT_MAX_P) return QT_ERR_UNSUPPORTED;
    return QT_OK;
}

}  // namespace

int choose_tile(int m, int n, int s, int precision) {
    TuneTable t;
    // untuned: the shape with the least padded area (ties: 128 x 64)
    return pick_tile(tuned(precision, &t) ? &t : nullptr, m, n, s);
}

// One-shot batched product on a workspace of ws_bytes (validated here).
int run_batched(int count, const qt_problem* probs, int precision, void* ws, size_t ws_bytes,
                hipStream_t stream) {
    DescLayout L;
    int st = validate(count, probs, precision, ws, ws_bytes, &L);
    if (st != QT_OK) return st;
    TuneTable t;
    st = ensure_tuned(precision, stream, &t);
    if (st != QT_OK) return st;
    HostLists H;
    st = build_lists(count, probs, precision, (char*)ws, L, t, stream, &H);
    if (st != QT_OK) return st;
    st = upload(H, (char*)ws, L, stream);
    if (st != QT_OK) return st;
    return enqueue(H, (char*)ws, L, precision, stream);
}

}  // namespace qt

struct qt_batched_plan_s {
    int device = -1;
    int precision = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" {

qt_status qt_autotune(qt_precision precision, hipStream_t stream) {
    if (precision != QT_FP32 && precision != QT_SPLIT_BF16 && precision != QT_SPLIT_FP16)
        return QT_ERR_UNSUPPORTED;
    qt::TuneTable t;
    return qt::to_status(qt::ensure_tuned(precision, stream, &t));
}

size_t qt_batched_workspace_size(int count, const qt_problem* probs, qt_precision precision) {
    if (count < 1 || !probs) return 0;
    if (precision != QT_FP32 && precision != QT_SPLIT_BF16 && precision != QT_SPLIT_FP16 &&
        precision != QT_FP64)
        return 0;
    for (int i = 0; i < count; ++i) {
        const qt_problem& q = probs[i];
        if (q.m < 1 || q.n < 1 || q.s < 1 || q.p < 1) return 0;
    }
    return qt::desc_layout(count, probs).total;
}

qt_status qt_tprod_batched(int count, const qt_problem* probs, qt_precision precision, void* ws, size_t ws_bytes,
                     hipStream_t stream) {
    return qt::with_workspace(ws, ws_bytes, qt_batched_workspace_size(count, probs, precision), stream,
                              [&](void* w, size_t wb) { return qt::run_batched(count, probs, precision, w, wb, stream); });
}

qt_status qt_batched_plan_create(int count, const qt_problem* probs, qt_precision precision, void* ws, size_t ws_bytes,
                           hipStream_t stream, qt_batched_plan* out) {
    if (!out) return QT_ERR_INVALID_ARG;
    *out = nullptr;
    qt::DescLayout L;
    int st = qt::validate(count, probs, precision, ws, ws_bytes, &L);
    if (st != QT_OK) return qt::to_status(st);
    qt::TuneTable t;
    st = qt::ensure_tuned(precision, stream, &t);
    if (st != QT_OK) return qt::to_status(st);
    qt::HostLists H;
    st = qt::build_lists(count, probs, precision, (char*)ws, L, t, stream, &H);
    if (st != QT_OK) return qt::to_status(st);
    st = qt::upload(H, (char*)ws, L, stream);
    if (st != QT_OK) return qt::to_status(st);
    if (hipStreamSynchronize(stream) != hipSuccess) return QT_ERR_HIP;

    hipStream_t cap = nullptr;
    if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) return QT_ERR_HIP;
    auto* plan = new qt_batched_plan_s();
    plan->precision = precision;
    plan->device = qt::current_device();
    bool ok = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
        st = qt::enqueue(H, (char*)ws, L, precision, cap);
        ok = hipStreamEndCapture(cap, &plan->graph) == hipSuccess && st == QT_OK;
    }
    if (ok) ok = hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0) == hipSuccess;
    (void)hipStreamDestroy(cap);
    if (!ok) {
        if (plan->graph) (void)hipGraphDestroy(plan->graph);
        delete plan;
        return QT_ERR_HIP;
    }
    *out = plan;
    return QT_OK;
}

qt_status qt_batched_plan_launch(qt_batched_plan plan, hipStream_t stream) {
    if (!plan || !plan->exec) return QT_ERR_INVALID_ARG;
    return qt::to_status(hipGraphLaunch(plan->exec, stream) == hipSuccess ? QT_OK : QT_ERR_HIP);
}

qt_status qt_batched_plan_destroy(qt_batched_plan plan) {
    if (!plan) return QT_ERR_INVALID_ARG;
    int st = QT_OK;
    if (plan->exec && hipGraphExecDestroy(plan->exec) != hipSuccess) st = QT_ERR_HIP;
    if (plan->graph && hipGraphDestroy(plan->graph) != hipSuccess) st = QT_ERR_HIP;
    delete plan;
    return qt::to_status(st);
}

}  // extern "C"
