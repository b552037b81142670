// Launch-parameter tuning and graph-captured progressive integration.
//
// The autotuner times each candidate launch shape with hipEvents on the caller's stream and
// keeps the fastest in the context; tuned values can be saved to and loaded from a small
// JSON file.  Progressive integration (Sec. 2.5: every pixel extends its own sequence, so
// passes can be added without communication) captures the per-pass launches once into a
// hipGraph on a private stream and replays the instantiated graph on the caller's stream.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <vector>

#include "common.hpp"

namespace qmc {

static uint32_t tune_key(uint32_t fkind, uint32_t d, bool backward) {
    return (fkind << 16) | (d << 1) | (backward ? 1u : 0u);
}

IntegrateTune& integrate_tune(qmc_context ctx, uint32_t fkind, uint32_t d, bool backward) {
    return ctx->integrate_tunes[tune_key(fkind, d, backward)];
}

namespace {

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    EventPair() {
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&b);
    }
    ~EventPair() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

// Median time in ms of `reps` runs of `fn` (after one untimed run), or a negative value on error.
template <typename F>
float time_ms(hipStream_t hs, int reps, F&& fn) {
    if (fn() != QMC_OK) return -1.0f;
    std::vector<float> t;
    for (int r = 0; r < reps; ++r) {
        EventPair ev;
        (void)hipEventRecord(ev.a, hs);
        if (fn() != QMC_OK) return -1.0f;
        (void)hipEventRecord(ev.b, hs);
        if (hipEventSynchronize(ev.b) != hipSuccess) return -1.0f;
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, ev.a, ev.b);
        t.push_back(ms);
    }
    std::sort(t.begin(), t.end());
    return t[t.size() / 2];
}

void append(char* report, size_t cap, const char* fmt, ...) {
    if (!report || !cap) return;
    const size_t used = std::strlen(report);
    if (used + 1 >= cap) return;
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(report + used, cap - used, fmt, ap);
    va_end(ap);
}

}  // namespace
}  // namespace qmc

using namespace qmc;

extern "C" qmc_status qmc_autotune_generate(qmc_context ctx, qmc_stream stream, uint32_t kind, const uint32_t* table,
                                            uint32_t s, uint64_t n, const uint32_t* nus_seeds,
                                            const uint32_t* shifts, uint32_t* scratch_u32, float* scratch_f32,
                                            char* report, size_t report_bytes) {
    if (!ctx) return fail(QMC_ERR_INVALID_ARGUMENT, "qmc_autotune_generate: context is NULL");
    if (kind != QMC_SAMPLER_SOBOL && kind != QMC_SAMPLER_LATTICE)
        return fail(QMC_ERR_INVALID_ARGUMENT, "qmc_autotune_generate: kind must be SOBOL or LATTICE");
    if (report && report_bytes) report[0] = 0;
    GenTune& slot = kind == QMC_SAMPLER_SOBOL ? ctx->sobol_tune : ctx->lattice_tune;
    const GenTune saved = slot;
    hipStream_t hs = as_stream(stream);
    auto run = [&]() -> qmc_status {
        if (kind == QMC_SAMPLER_SOBOL)
            return qmc_generate_sobol(ctx, stream, table, s, 0, n, nus_seeds, shifts, 0, scratch_u32, scratch_f32, n);
        return qmc_generate_lattice(ctx, stream, table, s, 0, n, shifts, 0, scratch_u32, scratch_f32, n);
    };
    GenTune best = saved;
    float best_ms = 1e30f;
    std::vector<GenTune> cands;
    for (uint32_t nt = 0; nt < 2; ++nt)
        for (uint32_t cpw : {1u, 2u, 4u, 8u}) cands.push_back(GenTune{cpw, nt});
    for (const GenTune& c : cands) {
        slot = c;
        const float ms = time_ms(hs, 3, run);
        if (ms < 0) {
            slot = saved;
            return fail(QMC_ERR_DEVICE, "qmc_autotune_generate: candidate failed: %s", last_error_slot().c_str());
        }
        append(report, report_bytes, "{\"chunks_per_wave\":%u,\"nontemporal\":%u,\"ms\":%.5f}\n",
               c.chunks_per_wave, c.nontemporal, ms);
        if (ms < best_ms) {
            best_ms = ms;
            best = c;
        }
    }
    slot = best;
    return QMC_OK;
}

extern "C" qmc_status qmc_autotune_integrate(qmc_context ctx, qmc_stream stream, const qmc_sampler* sampler,
                                             const qmc_integrand* integrand, uint32_t width, uint32_t height,
                                             const uint32_t* counts, uint32_t sample_begin, uint32_t sample_end,
                                             int backward, const float* grad_means, float* scratch,
                                             void* workspace, size_t workspace_bytes, char* report,
                                             size_t report_bytes) {
    if (!ctx || !integrand || !scratch) return fail(QMC_ERR_INVALID_ARGUMENT, "qmc_autotune_integrate: NULL argument");
    if (report && report_bytes) report[0] = 0;
    IntegrateTune& slot = integrate_tune(ctx, integrand->kind, integrand->d, backward != 0);
    const IntegrateTune saved = slot;
    hipStream_t hs = as_stream(stream);
    auto run = [&]() -> qmc_status {
        if (backward)
            return qmc_integrate_pixels_backward(ctx, stream, sampler, integrand, width, height, counts, sample_begin,
                                                 sample_end, grad_means, scratch, workspace, workspace_bytes);
        return qmc_integrate_pixels(ctx, stream, sampler, integrand, width, height, counts, sample_begin, sample_end,
                                    nullptr, scratch, workspace, workspace_bytes);
    };
    struct Timed {
        IntegrateTune t;
        float ms;
    };
    std::vector<Timed> timed;
    float best_ms = 1e30f;
    const uint32_t wpcs[] = {4, 8, 16, 32};
    for (uint32_t dyn = 0; dyn < 2; ++dyn) {
        for (uint32_t w : wpcs) {
            slot.waves_per_cu = w;
            slot.dynamic = dyn;
            const float ms = time_ms(hs, 3, run);
            if (ms < 0) {
                slot = saved;
                return fail(QMC_ERR_DEVICE, "qmc_autotune_integrate: candidate failed: %s", last_error_slot().c_str());
            }
            append(report, report_bytes, "{\"waves_per_cu\":%u,\"dynamic\":%u,\"ms\":%.5f}\n", w, dyn, ms);
            timed.push_back({slot, ms});
            best_ms = std::min(best_ms, ms);
        }
    }
    // Near-ties go to fewer waves per CU: the shape is timed with one sampler but serves every
    // sampler of the (integrand, d, direction) key, and the lattice samplers lose up to 10 % at
    // 32 waves per CU where the Sobol' sampler times 16 and 32 within 0.3 % of each other.
    const Timed* pick = nullptr;
    for (const Timed& c : timed) {
        if (c.ms > 1.01f * best_ms) continue;
        if (!pick || c.t.waves_per_cu < pick->t.waves_per_cu ||
            (c.t.waves_per_cu == pick->t.waves_per_cu && c.ms < pick->ms))
            pick = &c;
    }
    slot = pick->t;
    return QMC_OK;
}

extern "C" qmc_status qmc_tune_save(qmc_context ctx, const char* path) {
    if (!ctx || !path) return fail(QMC_ERR_INVALID_ARGUMENT, "qmc_tune_save: NULL argument");
    FILE* f = std::fopen(path, "w");
    if (!f) return fail(QMC_ERR_INVALID_ARGUMENT, "qmc_tune_save: cannot open %s", path);
    for (int k = 0; k < 2; ++k) {
        const GenTune& t = k == 0 ? ctx->sobol_tune : ctx->lattice_tune;
        std::fprintf(f, "%s\"%s\":{\"chunks_per_wave\":%u,\"nontemporal\":%u},\n", k == 0 ? "{" : " ",
                     k == 0 ? "sobol" : "lattice", t.chunks_per_wave, t.nontemporal);
    }
    std::fprintf(f, " \"integrate\":[");
    bool first = true;
    for (const auto& kv : ctx->integrate_tunes) {
        std::fprintf(f, "%s\n  {\"key\":%u,\"waves_per_cu\":%u,\"dynamic\":%u}", first ? "" : ",", kv.first,
                     kv.second.waves_per_cu, kv.second.dynamic);
        first = false;
    }
    std::fprintf(f, "]}\n");
    std::fclose(f);
    return QMC_OK;
}

extern "C" qmc_status qmc_tune_load(qmc_context ctx, const char* path) {
    if (!ctx || !path) return fail(QMC_ERR_INVALID_ARGUMENT, "qmc_tune_load: NULL argument");
    FILE* f = std::fopen(path, "r");
    if (!f) return fail(QMC_ERR_INVALID_ARGUMENT, "qmc_tune_load: cannot open %s", path);
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
    std::fclose(f);
    auto field = [&](size_t from, const char* name, uint32_t* out) -> size_t {
        const std::string pat = std::string("\"") + name + "\":";
        const size_t at = text.find(pat, from);
        if (at == std::string::npos) return std::string::npos;
        *out = static_cast<uint32_t>(std::strtoul(text.c_str() + at + pat.size(), nullptr, 10));
        return at + pat.size();
    };
    if (text.find("\"sobol\"") == std::string::npos)
        return fail(QMC_ERR_INVALID_ARGUMENT, "qmc_tune_load: not a tuning file");
    for (int k = 0; k < 2; ++k) {
        const size_t at = text.find(k == 0 ? "\"sobol\"" : "\"lattice\"");
        uint32_t cpw, nt;
        if (at == std::string::npos || field(at, "chunks_per_wave", &cpw) == std::string::npos ||
            field(at, "nontemporal", &nt) == std::string::npos)
            continue;
        if (cpw < 1 || cpw > 1024) continue;
        GenTune& t = k == 0 ? ctx->sobol_tune : ctx->lattice_tune;
        t = GenTune{cpw, nt ? 1u : 0u};
    }
    size_t pos = text.find("\"integrate\"");
    while (pos != std::string::npos) {
        uint32_t key, w, dyn;
        const size_t k = field(pos, "key", &key);
        if (k == std::string::npos) break;
        if (field(k, "waves_per_cu", &w) == std::string::npos || field(k, "dynamic", &dyn) == std::string::npos) break;
        if (w >= 1 && w <= 64) ctx->integrate_tunes[key] = IntegrateTune{w, dyn ? 1u : 0u};
        pos = text.find("}", k);
    }
    return QMC_OK;
}

extern "C" qmc_status qmc_integrate_progressive(qmc_context ctx, qmc_stream stream, const qmc_sampler* sampler,
                                                const qmc_integrand* integrand, uint32_t width, uint32_t height,
                                                const uint32_t* counts, uint32_t passes, uint32_t spp_per_pass,
                                                float* sums, float* means, void* workspace, size_t workspace_bytes,
                                                int use_graph) {
    const char* who = "qmc_integrate_progressive";
    if (!ctx || !sampler || !integrand) return fail(QMC_ERR_INVALID_ARGUMENT, "%s: NULL argument", who);
    if (!sums) return fail(QMC_ERR_INVALID_ARGUMENT, "%s: sums is required", who);
    if (passes == 0 || spp_per_pass == 0 || uint64_t(passes) * spp_per_pass > 0xFFFFFFFFull)
        return fail(QMC_ERR_OUT_OF_RANGE, "%s: passes * spp_per_pass must be in [1, 2^32)", who);
    auto enqueue = [&](qmc_stream st) -> qmc_status {
        for (uint32_t t = 0; t < passes; ++t) {
            const qmc_status r = qmc_integrate_pixels(ctx, st, sampler, integrand, width, height, counts,
                                                      t * spp_per_pass, (t + 1) * spp_per_pass, sums,
                                                      t + 1 == passes ? means : nullptr, workspace, workspace_bytes);
            if (r != QMC_OK) return r;
        }
        return QMC_OK;
    };
    if (!use_graph) return enqueue(stream);

    DeviceGuard guard(ctx->device);
    if (guard.status != QMC_OK) return guard.status;
    // Everything a replay depends on: a changed pointer, size or parameter means a new graph.
    const IntegrateTune& tn = integrate_tune(ctx, integrand->kind, integrand->d, false);
    std::vector<uint64_t> key = {
        sampler->kind, sampler->s, reinterpret_cast<uint64_t>(sampler->table), sampler->points_ld,
        reinterpret_cast<uint64_t>(sampler->offsets), sampler->seed, sampler->flags,
        reinterpret_cast<uint64_t>(sampler->xor_scramble), reinterpret_cast<uint64_t>(sampler->xor_reorder),
        reinterpret_cast<uint64_t>(sampler->shift_table),
        integrand->kind, integrand->d,
        integrand->num_lobes, integrand->pixel_seed, reinterpret_cast<uint64_t>(integrand->params),
        reinterpret_cast<uint64_t>(integrand->pixel_params), width, height, reinterpret_cast<uint64_t>(counts),
        passes, spp_per_pass, reinterpret_cast<uint64_t>(sums), reinterpret_cast<uint64_t>(means),
        reinterpret_cast<uint64_t>(workspace), workspace_bytes, tn.waves_per_cu, tn.dynamic};
    GraphEntry* entry = nullptr;
    for (auto& g : ctx->graphs)
        if (g.key == key) entry = &g;
    if (!entry) {
        if (!ctx->capture_stream &&
            hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking) != hipSuccess)
            return fail(QMC_ERR_DEVICE, "%s: cannot create the capture stream", who);
        // A pass that fails validation ends and discards the capture before returning.
        GraphEntry g;
        g.key = key;
        if (hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return fail(QMC_ERR_DEVICE, "%s: hipStreamBeginCapture failed", who);
        const qmc_status r = enqueue(ctx->capture_stream);
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(ctx->capture_stream, &graph);
        if (r != QMC_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return r;
        }
        if (e != hipSuccess || !graph) return fail(QMC_ERR_DEVICE, "%s: hipStreamEndCapture failed", who);
        if (hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return fail(QMC_ERR_DEVICE, "%s: hipGraphInstantiate failed", who);
        }
        g.graph = graph;
        if (ctx->graphs.size() >= 16) {  // bound the cache
            (void)hipGraphExecDestroy(ctx->graphs.front().exec);
            (void)hipGraphDestroy(ctx->graphs.front().graph);
            ctx->graphs.erase(ctx->graphs.begin());
        }
        ctx->graphs.push_back(g);
        entry = &ctx->graphs.back();
    }
    if (hipGraphLaunch(entry->exec, as_stream(stream)) != hipSuccess)
        return fail(QMC_ERR_DEVICE, "%s: hipGraphLaunch failed", who);
    return QMC_OK;
}
