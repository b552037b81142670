// Host-side checks of the library under AddressSanitizer and UndefinedBehaviorSanitizer.
//
// Built from the library's sources compiled for the host only (no device code: every call below
// must fail its argument validation or stay on the host), with a context filled in by hand so
// that no GPU is needed.  Prints one line per call, "name status", plus the setup outputs, which
// the Python test compares with the oracle; any sanitizer report aborts the program.
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "common.hpp"

namespace {

int failures = 0;

void report(const char* name, qmc_status got, qmc_status want) {
    std::printf("%s %d\n", name, static_cast<int>(got));
    if (got != want) {
        std::printf("MISMATCH %s: status %d, expected %d (%s)\n", name, static_cast<int>(got), static_cast<int>(want),
                    qmc_last_error());
        ++failures;
    }
    // the error text is a valid C string whatever happened
    (void)std::strlen(qmc_last_error());
}

// A small tuning file with the given text.
std::string tune_file(const char* dir, const char* name, const char* text) {
    const std::string path = std::string(dir) + "/" + name;
    FILE* f = std::fopen(path.c_str(), "w");
    if (f) {
        std::fputs(text, f);
        std::fclose(f);
    }
    return path;
}

}  // namespace

int main(int argc, char** argv) {
    const char* dir = argc > 1 ? argv[1] : ".";
    qmc_context_s ctx;
    ctx.device = 0;
    ctx.num_cus = 256;
    const qmc_status OK = QMC_OK, INV = QMC_ERR_INVALID_ARGUMENT, OOR = QMC_ERR_OUT_OF_RANGE,
                     UNS = QMC_ERR_UNSUPPORTED, DEV = QMC_ERR_DEVICE, WSP = QMC_ERR_WORKSPACE;

    // ------------------------------------------------------------- setup (host) ----
    std::vector<uint32_t> codes(300);
    report("poly_null", qmc_primitive_polynomials(5, nullptr), INV);
    report("poly_300", qmc_primitive_polynomials(300, codes.data()), OK);
    std::printf("poly:");
    for (uint32_t c : codes) std::printf(" %u", c);
    std::printf("\n");
    for (uint32_t s : {1u, 7u, 64u}) {
        std::vector<uint32_t> di(size_t(s) * QMC_MAX_DEGREE, 1u), m(size_t(s) * 32), w(size_t(s) * 64);
        for (size_t k = 0; k < di.size(); ++k) di[k] = (k * 2654435761u) | 1u;
        // direction numbers must be odd and below 2^(k+1): reduce them
        for (uint32_t j = 0; j < s; ++j)
            for (uint32_t k = 0; k < QMC_MAX_DEGREE; ++k) di[j * QMC_MAX_DEGREE + k] &= (2u << k) - 1u;
        char name[64];
        std::snprintf(name, sizeof name, "sobol_matrices_%u", s);
        report(name, qmc_sobol_matrices(s, di.data(), m.data()), OK);
        std::printf("mats_%u:", s);
        for (uint32_t v : m) std::printf(" %u", v);
        std::printf("\n");
        std::snprintf(name, sizeof name, "sobol_matrices_wide_%u", s);
        report(name, qmc_sobol_matrices_wide(s, di.data(), 64, w.data()), OK);
        std::printf("wide_%u:", s);
        for (uint32_t v : w) std::printf(" %u", v);
        std::printf("\n");
    }
    {
        std::vector<uint32_t> di(2 * QMC_MAX_DEGREE, 2u), m(64), w(2 * 65);
        report("sobol_matrices_even", qmc_sobol_matrices(2, di.data(), m.data()), INV);
        report("sobol_matrices_s0", qmc_sobol_matrices(0, di.data(), m.data()), OOR);
        report("sobol_matrices_s65", qmc_sobol_matrices(65, di.data(), m.data()), OOR);
        report("sobol_matrices_null", qmc_sobol_matrices(2, nullptr, m.data()), INV);
        for (auto& v : di) v = 1u;
        report("sobol_matrices_wide_c0", qmc_sobol_matrices_wide(2, di.data(), 0, w.data()), OOR);
        report("sobol_matrices_wide_c65", qmc_sobol_matrices_wide(2, di.data(), 65, w.data()), OOR);
    }

    // ------------------------------------------------- argument validation only ----
    uint32_t dummy_u[64] = {};
    float dummy_f[64] = {};
    uint32_t* du = dummy_u;  // never dereferenced: every call below fails validation first
    float* df = dummy_f;
    report("sobol_null_ctx", qmc_generate_sobol(nullptr, nullptr, du, 4, 0, 10, nullptr, nullptr, 0, du, df, 10), INV);
    report("sobol_null_mats", qmc_generate_sobol(&ctx, nullptr, nullptr, 4, 0, 10, nullptr, nullptr, 0, du, df, 10), INV);
    report("sobol_s0", qmc_generate_sobol(&ctx, nullptr, du, 0, 0, 10, nullptr, nullptr, 0, du, df, 10), OOR);
    report("sobol_s65", qmc_generate_sobol(&ctx, nullptr, du, 65, 0, 10, nullptr, nullptr, 0, du, df, 10), OOR);
    report("sobol_no_out", qmc_generate_sobol(&ctx, nullptr, du, 4, 0, 10, nullptr, nullptr, 0, nullptr, nullptr, 10),
           INV);
    report("sobol_ld", qmc_generate_sobol(&ctx, nullptr, du, 4, 0, 10, nullptr, nullptr, 0, du, df, 9), INV);
    report("sobol_range", qmc_generate_sobol(&ctx, nullptr, du, 4, 0xFFFFFFFFull, 2, nullptr, nullptr, 0, du, df, 2),
           OOR);
    report("sobol_flags", qmc_generate_sobol(&ctx, nullptr, du, 4, 0, 10, nullptr, nullptr, 0x8000u, du, df, 10), INV);
    report("sobol_pm_ld", qmc_generate_sobol(&ctx, nullptr, du, 4, 0, 10, nullptr, nullptr, QMC_POINT_MAJOR, du, df, 3),
           INV);
    report("lattice_null", qmc_generate_lattice(&ctx, nullptr, nullptr, 4, 0, 10, nullptr, 0, du, df, 10), INV);
    report("lattice_range", qmc_generate_lattice(&ctx, nullptr, du, 4, 1ull << 32, 1, nullptr, 0, du, df, 1), OOR);
    report("halton_mode", qmc_generate_halton(&ctx, nullptr, 4, 0, 10, 7u, nullptr, du, df, 10), INV);
    report("halton_s65", qmc_generate_halton(&ctx, nullptr, 65, 0, 10, QMC_HALTON_IDENTITY, nullptr, du, df, 10), OOR);
    report("halton_linear_null",
           qmc_generate_halton(&ctx, nullptr, 4, 0, 10, QMC_HALTON_LINEAR, nullptr, du, df, 10), INV);
    report("sobol64_columns", qmc_generate_sobol64(&ctx, nullptr, du, 65, 4, 0, 0, 0, 10, nullptr, nullptr, 0, du, df, 10),
           OOR);
    report("sobol64_part", qmc_generate_sobol64(&ctx, nullptr, du, 64, 4, 3, 8, 0, 10, nullptr, nullptr, 0, du, df, 10),
           OOR);
    report("sobol64_range",
           qmc_generate_sobol64(&ctx, nullptr, du, 40, 4, 8, 0, (1ull << 32) - 5, 10, nullptr, nullptr, 0, du, df, 10),
           OOR);
    report("lattice64_parts", qmc_generate_lattice64(&ctx, nullptr, du, 4, 33, 0, 0, 10, nullptr, 0, du, df, 10), OOR);
    report("unifloat_null", qmc_map_u32_to_unifloat(&ctx, nullptr, nullptr, df, 10), INV);

    qmc_sampler sp{};
    sp.kind = QMC_SAMPLER_SOBOL;
    sp.s = 8;
    sp.table = du;
    sp.flags = QMC_PIXEL_NUS | QMC_PIXEL_SHIFT;
    qmc_integrand genz{};
    genz.kind = QMC_F_GENZ;
    genz.d = 8;
    genz.pixel_params = df;
    qmc_integrand lobes{};
    lobes.kind = QMC_F_LOBES;
    lobes.d = 8;
    lobes.num_lobes = 64;
    lobes.params = df;
    size_t bytes = 0;
    report("ws_genz", qmc_workspace_size(&ctx, &sp, &genz, 1920, 1080, 0, &bytes), OK);
    std::printf("ws_genz_bytes %zu\n", bytes);
    report("ws_lobes_bwd", qmc_workspace_size(&ctx, &sp, &lobes, 1920, 1080, 1, &bytes), OK);
    std::printf("ws_lobes_bwd_bytes %zu\n", bytes);
    report("ws_lobes_step", qmc_workspace_size(&ctx, &sp, &lobes, 3840, 2160, 2, &bytes), OK);
    std::printf("ws_lobes_step_bytes %zu\n", bytes);
    report("ws_mode", qmc_workspace_size(&ctx, &sp, &lobes, 8, 8, 3, &bytes), INV);
    report("ws_null", qmc_workspace_size(&ctx, &sp, &lobes, 8, 8, 1, nullptr), INV);

    char ws[64];
    report("int_null_sampler",
           qmc_integrate_pixels(&ctx, nullptr, nullptr, &genz, 8, 8, du, 0, 64, df, df, ws, sizeof ws), INV);
    qmc_integrand genz_d7 = genz;
    genz_d7.d = 7;
    report("int_genz_d7", qmc_integrate_pixels(&ctx, nullptr, &sp, &genz_d7, 8, 8, du, 0, 64, df, df, ws, sizeof ws),
           UNS);
    qmc_sampler sp_small = sp;
    sp_small.s = 4;
    report("int_d_gt_s", qmc_integrate_pixels(&ctx, nullptr, &sp_small, &genz, 8, 8, du, 0, 64, df, df, ws, sizeof ws),
           INV);
    report("int_empty", qmc_integrate_pixels(&ctx, nullptr, &sp, &genz, 0, 8, du, 0, 64, df, df, ws, sizeof ws), OOR);
    report("int_window", qmc_integrate_pixels(&ctx, nullptr, &sp, &genz, 8, 8, du, 65, 64, df, df, ws, sizeof ws), INV);
    report("int_no_out", qmc_integrate_pixels(&ctx, nullptr, &sp, &genz, 8, 8, du, 0, 64, nullptr, nullptr, ws,
                                              sizeof ws),
           INV);
    report("int_workspace", qmc_integrate_pixels(&ctx, nullptr, &sp, &genz, 8, 8, du, 0, 64, df, df, ws, sizeof ws),
           WSP);
    qmc_sampler bad_flags = sp;
    bad_flags.flags = 1u << 20;
    report("int_flags", qmc_integrate_pixels(&ctx, nullptr, &bad_flags, &genz, 8, 8, du, 0, 64, df, df, ws, sizeof ws),
           INV);
    qmc_sampler xor_bad = sp;
    xor_bad.kind = QMC_SAMPLER_XOR_TABLE;
    xor_bad.flags = 0;
    xor_bad.points_ld = 3;
    xor_bad.xor_scramble = du;
    xor_bad.xor_reorder = du;
    report("int_xor_n", qmc_integrate_pixels(&ctx, nullptr, &xor_bad, &genz, 8, 8, du, 0, 64, df, df, ws, sizeof ws),
           INV);
    qmc_sampler hil = sp;
    hil.kind = QMC_SAMPLER_LATTICE;
    hil.flags = QMC_PIXEL_HILBERT_SHIFT;
    report("int_hilbert_size",
           qmc_integrate_pixels(&ctx, nullptr, &hil, &genz, 40000, 2, du, 0, 64, df, df, ws, sizeof ws), OOR);
    report("bwd_genz", qmc_integrate_pixels_backward(&ctx, nullptr, &sp, &genz, 8, 8, du, 0, 64, df, df, ws, sizeof ws),
           UNS);
    qmc_integrand lobes0 = lobes;
    lobes0.num_lobes = 0;
    report("bwd_lobes0",
           qmc_integrate_pixels_backward(&ctx, nullptr, &sp, &lobes0, 8, 8, du, 0, 64, df, df, ws, sizeof ws), OOR);
    report("step_loss_null",
           qmc_integrate_pixels_l2_step(&ctx, nullptr, &sp, &lobes, 8, 8, du, df, df, nullptr, df, ws, sizeof ws), INV);
    report("noalloc_no_scratch",
           qmc_integrate_pixels_l2_step_noalloc(&ctx, nullptr, &sp, &lobes, 8, 8, du, df, df, df, df), DEV);
    report("offsets_null", qmc_sample_offsets(&ctx, nullptr, nullptr, 64, nullptr, ws, sizeof ws), INV);
    report("offsets_ws", qmc_sample_offsets(&ctx, nullptr, du, 1u << 20, reinterpret_cast<uint64_t*>(du), ws, 8), WSP);
    qmc_sampler pts = sp;
    pts.kind = QMC_SAMPLER_POINTS;
    report("samples_points",
           qmc_generate_pixel_samples(&ctx, nullptr, &pts, 8, 8, 8, du, reinterpret_cast<uint64_t*>(du), df, 64, ws,
                                      sizeof ws),
           INV);
    report("samples_d0",
           qmc_generate_pixel_samples(&ctx, nullptr, &sp, 0, 8, 8, du, reinterpret_cast<uint64_t*>(du), df, 64, ws,
                                      sizeof ws),
           OOR);
    report("progressive_passes",
           qmc_integrate_progressive(&ctx, nullptr, &sp, &genz, 8, 8, du, 0, 64, df, df, ws, sizeof ws, 1), OOR);
    report("progressive_range",
           qmc_integrate_progressive(&ctx, nullptr, &sp, &genz, 8, 8, du, 1u << 16, 1u << 16, df, df, ws, sizeof ws, 1),
           OOR);

    // ------------------------------------------------------------ tuning files ----
    report("tune_save", qmc_tune_save(&ctx, tune_file(dir, "saved.json", "").c_str()), OK);
    report("tune_load_saved", qmc_tune_load(&ctx, (std::string(dir) + "/saved.json").c_str()), OK);
    report("tune_load_missing", qmc_tune_load(&ctx, (std::string(dir) + "/absent.json").c_str()), INV);
    report("tune_load_empty", qmc_tune_load(&ctx, tune_file(dir, "empty.json", "").c_str()), INV);
    report("tune_load_truncated",
           qmc_tune_load(&ctx, tune_file(dir, "trunc.json", "{\"sobol\": {\"chunks_per_wave\":").c_str()), OK);
    report("tune_load_huge",
           qmc_tune_load(&ctx, tune_file(dir, "huge.json",
                                         "{\"sobol\": {\"chunks_per_wave\": 99999999999999999999, \"nontemporal\": -7},"
                                         " \"integrate\": [{\"key\": 4294967296, \"waves_per_cu\": 0, \"dynamic\": 1},"
                                         " {\"key\": 18, \"waves_per_cu\": 8, \"dynamic\":")
                                   .c_str()),
           OK);
    report("tune_load_garbage",
           qmc_tune_load(&ctx, tune_file(dir, "garbage.json", "\"sobol\"\"integrate\"\"key\":}}}}\"key\"").c_str()), OK);
    report("tune_load_null", qmc_tune_load(&ctx, nullptr), INV);
    std::printf("sobol_tune %u %u\n", ctx.sobol_tune.chunks_per_wave, ctx.sobol_tune.nontemporal);
    std::printf("failures %d\n", failures);
    return failures ? 1 : 0;
}
