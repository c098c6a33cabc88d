// C ABI of alphacirc: tiling control and the tile tuner.
#include "host.h"

using namespace ach;

// ---------------------------------------------------------------------------
// tiling control (used by the tile tuner)
int ac_ctx_set_shift_groups(ac_ctx* c, int mode) {
    if (!c) return fail(AC_ERR_ARG, "ctx is NULL");
    if (mode < -1 || mode > 1) return fail(AC_ERR_ARG, "mode must be -1, 0 or 1");
    c->shift_groups = mode;
    return AC_OK;
}

int ac_ctx_set_step_triples(ac_ctx* c, int mode, int rows_per_wave, int waves_per_simd, int points_per_lane) {
    if (!c) return fail(AC_ERR_ARG, "ctx is NULL");
    if (mode < 0 || mode > 1) return fail(AC_ERR_ARG, "mode must be 0 or 1");
    if (rows_per_wave < 0 || rows_per_wave > 4096) return fail(AC_ERR_ARG, "rows_per_wave out of range");
    if (waves_per_simd < 0 || waves_per_simd > 8) return fail(AC_ERR_ARG, "waves_per_simd must be 0..8");
    if (points_per_lane < 0 || points_per_lane > 2) return fail(AC_ERR_ARG, "points_per_lane must be 0..2");
    c->triples = mode;
    c->triple_h = rows_per_wave;
    c->triple_occ = waves_per_simd > 0 ? waves_per_simd : 4;
    c->triple_vx = points_per_lane;
    return AC_OK;
}

int ac_ctx_set_step_pairs(ac_ctx* c, int mode, int rows_per_wave, int waves_per_block, int points_per_lane) {
    if (!c) return fail(AC_ERR_ARG, "ctx is NULL");
    if (mode < 0 || mode > 1) return fail(AC_ERR_ARG, "mode must be 0 or 1");
    if (rows_per_wave < 0 || rows_per_wave > 4096) return fail(AC_ERR_ARG, "rows_per_wave out of range");
    if (waves_per_block < 0 || waves_per_block > 4) return fail(AC_ERR_ARG, "waves_per_block must be 0..4");
    if (points_per_lane < 0 || points_per_lane > 2) return fail(AC_ERR_ARG, "points_per_lane must be 0..2");
    c->pairs = mode;
    c->pair_h = rows_per_wave;
    c->pair_wpb = waves_per_block;
    c->pair_vx = points_per_lane;
    return AC_OK;
}

int ac_ctx_set_tiling(ac_ctx* c, int rows_per_wave, int waves_per_block, int points_per_lane) {
    if (!c) return fail(AC_ERR_ARG, "ctx is NULL");
    if (rows_per_wave < 0 || rows_per_wave > 4096) return fail(AC_ERR_ARG, "rows_per_wave out of range");
    if (waves_per_block < 0 || waves_per_block > 4) return fail(AC_ERR_ARG, "waves_per_block must be 0..4");
    if (points_per_lane < 0 || points_per_lane > 2) return fail(AC_ERR_ARG, "points_per_lane must be 0..2");
    c->tile_h = rows_per_wave;
    c->tile_wpb = waves_per_block;
    c->tile_vx = points_per_lane;
    return AC_OK;
}

// ---------------------------------------------------------------------------
// Tile tuner: times the Chebyshev sweeps of one problem for candidate tilings and
// keeps the fastest; choices are cached in a small JSON file, one entry per line.

namespace {

struct TileEntry {
    int nx, ny, ell, prec, h, wpb, vx;
    double us;
};

const char* kTileFmt =
    "{\"nx\": %d, \"ny\": %d, \"ell\": %d, \"prec\": %d, \"rows_per_wave\": %d, \"waves_per_block\": %d, "
    "\"points_per_lane\": %d, \"us\": %lf}";

std::vector<TileEntry> read_tile_cache(const char* path) {
    std::vector<TileEntry> out;
    FILE* f = std::fopen(path, "r");
    if (!f) return out;
    char line[512];
    while (std::fgets(line, sizeof line, f)) {
        const char* brace = std::strchr(line, '{');
        if (!brace || std::strstr(line, "alphacirc_tiling")) continue;  // the header line
        TileEntry e{};
        if (std::sscanf(brace, kTileFmt, &e.nx, &e.ny, &e.ell, &e.prec, &e.h, &e.wpb, &e.vx, &e.us) == 8)
            out.push_back(e);
    }
    std::fclose(f);
    return out;
}

int write_tile_cache(const char* path, const std::vector<TileEntry>& es) {
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return fail(AC_ERR_ARG, std::string("cannot write tiling cache ") + tmp);
    std::fprintf(f, "{\"alphacirc_tiling\": [\n");
    for (size_t i = 0; i < es.size(); ++i) {
        std::fprintf(f, "  ");
        std::fprintf(f, kTileFmt, es[i].nx, es[i].ny, es[i].ell, es[i].prec, es[i].h, es[i].wpb, es[i].vx, es[i].us);
        std::fprintf(f, i + 1 < es.size() ? ",\n" : "\n");
    }
    std::fprintf(f, "]}\n");
    std::fclose(f);
    if (std::rename(tmp.c_str(), path) != 0) return fail(AC_ERR_ARG, std::string("cannot replace ") + path);
    return AC_OK;
}

bool same_key(const TileEntry& e, const ac_problem* p, int prec) {
    return e.nx == p->g.nx && e.ny == p->g.ny && e.ell == p->ell && e.prec == prec;
}

}  // namespace

int ac_problem_set_tiling(ac_problem* p, int rows_per_wave, int waves_per_block, int points_per_lane) {
    if (!p) return fail(AC_ERR_ARG, "problem is NULL");
    if (rows_per_wave < 0 || rows_per_wave > 4096) return fail(AC_ERR_ARG, "rows_per_wave out of range");
    if (waves_per_block < 0 || waves_per_block > 4) return fail(AC_ERR_ARG, "waves_per_block must be 0..4");
    if (points_per_lane < 0 || points_per_lane > 2) return fail(AC_ERR_ARG, "points_per_lane must be 0..2");
    p->tile_h = rows_per_wave;
    p->tile_wpb = waves_per_block;
    p->tile_vx = points_per_lane;
    return AC_OK;
}

int ac_tune_tiling(ac_problem* p, int prec, const char* cache_path, void* ws, size_t ws_bytes, int* out,
                   double* us_out) {
    if (!p) return fail(AC_ERR_ARG, "problem is NULL");
    if (prec < 0 || prec > 2) return fail(AC_ERR_ARG, "unknown precision");
    auto report = [&](const Tiling& t, double us) {
        if (out) {
            out[0] = t.h;
            out[1] = t.wpb;
            out[2] = t.vx;
        }
        if (us_out) *us_out = us;
    };
    std::vector<TileEntry> cache;
    if (cache_path) {
        cache = read_tile_cache(cache_path);
        for (const TileEntry& e : cache)
            if (same_key(e, p, prec)) {
                AC_TRY(ac_problem_set_tiling(p, e.h, e.wpb, e.vx));
                report(sweep_tiling(p), 0.0);
                return AC_OK;
            }
    }
    if (!ws || ws_bytes < prec_ws_bytes(p, prec)) return fail(AC_ERR_WORKSPACE, "workspace too small");
    AC_HIP(hipSetDevice(p->ctx->device));
    ac_ctx* c = p->ctx;
    const bool prof = c->profiling;
    c->profiling = false;
    const PrecBufs bufs = carve_prec(p, prec, ws);
    {
        const long long words = static_cast<long long>(prec_ws_bytes(p, prec) - 256) / 8;
        AC_HIP(launch_zero(reinterpret_cast<double*>(bufs.rhat), words, c->stream));
    }
    constexpr int kSteps = 8;  // one sweep from x_1 = rhat/theta, then steady sweeps
    const std::vector<int> pm(p->ell, kSteps);
    hipEvent_t e0, e1;
    AC_HIP(hipEventCreate(&e0));
    AC_HIP(hipEventCreate(&e1));
    const int keep_h = p->tile_h, keep_wpb = p->tile_wpb, keep_vx = p->tile_vx;
    double best = 1e300;
    int bh = 0, bw = 0, bv = 0;
    std::vector<std::array<int, 3>> seen;
    int status = AC_OK;
    for (int vx : {2, 1}) {
        for (int h : {4, 8, 16, 32, 64}) {
            for (int wpb : {1, 2, 4}) {
                p->tile_h = h;
                p->tile_wpb = wpb;
                p->tile_vx = vx;
                const Tiling t = sweep_tiling(p);
                const std::array<int, 3> key{t.h, t.wpb, t.vx};
                if (std::find(seen.begin(), seen.end(), key) != seen.end()) continue;
                seen.push_back(key);
                double ms_best = 1e300;
                for (int rep = 0; rep < 4 && status == AC_OK; ++rep) {
                    if (hipEventRecord(e0, c->stream) != hipSuccess) {
                        status = fail(AC_ERR_HIP, "tile tuner: hipEventRecord failed");
                        break;
                    }
                    status = run_cheb(p, prec, pm, bufs.rhat, bufs.buf, false, nullptr, nullptr);
                    if (status != AC_OK) break;
                    if (hipEventRecord(e1, c->stream) != hipSuccess) {
                        status = fail(AC_ERR_HIP, "tile tuner: hipEventRecord failed");
                        break;
                    }
                    if (hipEventSynchronize(e1) != hipSuccess) {
                        status = fail(AC_ERR_HIP, "tile tuner: event synchronisation failed");
                        break;
                    }
                    float ms = 0.f;
                    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                        status = fail(AC_ERR_HIP, "tile tuner: hipEventElapsedTime failed");
                        break;
                    }
                    if (rep > 0) ms_best = std::min(ms_best, static_cast<double>(ms));
                }
                if (status != AC_OK) break;
                if (ms_best < best) {
                    best = ms_best;
                    bh = t.h;
                    bw = t.wpb;
                    bv = t.vx;
                }
            }
            if (status != AC_OK) break;
        }
        if (status != AC_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->profiling = prof;
    if (status != AC_OK) {
        p->tile_h = keep_h;
        p->tile_wpb = keep_wpb;
        p->tile_vx = keep_vx;
        return status;
    }
    AC_TRY(ac_problem_set_tiling(p, bh, bw, bv));
    const double us = 1000.0 * best / (kSteps - 1);
    report(sweep_tiling(p), us);
    if (cache_path) {
        cache.push_back(TileEntry{p->g.nx, p->g.ny, p->ell, prec, bh, bw, bv, us});
        AC_TRY(write_tile_cache(cache_path, cache));
    }
    return AC_OK;
}
