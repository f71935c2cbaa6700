// Autotuner for the launch configurations of plans and batches.
//
// For every stage it times each candidate (lanes per ray of the forward
// projector and where it reads its taps, the backprojector's form, block and
// view-splitting wavefronts, TV tile) on synthetic data of the stage's real shape with
// HIP events, keeps the fastest candidate whose output agrees with the default
// configuration's (relative L2 difference at most 1e-5; candidates differ only
// in summation order), and stores it in the plan or batch. Results are cached
// in a text file, one line per (device, geometry, stage, view selection):
//   <key> <fp_seg> <bp_px> <bp_vg> <tv_tile> <fp_lds>
// (a line without fp_lds reads as fp_lds = 1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <functional>
#include <set>
#include <sstream>
#include <string>
#include <vector>

#include "batch.h"
#include "fbpnp_impl.h"

using namespace fbpnp;

namespace {

constexpr int kWarm = 2, kReps = 8, kRounds = 5;
constexpr double kAgree = 1e-5;
constexpr float kMargin = 0.03f;  // a candidate replaces the default only if >= 3 % faster

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    fb_status alloc(size_t n) {
        if (hipMalloc(&p, std::max<size_t>(n, 4)) != hipSuccess) return fail(FB_ENOMEM, "autotune: allocation");
        bytes = n;
        return FB_OK;
    }
    float* f() const { return (float*)p; }
};

// Host-side check, before the launches that use it, that a scratch buffer
// holds what they read or write (floats).
fb_status need(const DevBuf& d, size_t floats, const char* what) {
    if (d.bytes >= floats * sizeof(float)) return FB_OK;
    return fail(FB_EINVAL, std::string("autotune: scratch buffer too small for ") + what);
}

// Smooth deterministic test data in [0, 1): a sum of two products of sines.
std::vector<float> pattern(size_t n, int period, float phase) {
    std::vector<float> v(n);
    for (size_t i = 0; i < n; ++i) {
        const double a = (double)(i % period) / period, b = (double)(i / period) / period;
        v[i] = (float)(0.5 + 0.25 * std::sin(6.1 * a + phase) * std::sin(4.3 * b) + 0.2 * std::sin(17.0 * a * b));
    }
    return v;
}

fb_status upload(float* d, const std::vector<float>& h) {
    hipError_t e = hipMemcpy(d, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice);
    return e == hipSuccess ? FB_OK : hip_fail(e, "autotune: upload");
}

fb_status download(std::vector<float>& h, const float* d, size_t n) {
    h.resize(n);
    hipError_t e = hipMemcpy(h.data(), d, n * sizeof(float), hipMemcpyDeviceToHost);
    return e == hipSuccess ? FB_OK : hip_fail(e, "autotune: download");
}

double rel_l2(const std::vector<float>& a, const std::vector<float>& b) {
    double num = 0, den = 0;
    for (size_t i = 0; i < a.size(); ++i) {
        const double d = (double)a[i] - (double)b[i];
        num += d * d;
        den += (double)b[i] * b[i];
    }
    if (!std::isfinite(num)) return INFINITY;
    return den > 0 ? std::sqrt(num / den) : std::sqrt(num);
}

// Mean time (ms) of kReps calls of run after kWarm untimed ones.
fb_status time_ms(const std::function<fb_status()>& run, hipStream_t s, float* ms) {
    fb_status st;
    for (int i = 0; i < kWarm; ++i)
        if ((st = run()) != FB_OK) return st;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return fail(FB_EHIP, "autotune: event");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(FB_EHIP, "autotune: event");
    }
    st = FB_OK;
    if (hipEventRecord(e0, s) != hipSuccess) st = fail(FB_EHIP, "autotune: event record");
    for (int i = 0; i < kReps && st == FB_OK; ++i) st = run();
    if (st == FB_OK && hipEventRecord(e1, s) != hipSuccess) st = fail(FB_EHIP, "autotune: event record");
    if (st == FB_OK && hipEventSynchronize(e1) != hipSuccess) st = fail(FB_EHIP, "autotune: event sync");
    float t = 0.f;
    if (st == FB_OK && hipEventElapsedTime(&t, e0, e1) != hipSuccess) st = fail(FB_EHIP, "autotune: elapsed");
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = t / kReps;
    return st;
}

// The fastest candidate whose output agrees with the first one's (the
// default). Each candidate's time is the median of kRounds rounds, the rounds
// interleaved over the candidates so that clock or thermal drift affects all
// alike; another candidate replaces the default only when it is at least
// kMargin faster.
template <typename Cand>
fb_status pick(const std::vector<Cand>& cands, const std::function<fb_status(const Cand&)>& run,
               const std::function<fb_status(std::vector<float>&)>& read, hipStream_t s, Cand* best) {
    const size_t n = cands.size();
    std::vector<char> ok(n, 1);
    std::vector<float> ref, out;
    for (size_t i = 0; i < n; ++i) {  // agreement with the default
        fb_status st = run(cands[i]);
        if (st != FB_OK) return st;
        if (hipStreamSynchronize(s) != hipSuccess) return fail(FB_EHIP, "autotune: sync");
        if ((st = read(i == 0 ? ref : out)) != FB_OK) return st;
        if (i > 0) ok[i] = rel_l2(out, ref) <= kAgree;  // disagreeing candidates are never chosen
    }
    std::vector<std::vector<float>> t(n);
    for (int round = 0; round < kRounds; ++round)
        for (size_t i = 0; i < n; ++i) {
            if (!ok[i]) continue;
            float ms;
            fb_status st = time_ms([&] { return run(cands[i]); }, s, &ms);
            if (st != FB_OK) return st;
            t[i].push_back(ms);
        }
    auto median = [](std::vector<float> v) {
        std::sort(v.begin(), v.end());
        return v[v.size() / 2];
    };
    const float t0 = median(t[0]);
    float best_ms = t0 * (1.f - kMargin);
    *best = cands[0];
    for (size_t i = 1; i < n; ++i) {
        if (!ok[i]) continue;
        const float m = median(t[i]);
        if (m < best_ms) {
            best_ms = m;
            *best = cands[i];
        }
    }
    return FB_OK;
}

std::string device_tag() {
    int dev = 0;
    hipDeviceProp_t prop{};
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::ostringstream o;
    o << prop.gcnArchName << "/" << prop.multiProcessorCount;
    std::string t = o.str();
    for (char& c : t)
        if (c == ' ' || c == ':') c = '_';
    return t;
}

uint64_t fnv1a(const void* data, size_t n, uint64_t h = 1469598103934665603ull) {
    const unsigned char* p = (const unsigned char*)data;
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 1099511628211ull;
    }
    return h;
}

uint64_t geom_hash(const fb_geom& g, uint64_t h) {
    const double v[] = {(double)g.nx, (double)g.ny, g.pixel_mm, (double)g.n_views, (double)g.n_bins, g.sod_mm,
                        g.sdd_mm, g.det_pitch_mm, g.det_offset_mm, g.angle0_rad, g.angle_step_rad};
    return fnv1a(v, sizeof(v), h);
}

bool cache_get(const char* path, const std::string& key, fb_launch_config* c) {
    if (!path) return false;
    std::ifstream in(path);
    std::string line;
    bool found = false;
    while (std::getline(in, line)) {  // the last entry for a key wins
        std::istringstream ls(line);
        std::string k;
        fb_launch_config v{};
        if (ls >> k >> v.fp_seg >> v.bp_px >> v.bp_vg >> v.tv_tile && k == key && v.fp_seg && v.bp_px && v.bp_vg &&
            v.tv_tile) {
            if (!(ls >> v.fp_lds)) v.fp_lds = 1;  // lines written before the field existed
            if (check_config(v) == FB_OK && v.fp_lds) {
                *c = v;
                found = true;
            }
        }
    }
    return found;
}

void cache_put(const char* path, const std::string& key, const fb_launch_config& c) {
    if (!path) return;
    std::ofstream out(path, std::ios::app);
    out << key << " " << c.fp_seg << " " << c.bp_px << " " << c.bp_vg << " " << c.tv_tile << " " << c.fp_lds << "\n";
}

std::vector<std::pair<int, int>> bp_candidates(int n_sel_min) {
    std::vector<std::pair<int, int>> c;
    // gather form: pixels per lane 1, 2, 4
    for (int px : {1, 2, 4})
        for (int vg : {1, 2, 4, 8, 16})
            if ((px < 4 || vg <= 4) && vg <= std::max(1, n_sel_min)) c.push_back({px, vg});
    // scatter form: block sides 16 and 32 (it pays only with several wavefronts per block)
    for (int b : {16, 32})
        for (int vg : {4, 8, 16})
            if (vg <= std::max(1, n_sel_min)) c.push_back({b, vg});
    return c;
}

std::vector<int> tv_candidates(const std::vector<int>& factors) {
    std::vector<int> c;
    for (int t : {32, 16}) {
        bool ok = true;
        for (int f : factors) ok = ok && t % f == 0;
        if (ok) c.push_back(t);
    }
    return c;
}

}  // namespace

static fb_status autotune_plan(fb_plan* p, int n_sel, const char* cache_path, hipStream_t s) {
    fb_status st = check_stage(p, 0);
    if (st != FB_OK) return st;
    const int V = p->g.n_views, nb = p->g.n_bins, nx = p->g.nx, ny = p->g.ny;
    if (n_sel < 1 || n_sel > V) return fail(FB_EINVAL, "fb_autotune: need 1 <= n_sel <= n_views");
    const size_t npix = (size_t)nx * ny;
    std::vector<int> factors;
    for (const Stage& S : p->stages) factors.push_back(S.f);
    // n_sel views spread evenly over the scan, as an interleaved subset is
    std::vector<int32_t> hv(n_sel);
    for (int i = 0; i < n_sel; ++i) hv[i] = (int32_t)(((long)i * V) / n_sel);
    // proj: a projection of the selected views [n_sel][nb]; out: an image [ny][nx]
    const size_t nproj = (size_t)n_sel * nb;
    DevBuf views, img, sino, b, proj, out, yprev, xprev;
    if ((st = views.alloc(n_sel * sizeof(int32_t))) != FB_OK || (st = img.alloc(npix * 4)) != FB_OK ||
        (st = sino.alloc(nproj * 4)) != FB_OK || (st = b.alloc((size_t)V * nb * 4)) != FB_OK ||
        (st = proj.alloc(nproj * 4)) != FB_OK || (st = out.alloc(npix * 4)) != FB_OK ||
        (st = yprev.alloc(npix * 4)) != FB_OK || (st = xprev.alloc(npix * 4)) != FB_OK)
        return st;
    if (hipMemcpy(views.p, hv.data(), hv.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
        return fail(FB_EHIP, "autotune: upload");
    if ((st = upload(img.f(), pattern(npix, nx, 0.3f))) != FB_OK ||
        (st = upload(sino.f(), pattern((size_t)n_sel * nb, nb, 1.1f))) != FB_OK ||
        (st = upload(b.f(), pattern((size_t)V * nb, nb, 2.0f))) != FB_OK ||
        (st = upload(yprev.f(), pattern(npix, nx, 0.7f))) != FB_OK ||
        (st = upload(xprev.f(), pattern(npix, nx, 0.9f))) != FB_OK)
        return st;
    const int32_t* vp = n_sel == V ? nullptr : (const int32_t*)views.p;
    char gkey[32];
    std::snprintf(gkey, sizeof gkey, "%016llx", (unsigned long long)geom_hash(p->g, 1469598103934665603ull));
    for (int k = 0; k < (int)p->stages.size(); ++k) {
        const Stage& S = p->stages[k];
        const std::string key = "plan:" + device_tag() + ":" + gkey + ":f" + std::to_string(S.f) + ":sel" +
                                std::to_string(n_sel);
        fb_launch_config best{};
        if (cache_get(cache_path, key, &best)) {
            p->cfg[k] = best;
            continue;
        }
        const size_t ncoarse = (size_t)S.nxs * S.nys;
        // what the candidate launches below read and write
        if ((st = need(img, npix, "the image pooled into the line images")) != FB_OK ||
            (st = need(b, (size_t)V * nb, "the data b")) != FB_OK ||
            (st = need(proj, nproj, "the residual projection")) != FB_OK ||
            (st = need(sino, nproj, "the back-projected sinogram")) != FB_OK ||
            (st = need(yprev, npix, "y_prev")) != FB_OK || (st = need(out, ncoarse, "the coarse gradient")) != FB_OK ||
            (st = need(out, npix, "the denoised image")) != FB_OK || (st = need(xprev, npix, "x_prev")) != FB_OK ||
            (st = need(views, (size_t)n_sel, "the view list")) != FB_OK)
            return st;
        p->cfg[k] = fb_launch_config{0, 0, 0, 0, 0};
        const fb_launch_config def = plan_config(p, k, n_sel);
        if ((st = launch_prepare(p, k, img.f(), nx, S.f, s)) != FB_OK) return st;
        // forward projection (residual form, as in the iteration): lanes per
        // ray, and taps from global memory or (where the stage fits) from LDS
        std::vector<std::pair<int, int>> fps = {{def.fp_seg, def.fp_lds}};
        for (int lds : {1, 2})
            for (int v : {1, 2, 4, 8})
                if ((lds == 1 || fp_lds_fits(p, k)) && std::make_pair(v, lds) != fps[0]) fps.push_back({v, lds});
        std::pair<int, int> fpc = fps[0];
        st = pick<std::pair<int, int>>(
            fps,
            [&](const std::pair<int, int>& c) {
                p->cfg[k].fp_seg = c.first;
                p->cfg[k].fp_lds = c.second;
                return launch_fp(p, k, true, ViewSel{vp, n_sel}, b.f(), proj.f(), s);
            },
            [&](std::vector<float>& h) { return download(h, proj.f(), nproj); }, s, &fpc);
        if (st != FB_OK) return st;
        p->cfg[k].fp_seg = fpc.first;
        p->cfg[k].fp_lds = fpc.second;
        // backprojection: the fused form is timed, the plain gradient compared
        std::vector<std::pair<int, int>> bps = {{def.bp_px, def.bp_vg}};
        for (auto c : bp_candidates(n_sel))
            if (c != bps[0]) bps.push_back(c);
        std::pair<int, int> bpc = bps[0];
        st = pick<std::pair<int, int>>(
            bps,
            [&](const std::pair<int, int>& c) {
                p->cfg[k].bp_px = c.first;
                p->cfg[k].bp_vg = c.second;
                return launch_bp(p, k, sino.f(), ViewSel{vp, n_sel}, 1e-3f, nullptr, yprev.f(), p->zbuf, true, s);
            },
            [&](std::vector<float>& h) {
                fb_status r = launch_bp(p, k, sino.f(), ViewSel{vp, n_sel}, 1.f, out.f(), nullptr, nullptr, false, s);
                if (r == FB_OK && hipStreamSynchronize(s) != hipSuccess) r = fail(FB_EHIP, "autotune: sync");
                return r == FB_OK ? download(h, out.f(), ncoarse) : r;
            },
            s, &bpc);
        if (st != FB_OK) return st;
        p->cfg[k].bp_px = bpc.first;
        p->cfg[k].bp_vg = bpc.second;
        // TV-prox with relaxation and momentum at full resolution
        std::vector<int> tiles = {def.tv_tile};
        for (int t : tv_candidates(factors))
            if (t != def.tv_tile) tiles.push_back(t);
        int tile = def.tv_tile;
        st = pick<int>(
            tiles,
            [&](const int& t) {
                return launch_tv_single(yprev.f(), nx, ny, 0.01f, 0.125f, 5, nullptr, nullptr, 1, 1.f, 0.5f,
                                        xprev.f(), out.f(), img.f(), nullptr, s, PoolTarget(), t);
            },
            [&](std::vector<float>& h) { return download(h, out.f(), npix); }, s, &tile);
        if (st != FB_OK) return st;
        p->cfg[k].tv_tile = tile;
        cache_put(cache_path, key, p->cfg[k]);
    }
    return hipStreamSynchronize(s) == hipSuccess ? FB_OK : fail(FB_EHIP, "autotune: sync");
}

static fb_status autotune_batch(fb_batch* B, int n_sub, const char* cache_path, hipStream_t s) {
    n_sub = std::max(1, n_sub);
    BuildScope scope(B);  // candidates launch with work lists of their own
    const int n = (int)B->h_desc.size();
    const int64_t img_n = B->img_off.back(), sino_n = B->sino_off.back();
    DevBuf img, b, eta, xo, yo, xp;
    fb_status st;
    if ((st = img.alloc(img_n * 4)) != FB_OK || (st = b.alloc(sino_n * 4)) != FB_OK ||
        (st = eta.alloc(n * 4)) != FB_OK || (st = xo.alloc(img_n * 4)) != FB_OK ||
        (st = yo.alloc(img_n * 4)) != FB_OK || (st = xp.alloc(img_n * 4)) != FB_OK)
        return st;
    if (hipMemset(xo.p, 0, img_n * 4) != hipSuccess) return fail(FB_EHIP, "autotune: memset");
    if ((st = upload(img.f(), pattern(img_n, 256, 0.3f))) != FB_OK ||
        (st = upload(b.f(), pattern(sino_n, 512, 1.3f))) != FB_OK ||
        (st = upload(xp.f(), pattern(img_n, 256, 0.8f))) != FB_OK ||
        (st = upload(eta.f(), std::vector<float>(n, 1e-4f))) != FB_OK)
        return st;
    uint64_t h = 1469598103934665603ull;
    for (fb_plan* p : B->plans) h = geom_hash(p->g, h);
    char gkey[32];
    std::snprintf(gkey, sizeof gkey, "%016llx", (unsigned long long)h);
    // every slice's residual rows and z image, gathered on the host
    auto gather = [&](bool resid, std::vector<float>& out) {
        out.clear();
        std::vector<float> part;
        for (const SliceDesc& D : B->h_desc) {
            const size_t m = resid ? (size_t)cdiv(D.n_views, n_sub) * D.n_bins : (size_t)D.nx * D.ny;
            fb_status r = download(part, resid ? D.resid : D.zbuf, m);
            if (r != FB_OK) return r;
            out.insert(out.end(), part.begin(), part.end());
        }
        return FB_OK;
    };
    for (int k = 0; k < B->n_stages; ++k) {
        const std::string key = "batch:" + device_tag() + ":" + gkey + ":n" + std::to_string(n) + ":f" +
                                std::to_string(B->factors[k]) + ":sub" + std::to_string(n_sub);
        fb_launch_config best{};
        if (cache_get(cache_path, key, &best)) {
            B->cfg[k] = best;
            continue;
        }
        // what the candidate launches below read and write (the residuals and z
        // images they write belong to the slice plans)
        if ((st = need(img, (size_t)img_n, "the image arena")) != FB_OK ||
            (st = need(b, (size_t)sino_n, "the sinogram arena")) != FB_OK ||
            (st = need(eta, (size_t)n, "the step sizes")) != FB_OK ||
            (st = need(xp, (size_t)img_n, "x_prev")) != FB_OK || (st = need(xo, (size_t)img_n, "x_out")) != FB_OK ||
            (st = need(yo, (size_t)img_n, "y_out")) != FB_OK)
            return st;
        B->cfg[k] = fb_launch_config{0, 0, 0, 0, 0};
        const fb_launch_config def = batch_config(B, k, n_sub);
        if ((st = launch_prepare_batch(B, k, img.f(), s)) != FB_OK) return st;
        std::vector<int> segs = {def.fp_seg};
        for (int v : {1, 2, 4, 8})
            if (v != def.fp_seg) segs.push_back(v);
        int seg = def.fp_seg;
        st = pick<int>(
            segs, [&](const int& c) { return launch_fp_batch(B, k, n_sub, 0, b.f(), c, s); },
            [&](std::vector<float>& o) { return gather(true, o); }, s, &seg);
        if (st != FB_OK) return st;
        B->cfg[k].fp_seg = seg;
        B->cfg[k].fp_lds = 1;
        int nsel_min = 1 << 30;
        for (const SliceDesc& D : B->h_desc) nsel_min = std::min(nsel_min, cdiv(D.n_views, n_sub));
        std::vector<std::pair<int, int>> bps = {{def.bp_px, def.bp_vg}};
        for (auto c : bp_candidates(nsel_min))
            if (c != bps[0]) bps.push_back(c);
        std::pair<int, int> bpc = bps[0];
        st = pick<std::pair<int, int>>(
            bps,
            [&](const std::pair<int, int>& c) {
                return launch_bp_batch(B, k, n_sub, 0, eta.f(), 1.f, xp.f(), c.first, c.second, s);
            },
            [&](std::vector<float>& o) { return gather(false, o); }, s, &bpc);
        if (st != FB_OK) return st;
        B->cfg[k].bp_px = bpc.first;
        B->cfg[k].bp_vg = bpc.second;
        std::vector<int> tiles = {def.tv_tile};
        for (int t : tv_candidates(B->factors))
            if (t != def.tv_tile) tiles.push_back(t);
        int tile = def.tv_tile;
        st = pick<int>(
            tiles,
            [&](const int& t) {
                return launch_tv_batch(B, -1, 0.01f, 0.125f, 5, 1.f, 0.5f, xp.f(), xo.f(), yo.f(), nullptr, t, s);
            },
            [&](std::vector<float>& o) { return download(o, xo.f(), img_n); }, s, &tile);
        if (st != FB_OK) return st;
        B->cfg[k].tv_tile = tile;
        cache_put(cache_path, key, B->cfg[k]);
    }
    return hipStreamSynchronize(s) == hipSuccess ? FB_OK : fail(FB_EHIP, "autotune: sync");
}

extern "C" {

fb_status fb_autotune(fb_plan* p, int n_sel, const char* cache_path, hipStream_t s) {
    fb_status st = check_stage(p, 0);
    if (st != FB_OK) return st;
    const std::vector<fb_launch_config> saved = p->cfg;
    st = autotune_plan(p, n_sel, cache_path, s);
    if (st != FB_OK) p->cfg = saved;  // a failed run leaves the configuration as it was
    return st;
}

fb_status fb_batch_autotune(fb_batch* B, int n_sub, const char* cache_path, hipStream_t s) {
    if (!B) return fail(FB_EINVAL, "fb_batch_autotune: batch is NULL");
    const std::vector<fb_launch_config> saved = B->cfg;
    fb_status st = autotune_batch(B, n_sub, cache_path, s);
    // steps with the tuned subset count, and with every count prepared before,
    // find their work lists under the chosen configuration
    std::set<int> counts = B->prepared;
    counts.insert(std::max(1, n_sub));
    for (int n : counts)
        if (st == FB_OK) st = ensure_tables(B, n);
    if (st != FB_OK) B->cfg = saved;
    return st;
}

}  // extern "C"
