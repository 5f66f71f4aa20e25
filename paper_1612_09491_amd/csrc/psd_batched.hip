// psd_batched.hip -- many independent boxes in one persistent launch, and the
// autotuner that picks its launch shape.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "psd.h"
#include "psd_internal.h"

namespace psd {

namespace {

__global__ void fill_f32_kernel(float* p, int64_t n, float v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void fill_f64_kernel(double* p, int64_t n, double v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

std::mutex g_cache_mutex;

}  // namespace

std::vector<BoxDesc> batch_descs(const psd_box* boxes, int n, double* mass_sums, bool density)
{
    std::vector<BoxDesc> d((size_t)n);
    for (int b = 0; b < n; ++b) {
        const psd_box& B = boxes[b];
        BoxDesc& x = d[(size_t)b];
        memset(&x, 0, sizeof(x));
        x.pos = B.pos;
        for (int a = 0; a < 3; ++a) {
            x.np[a] = B.p.np[a];
            x.nc[a] = B.nc[a];
            x.scale[a] = (double)B.nc[a] / B.p.box;
        }
        x.ntet = 6 * (int64_t)B.p.np[0] * B.p.np[1] * B.p.np[2];
        x.m = B.p.total_mass / (6.0 * (double)B.p.np[0] * (double)B.p.np[1] * (double)B.p.np[2]);
        x.out_scale = density ? (double)B.nc[0] * B.nc[1] * B.nc[2] / (B.p.box * B.p.box * B.p.box) : 1.0;
        x.out = B.out;
        x.mass_sum = mass_sums ? mass_sums + b : nullptr;
    }
    return d;
}

hipError_t launch_batched(const psd_box* boxes, int n, double* mass_sums, bool density,
                          bool accumulate, const Tuning& tune, void* ws, size_t ws_bytes,
                          unsigned long long* stats, hipStream_t stream)
{
    const std::vector<BoxDesc> d = batch_descs(boxes, n, mass_sums, density);
    if (!accumulate) {
        for (int b = 0; b < n; ++b) {
            const int64_t cells = (int64_t)boxes[b].nc[0] * boxes[b].nc[1] * boxes[b].nc[2];
            const int64_t want = (cells + 255) / 256;
            hipLaunchKernelGGL(fill_f32_kernel, dim3((unsigned)(want < 65536 ? want : 65536)), dim3(256), 0,
                               stream, boxes[b].out, cells, 0.0f);
        }
        if (mass_sums)
            hipLaunchKernelGGL(fill_f64_kernel, dim3(1), dim3(256), 0, stream, mass_sums, (int64_t)n, 0.0);
    }
    return launch_queue(d.data(), n, false, tune, ws, ws_bytes, stats, stream);
}

size_t batched_ws_bytes(const psd_box* boxes, int n, bool ordered)
{
    int64_t chunks = 0;
    for (int b = 0; b < n; ++b) chunks += (6 * (int64_t)boxes[b].p.np[0] * boxes[b].p.np[1] * boxes[b].p.np[2] + 63) / 64;
    return queue_workspace_bytes(chunks, n, ordered);
}

// ---------------------------------------------------------------------------
// Autotuner cache: a flat JSON object {"<key>": {"lds_cap": c, "waves_per_cu":
// w, "ordered": o, "ms": t}, ...}, keyed by device name and batch signature.
// ---------------------------------------------------------------------------

static bool cache_lookup(const char* path, const std::string& key, Tuning& t, double& ms)
{
    FILE* f = fopen(path, "rb");
    if (!f) return false;
    std::string text;
    char buf[4096];
    size_t n;
    while ((n = fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, n);
    fclose(f);
    const std::string needle = "\"" + key + "\"";
    const size_t at = text.find(needle);
    if (at == std::string::npos) return false;
    const size_t open = text.find('{', at);
    const size_t close = text.find('}', at);
    if (open == std::string::npos || close == std::string::npos || close < open) return false;
    const std::string obj = text.substr(open, close - open + 1);
    int c = 0, w = 0, o = 0;
    double m = 0.0;
    auto num = [&](const char* name, double& v) {
        const size_t p = obj.find(std::string("\"") + name + "\"");
        if (p == std::string::npos) return false;
        const size_t colon = obj.find(':', p);
        if (colon == std::string::npos) return false;
        v = atof(obj.c_str() + colon + 1);
        return true;
    };
    double dc, dw, dord;
    if (!num("lds_cap", dc) || !num("waves_per_cu", dw) || !num("ordered", dord) || !num("ms", m))
        return false;
    c = (int)dc;
    w = (int)dw;
    o = (int)dord;
    if (!(c == 512 || c == 960 || c == 1024 || c == 1408 || c == 2048) || w < 1 || w > 64) return false;
    t.cap = c;
    t.waves_per_cu = w;
    t.ordered = o ? 1 : 0;
    ms = m;
    return true;
}

static void cache_store(const char* path, const std::string& key, const Tuning& t, double ms)
{
    std::string text;
    if (FILE* f = fopen(path, "rb")) {
        char buf[4096];
        size_t n;
        while ((n = fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, n);
        fclose(f);
    }
    char entry[512];
    snprintf(entry, sizeof(entry),
             "  \"%s\": {\"lds_cap\": %d, \"waves_per_cu\": %d, \"ordered\": %d, \"ms\": %.6f}",
             key.c_str(), t.cap, t.waves_per_cu, t.ordered, ms);
    const size_t last = text.rfind('}');
    std::string out;
    if (last == std::string::npos || text.find('"') == std::string::npos) {
        out = std::string("{\n") + entry + "\n}\n";
    } else {
        std::string head = text.substr(0, last);
        while (!head.empty() && (head.back() == '\n' || head.back() == ' ')) head.pop_back();
        out = head + ",\n" + entry + "\n}\n";
    }
    const std::string tmp = std::string(path) + ".tmp";
    if (FILE* f = fopen(tmp.c_str(), "wb")) {
        fwrite(out.data(), 1, out.size(), f);
        fclose(f);
        rename(tmp.c_str(), path);
    }
}

std::string batch_signature(const psd_box* boxes, int n, uint32_t flags)
{
    hipDeviceProp_t prop;
    int dev = 0;
    std::string name = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        name = prop.gcnArchName;
    double tets = 0, cells = 0, spread = 0;
    for (int b = 0; b < n; ++b) {
        const double nt = 6.0 * boxes[b].p.np[0] * boxes[b].p.np[1] * boxes[b].p.np[2];
        const double nc = (double)boxes[b].nc[0] * boxes[b].nc[1] * boxes[b].nc[2];
        tets += nt;
        cells += nc;
        spread += nt * log2(1.0 + nc / nt);  // cells per tetrahedron, weighted
    }
    char sig[256];
    snprintf(sig, sizeof(sig), "%s|boxes=%d|tets=%.0f|cells=%.0f|spread=%.4f|flags=%u", name.c_str(), n,
             tets, cells, tets > 0 ? spread / tets : 0.0, flags);
    return sig;
}

hipError_t autotune_batched(const psd_box* boxes, int n, uint32_t flags, void* ws, size_t ws_bytes,
                            hipStream_t stream, const char* cache_path, Tuning& best, double& best_ms)
{
    const std::string key = batch_signature(boxes, n, flags);
    if (cache_path) {
        std::lock_guard<std::mutex> lock(g_cache_mutex);
        if (cache_lookup(cache_path, key, best, best_ms)) return hipSuccess;
    }
    const bool density = (flags & PSD_OUT_DENSITY) != 0;
    const int caps[3] = {960, 1024, 2048};
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess) return e;
    e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        (void)hipEventDestroy(e0);
        return e;
    }
    best = default_tuning();
    best_ms = INFINITY;
    // warm-up with the default shape
    e = launch_batched(boxes, n, nullptr, density, false, best, ws, ws_bytes, nullptr, stream);
    for (int ord = 0; ord < 2 && e == hipSuccess; ++ord)
        for (int ci = 0; ci < 3 && e == hipSuccess; ++ci)
            for (int wi = 0; wi < 2 && e == hipSuccess; ++wi) {
                Tuning t = default_tuning();
                t.cap = caps[ci];
                int fit = 1;
                e = queue_resident_waves(t.cap, false, fit);
                if (e != hipSuccess) break;
                t.waves_per_cu = wi == 0 ? fit : (fit + 1) / 2;
                t.ordered = ord;
                e = hipEventRecord(e0, stream);
                if (e != hipSuccess) break;
                e = launch_batched(boxes, n, nullptr, density, false, t, ws, ws_bytes, nullptr, stream);
                if (e != hipSuccess) break;
                e = hipEventRecord(e1, stream);
                if (e != hipSuccess) break;
                e = hipEventSynchronize(e1);
                if (e != hipSuccess) break;
                float ms = 0.0f;
                e = hipEventElapsedTime(&ms, e0, e1);
                if (e == hipSuccess && ms < best_ms) {
                    best_ms = ms;
                    best = t;
                }
            }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return e;
    if (cache_path) {
        std::lock_guard<std::mutex> lock(g_cache_mutex);
        cache_store(cache_path, key, best, best_ms);
    }
    return hipSuccess;
}

}  // namespace psd
