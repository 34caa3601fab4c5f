// Autotuning of launch parameters (NTT pass split and tile, MAC and
// key-switch workgroup targets, key-switch group size).  Every candidate
// computes identical results; the tuner only times them.
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "internal.h"

namespace {

struct Buf {
    u64* p = nullptr;
    ~Buf() { (void)hipFree(p); }
    int alloc(size_t words)
    {
        if (hipMalloc(&p, sizeof(u64) * words) != hipSuccess) return uh_fail(UNIHENN_ENOMEM, "tuning buffers");
        return UNIHENN_OK;
    }
};

struct Events {
    hipEvent_t a = nullptr, b = nullptr;
    ~Events()
    {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
    int init()
    {
        UH_CHECK_HIP(hipEventCreate(&a));
        UH_CHECK_HIP(hipEventCreate(&b));
        return UNIHENN_OK;
    }
};

// mean milliseconds of `reps` runs of fn after one warm-up run; reps <= 0:
// as many runs (2..20) as fill about 40 ms, judged from the warm-up
template <class F>
int time_ms(hipStream_t s, int reps, F fn, double* ms)
{
    Events ev;
    int rc = ev.init();
    if (rc) return rc;
    UH_CHECK_HIP(hipEventRecord(ev.a, s));
    rc = fn();
    if (rc) return rc;
    UH_CHECK_HIP(hipEventRecord(ev.b, s));
    UH_CHECK_HIP(hipEventSynchronize(ev.b));
    if (reps <= 0) {
        float w = 0;
        UH_CHECK_HIP(hipEventElapsedTime(&w, ev.a, ev.b));
        reps = w > 0 ? (int)(40.0f / w) : 20;
        reps = reps < 2 ? 2 : (reps > 20 ? 20 : reps);
    }
    UH_CHECK_HIP(hipEventRecord(ev.a, s));
    for (int r = 0; r < reps; ++r) {
        rc = fn();
        if (rc) return rc;
    }
    UH_CHECK_HIP(hipEventRecord(ev.b, s));
    UH_CHECK_HIP(hipEventSynchronize(ev.b));
    float t = 0;
    UH_CHECK_HIP(hipEventElapsedTime(&t, ev.a, ev.b));
    *ms = t / reps;
    return UNIHENN_OK;
}

int ntt_rows(const unihenn_ctx* c, int batch)
{
    const long r = 8L * c->n_data * (batch > 0 ? batch : 1);
    return (int)std::min<long>(4096, std::max<long>(64, r));
}

int time_ntt(unihenn_ctx* c, u64* data, int rows, hipStream_t s, double* ms)
{
    const RowMap m = rowmap_ct(c->n_data);
    return time_ms(s, 3, [&]() {
        launch_ntt_fwd(c, data, rows, m, s);
        launch_ntt_inv(c, data, rows, m, s);
        UH_CHECK_HIP(hipGetLastError());
        return (int)UNIHENN_OK;
    }, ms);
}

// whole evaluations in the net's own mode; captured graphs are dropped first
// so that a graph mode records the current launch shapes (in the warm-up)
int time_net(unihenn_ctx* c, unihenn_net* net, int batch, u64* in, u64* outs, hipStream_t s, double* ms)
{
    const int nl = net_in_limbs(net), no = net_n_out(net);
    // every network input reads the same (zero) buffer
    std::vector<unihenn_ct> cin((size_t)net_n_inputs(net), unihenn_ct{in, (uint32_t)nl, (uint32_t)batch, c->scale});
    std::vector<unihenn_ct> co(no);
    for (int o = 0; o < no; ++o) co[o] = unihenn_ct{outs + (size_t)o * batch * 2 * c->n, 1, (uint32_t)batch, 0.0};
    net_drop_graphs(net);
    return time_ms(s, 0, [&]() { return unihenn_eval_network(c, net, cin.data(), co.data(), s); }, ms);
}

// ---- cache file: one JSON object, one entry per line
const char* kFmt = "{\"ntt_split\": %d, \"ntt_tile_log\": %d, \"mac_min_wg\": %d, \"ks_min_wg\": %d, "
                   "\"ks_group\": %d, \"ks_order\": %d, \"ntt_ms\": %lf, \"net_ms\": %lf}";

std::map<std::string, unihenn_tuning> read_cache(const char* path)
{
    std::map<std::string, unihenn_tuning> out;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        const size_t a = line.find('"');
        if (a == std::string::npos) continue;
        const size_t b = line.find('"', a + 1);
        const size_t brace = line.find('{', b == std::string::npos ? 0 : b);
        if (b == std::string::npos || brace == std::string::npos) continue;
        unihenn_tuning t{};
        if (sscanf(line.c_str() + brace, kFmt, &t.ntt_split, &t.ntt_tile_log, &t.mac_min_wg, &t.ks_min_wg,
                   &t.ks_group, &t.ks_order, &t.ntt_ms, &t.net_ms) == 8)
            out[line.substr(a + 1, b - a - 1)] = t;
    }
    return out;
}

int write_cache(const char* path, const std::map<std::string, unihenn_tuning>& m)
{
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = fopen(tmp.c_str(), "w");
    if (!f) return uh_fail(UNIHENN_EINVAL, std::string("cannot write tuning cache ") + path);
    fprintf(f, "{\n");
    size_t i = 0;
    for (const auto& kv : m) {
        const unihenn_tuning& t = kv.second;
        fprintf(f, "\"%s\": ", kv.first.c_str());
        fprintf(f, kFmt, t.ntt_split, t.ntt_tile_log, t.mac_min_wg, t.ks_min_wg, t.ks_group, t.ks_order, t.ntt_ms,
                t.net_ms);
        fprintf(f, "%s\n", ++i < m.size() ? "," : "");
    }
    fprintf(f, "}\n");
    if (fclose(f) != 0 || rename(tmp.c_str(), path) != 0)
        return uh_fail(UNIHENN_EINVAL, std::string("cannot write tuning cache ") + path);
    return UNIHENN_OK;
}

std::string cache_key(const unihenn_ctx* c, const unihenn_net* net, int batch)
{
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    int cus = 0;
    if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) {
        arch = prop.gcnArchName;
        cus = prop.multiProcessorCount;
    }
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
    char buf[256];
    snprintf(buf, sizeof(buf), "%s/cu%d/logn%d/nd%d/b%d/net%016llx/mode%d", arch.c_str(), cus, c->log_n, c->n_data,
             batch, net ? (unsigned long long)net_fingerprint(net) : 0ull,
             net ? net_mode(net) : 0);
    return buf;
}

void current(const unihenn_ctx* c, const unihenn_net* net, unihenn_tuning* t)
{
    int l1 = c->ntt_split > 0 && c->ntt_split < c->log_n ? c->ntt_split : c->log_n / 2;
    t->ntt_split = l1;
    t->ntt_tile_log = c->ntt_tile_log;
    t->mac_min_wg = c->mac_min_wg;
    t->ks_min_wg = c->ks_min_wg;
    t->ks_group = net ? net_ks_group(net) : 0;
    t->ks_order = c->ks_order;
}

int apply(unihenn_ctx* c, unihenn_net* net, const unihenn_tuning* t)
{
    if (t->ntt_split > 0 && t->ntt_split >= c->log_n) return uh_fail(UNIHENN_EINVAL, "NTT split out of range");
    if (t->ntt_tile_log > 0 && t->ntt_tile_log != 11 && t->ntt_tile_log != 12)
        return uh_fail(UNIHENN_EINVAL, "NTT tile must be 2^11 or 2^12 words");
    if (t->ks_order < 0 || t->ks_order > 2) return uh_fail(UNIHENN_EINVAL, "workgroup order must be 0, 1 or 2");
    if (net && t->ks_group > 0) {
        int rc = net_set_ks_group(c, net, t->ks_group);
        if (rc) return rc;
    }
    if (net) net_drop_graphs(net);
    if (t->ntt_split > 0) c->ntt_split = t->ntt_split;
    if (t->ntt_tile_log > 0) c->ntt_tile_log = t->ntt_tile_log;
    if (t->mac_min_wg > 0) c->mac_min_wg = t->mac_min_wg;
    if (t->ks_min_wg > 0) c->ks_min_wg = t->ks_min_wg;
    c->ks_order = t->ks_order;
    return UNIHENN_OK;
}

}  // namespace

extern "C" int unihenn_tuning_get(const unihenn_ctx* c, const unihenn_net* net, unihenn_tuning* out)
{
    if (!c || !out) return uh_fail(UNIHENN_EINVAL, "null argument");
    memset(out, 0, sizeof(*out));
    current(c, net, out);
    return UNIHENN_OK;
}

extern "C" int unihenn_tuning_set(unihenn_ctx* c, unihenn_net* net, const unihenn_tuning* t)
{
    if (!c || !t) return uh_fail(UNIHENN_EINVAL, "null argument");
    return apply(c, net, t);
}

extern "C" int unihenn_autotune(unihenn_ctx* c, unihenn_net* net, uint32_t batch_u, const char* cache_path,
                                unihenn_tuning* out, void* stream)
{
    if (!c) return uh_fail(UNIHENN_EINVAL, "null argument");
    hipStream_t s = (hipStream_t)stream;
    const int batch = (int)std::max<uint32_t>(1, batch_u);
    if (net && batch > net_max_batch(net)) return uh_fail(UNIHENN_EINVAL, "batch exceeds max_batch");
    const std::string key = cache_key(c, net, batch);
    std::map<std::string, unihenn_tuning> cache;
    if (cache_path) {
        cache = read_cache(cache_path);
        auto it = cache.find(key);
        if (it != cache.end()) {
            int rc = apply(c, net, &it->second);
            if (rc) return rc;
            if (out) *out = it->second;
            return UNIHENN_OK;
        }
    }
    UH_CHECK_HIP(hipDeviceSynchronize());
    unihenn_tuning best{};
    current(c, net, &best);

    // candidate NTT splits keep both passes in the radix-8 range 3..8
    std::vector<std::pair<int, int>> ntt_cands;
    for (int l1 = 3; l1 <= c->log_n - 3; ++l1)
        if (l1 <= 8 && c->log_n - l1 <= 8)
            for (int tile : {11, 12}) ntt_cands.push_back({l1, tile});

    // 1. NTT split and tile on a forward + inverse transform of a batch of rows
    {
        const int rows = ntt_rows(c, batch);
        Buf d;
        int rc = d.alloc((size_t)rows * c->n);
        if (rc) return rc;
        UH_CHECK_HIP(hipMemsetAsync(d.p, 0, sizeof(u64) * (size_t)rows * c->n, s));
        double best_ms = 1e30;
        for (auto [l1, tile] : ntt_cands) {
            c->ntt_split = l1;
            c->ntt_tile_log = tile;
            double ms = 0;
            rc = time_ntt(c, d.p, rows, s, &ms);
            if (rc) return rc;
            if (ms < best_ms) {
                best_ms = ms;
                best.ntt_split = l1;
                best.ntt_tile_log = tile;
            }
        }
        c->ntt_split = best.ntt_split;
        c->ntt_tile_log = best.ntt_tile_log;
        best.ntt_ms = best_ms < 1e29 ? best_ms : 0.0;
    }

    // 2. network: one coordinate at a time on whole evaluations in the net's
    //    mode (NTT split and tile, group size, MAC and inner-product targets)
    bool keys_ok = false;
    if (net) {
        const int nl = net_in_limbs(net), no = net_n_out(net);
        Buf in, outs;
        int rc = in.alloc((size_t)batch * 2 * nl * c->n);
        if (!rc) rc = outs.alloc((size_t)no * batch * 2 * c->n);
        if (rc) return rc;
        UH_CHECK_HIP(hipMemsetAsync(in.p, 0, sizeof(u64) * (size_t)batch * 2 * nl * c->n, s));
        UH_CHECK_HIP(hipStreamSynchronize(s));
        double cur = 0;
        rc = time_net(c, net, batch, in.p, outs.p, s, &cur);
        if (rc == UNIHENN_ENOKEY) {
            rc = UNIHENN_OK;  // keys not bound: the transform-level choice stands
        } else if (rc == UNIHENN_OK) {
            keys_ok = true;
            // NTT
            {
                int b1 = c->ntt_split, bt = c->ntt_tile_log;
                for (auto [l1, tile] : ntt_cands) {
                    if (l1 == b1 && tile == bt) continue;
                    c->ntt_split = l1;
                    c->ntt_tile_log = tile;
                    double ms = 0;
                    rc = time_net(c, net, batch, in.p, outs.p, s, &ms);
                    if (rc) break;
                    if (ms < cur) {
                        cur = ms;
                        best.ntt_split = l1;
                        best.ntt_tile_log = tile;
                    }
                }
                c->ntt_split = best.ntt_split;
                c->ntt_tile_log = best.ntt_tile_log;
            }
            // group size, under each workgroup order of the inner product
            const int cap = net_ks_group_cap(c, net);
            int g_best = net_ks_group(net), o_best = c->ks_order;
            // order 2 (row-fused inner product) applies to plain rotations only
            const int n_orders = (net_mode(net) & UNIHENN_EVAL_HOISTED) ? 2 : 3;
            for (int order = 0; order < n_orders && !rc; ++order) {
                c->ks_order = order;
                for (int e = 1; e <= cap && !rc; e *= 2) {
                    if (e == g_best && order == o_best) continue;
                    rc = net_set_ks_group(c, net, e);
                    double ms = 0;
                    if (!rc) rc = time_net(c, net, batch, in.p, outs.p, s, &ms);
                    if (!rc && ms < cur) {
                        cur = ms;
                        g_best = e;
                        o_best = order;
                    }
                }
            }
            c->ks_order = o_best;
            if (!rc) rc = net_set_ks_group(c, net, g_best);
            best.ks_group = g_best;
            best.ks_order = o_best;
            // workgroup targets
            for (int which = 0; which < 2 && !rc; ++which) {
                int* field = which == 0 ? &c->mac_min_wg : &c->ks_min_wg;
                int v_best = *field;
                for (int v : {512, 1024, 2048, 4096, 8192}) {
                    if (v == v_best) continue;
                    *field = v;
                    double ms = 0;
                    rc = time_net(c, net, batch, in.p, outs.p, s, &ms);
                    if (rc) break;
                    if (ms < cur) {
                        cur = ms;
                        v_best = v;
                    }
                }
                *field = v_best;
            }
            best.mac_min_wg = c->mac_min_wg;
            best.ks_min_wg = c->ks_min_wg;
            best.net_ms = cur;
        }
        net_drop_graphs(net);
        if (rc) return rc;
    }
    if (out) *out = best;
    if (cache_path && (keys_ok || !net)) {
        cache[key] = best;
        return write_cache(cache_path, cache);
    }
    return UNIHENN_OK;
}
