// Host side of the batched scan: plan creation (threshold tables, lattice and
// trace layout, buckets by lattice size, launch shapes from the autotuner),
// hipGraph capture of the persistent launch, and plan teardown.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "sd_autotune.hpp"
#include "sd_batch.hpp"
#include "sd_host.hpp"

struct sd_batch_plan {
    int device = 0;
    int32_t n_chains = 0;
    int32_t layout = SD_P64;
    uint64_t seed = 0;
    uint32_t k_steps = 0, obs_every = 0, n_rec = 0, flags = 0;
    std::vector<sd::ChainDesc> descs;
    size_t lattice_total = 0;

    struct Bucket {
        uint32_t L = 0;
        uint32_t paired = 1;             // compare form shared by the bucket's chains
        uint32_t max_words = 0;
        uint32_t first = 0, count = 0;   // range in the order array
        uint32_t threads = 256, blocks = 1;
    };
    std::vector<Bucket> buckets;

    sd::ChainDesc* d_descs = nullptr;
    uint32_t* d_order = nullptr;
    uint32_t* d_counters = nullptr;

    // cached graph of the last run shape
    bool have_graph = false;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    void* g_lattices = nullptr;
    int64_t* g_traces = nullptr;
    uint64_t g_step0 = 0;
    hipStream_t capture = nullptr;   // stream the graph is captured on
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> events;
    // device wall clock of each bucket's launch in the last run: first start
    // (entries 0 .. n-1), last end (entries n .. 2n-1)
    unsigned long long* d_times = nullptr;
    bool ran = false;
};

namespace sd {

uint32_t lattice_words(uint32_t L) { return (uint32_t)(((uint64_t)L * L) / 64u); }

void set_divisors(ChainDesc& d, uint32_t L) {
    d.divW = make_fastdiv(L >= 64u ? L / 64u : 1u);
    d.divL = make_fastdiv(L);
}

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

void release_graph(sd_batch_plan* p) {
    if (p->exec)
        (void)hipGraphExecDestroy(p->exec);
    if (p->graph)
        (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
    p->have_graph = false;
}

BatchArgs bucket_args(const sd_batch_plan* p, size_t b, void* lattices, int64_t* traces, uint64_t step0) {
    const sd_batch_plan::Bucket& bk = p->buckets[b];
    BatchArgs a;
    std::memset(&a, 0, sizeof a);
    a.chains = p->d_descs;
    a.order = p->d_order + bk.first;
    a.n_chains = bk.count;
    a.counter = p->d_counters + b;
    a.t_start = p->d_times + b;
    a.t_end = p->d_times + p->buckets.size() + b;
    a.lattices = static_cast<uint8_t*>(lattices);
    a.traces = p->n_rec ? traces : nullptr;
    a.key0 = (uint32_t)(p->seed & 0xFFFFFFFFu);
    a.key1 = (uint32_t)(p->seed >> 32);
    a.step0 = (uint32_t)step0;
    a.k_steps = p->k_steps;
    a.obs_every = p->obs_every ? p->obs_every : 1u;
    a.rng_xor = (p->flags & SD_FLAG_COMPLEMENT_RNG) ? 0xFFFFFFFFu : 0u;
    a.moments = (p->flags & SD_FLAG_MOMENTS) ? 1u : 0u;
    a.max_words = bk.max_words;
    a.bits = bk.L % 64u != 0 ? 1u : 0u;
    a.int8_io = p->layout == SD_I8 ? 1u : 0u;
    a.paired = bk.paired;
    // later buckets (smaller lattices) of the same kernel form: taken from
    // once this bucket's queue is empty, so that no bucket's workgroups idle
    // while another bucket still has chains waiting
    for (size_t c = b + 1; c < p->buckets.size() && a.n_steal < kMaxSteal; ++c) {
        const sd_batch_plan::Bucket& o = p->buckets[c];
        if (o.paired != bk.paired || (o.L % 64u != 0) != (bk.L % 64u != 0) || o.max_words > bk.max_words)
            continue;
        a.steal_order[a.n_steal] = p->d_order + o.first;
        a.steal_count[a.n_steal] = o.count;
        a.steal_counter[a.n_steal] = p->d_counters + c;
        ++a.n_steal;
    }
    return a;
}

// The launches of a run: the queue counters and the time stamps reset, then
// every bucket's persistent launch on its own side stream.
hipError_t enqueue_batch(sd_batch_plan* p, void* lattices, int64_t* traces, uint64_t step0, hipStream_t st) {
    const uint32_t nb = (uint32_t)p->buckets.size();
    hipError_t e = launch_zero_u32(p->d_counters, nb, st);
    if (e == hipSuccess)
        e = launch_times_reset(p->d_times, p->d_times + nb, nb, st);
    if (e != hipSuccess)
        return e;
    if (nb == 1) {
        const auto& bk = p->buckets[0];
        return launch_batch_chains(bucket_args(p, 0, lattices, traces, step0), bk.blocks, bk.threads, st);
    }
    // fork: every bucket runs on its own stream after the counters are zeroed
    e = hipEventRecord(p->events[0], st);
    for (size_t b = 0; b < nb && e == hipSuccess; ++b) {
        hipStream_t s = p->side[b];
        e = hipStreamWaitEvent(s, p->events[0], 0);
        if (e == hipSuccess) {
            const auto& bk = p->buckets[b];
            e = launch_batch_chains(bucket_args(p, b, lattices, traces, step0), bk.blocks, bk.threads, s);
        }
        if (e == hipSuccess)
            e = hipEventRecord(p->events[1 + b], s);
        if (e == hipSuccess)
            e = hipStreamWaitEvent(st, p->events[1 + b], 0);
    }
    return e;
}

}  // namespace

// Measured choice of the batched kernel's block size for chains of size L: a
// sample of this plan's chains of that size runs 64 steps on scratch lattices
// for every candidate (best of three launches after a warm-up); the fastest
// is kept in the cache file.
uint32_t autotune_batch_threads(const char* cache_path, uint32_t L, uint32_t paired, uint32_t n_chains,
                                sd_batch_plan* p) {
    const uint32_t fallback = 256;
    if (!cache_path || !*cache_path)
        return fallback;
    const std::string key = "batch:" + device_arch() + ":L=" + std::to_string(L) + ":p=" + std::to_string(paired) +
                            ":k=" + std::to_string(p->obs_every ? 1 : 0);
    // a cached block size is taken only if the kernel of this form can run it;
    // and no workgroup gets more wavefronts than a half-step has 64-word tiles
    // (the rest would idle in every half-step while holding a slot that the
    // scan's other buckets could use)
    const long tiles = (long)((lattice_words(L) + 63u) / 64u);
    const long max_threads = std::min<long>(paired ? (long)kBatchMaxThreads : 512, std::max<long>(64, 64 * tiles));
    const long cached = tune_cache_get(cache_path, key);
    if (cached >= 64 && cached <= max_threads && cached % 64 == 0)
        return (uint32_t)cached;
    int dev = 0, n_cu = 1;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return fallback;
    std::vector<ChainDesc> sample;
    for (const ChainDesc& d : p->descs)
        if (d.L == L && d.paired == paired && sample.size() < std::min<uint32_t>(n_chains, 2u * (uint32_t)n_cu))
            sample.push_back(d);
    const uint32_t S = (uint32_t)sample.size();
    const uint32_t k = 64;   // long enough that the small lattices' launches are not timed in noise
    const size_t bytes = lattice_bytes((int32_t)L, p->layout);
    size_t off = 0;
    for (uint32_t i = 0; i < S; ++i) {
        sample[i].sig_offset = off;
        off = align_up(off + bytes);
        sample[i].tau_offset = off;
        off = align_up(off + bytes);
        sample[i].trace_offset = (uint64_t)i * k * 3u;
    }
    std::vector<uint32_t> order(S);
    for (uint32_t i = 0; i < S; ++i)
        order[i] = i;
    void* lat = nullptr;
    int64_t* tr = nullptr;
    ChainDesc* dd = nullptr;
    uint32_t* dord = nullptr;
    uint32_t* cnt = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(&lat, off);
    if (e == hipSuccess) e = hipMalloc(&tr, sizeof(int64_t) * S * k * 3u);
    if (e == hipSuccess) e = hipMalloc(&dd, sizeof(ChainDesc) * S);
    if (e == hipSuccess) e = hipMalloc(&dord, sizeof(uint32_t) * S);
    if (e == hipSuccess) e = hipMalloc(&cnt, sizeof(uint32_t));
    if (e == hipSuccess) e = hipMemset(lat, 0x5A, off);
    if (e == hipSuccess) e = hipMemcpy(dd, sample.data(), sizeof(ChainDesc) * S, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dord, order.data(), sizeof(uint32_t) * S, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    long best = -1;
    if (e == hipSuccess) {
        auto measure = [&](long threads) -> double {
            const size_t lds = batch_lds_bytes(lattice_words(L), (uint32_t)threads);
            BatchArgs a;
            std::memset(&a, 0, sizeof a);
            a.chains = dd;
            a.order = dord;
            a.n_chains = S;
            a.counter = cnt;
            a.lattices = static_cast<uint8_t*>(lat);
            a.traces = tr;
            a.key0 = 1;
            a.k_steps = k;
            a.obs_every = 1;
            a.max_words = lattice_words(L);
            a.bits = L % 64u != 0 ? 1u : 0u;
            a.int8_io = p->layout == SD_I8 ? 1u : 0u;
            a.paired = paired;
            int per_cu = 0;
            if (batch_occupancy((uint32_t)threads, lds, paired != 0, L % 64u != 0, &per_cu) != hipSuccess || per_cu < 1)
                return -1.0;
            const uint32_t blocks = std::max<uint32_t>(1, std::min<uint32_t>(S, (uint32_t)per_cu * (uint32_t)n_cu));
            float best_ms = -1.0f;
            for (int rep = 0; rep < 4; ++rep) {   // the first launch warms up, the best of the other three counts
                if (launch_zero_u32(cnt, 1, nullptr) != hipSuccess) return -1.0;
                if (hipEventRecord(e0, nullptr) != hipSuccess) return -1.0;
                if (launch_batch_chains(a, blocks, (uint32_t)threads, nullptr) != hipSuccess) return -1.0;
                if (hipEventRecord(e1, nullptr) != hipSuccess) return -1.0;
                if (hipEventSynchronize(e1) != hipSuccess) return -1.0;
                float ms = 0.0f;
                if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return -1.0;
                if (rep > 0 && (best_ms < 0.0f || ms < best_ms))
                    best_ms = ms;
            }
            return best_ms / 1e3;
        };
        std::vector<long> cand;
        for (long t : {64L, 128L, 256L, 512L, (long)kBatchMaxThreads})
            if (t <= max_threads)
                cand.push_back(t);
        best = tune_pick(cand, measure);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (lat) (void)hipFree(lat);
    if (tr) (void)hipFree(tr);
    if (dd) (void)hipFree(dd);
    if (dord) (void)hipFree(dord);
    if (cnt) (void)hipFree(cnt);
    (void)hipGetLastError();
    if (best <= 0)
        return fallback;
    tune_cache_put(cache_path, key, best);
    return (uint32_t)best;
}

// Single-chain LDS-resident run used by sd_run for small lattices.
hipError_t launch_trajectories_lds(const void* sigma0, void* traj, uint32_t n_traj, int32_t L, double J, double q,
                                   uint64_t seed, uint32_t stream0, uint64_t step0, uint32_t k_steps,
                                   uint32_t threads, hipStream_t st) {
    BatchArgs a;
    std::memset(&a, 0, sizeof a);
    threshold_table(J, q, a.single.T);
    a.single.paired = thresholds_paired(a.single.T) ? 1u : 0u;
    a.single.L = (uint32_t)L;
    a.single.stream = stream0;
    set_divisors(a.single, (uint32_t)L);
    a.single_sig = static_cast<uint8_t*>(const_cast<void*>(sigma0));
    a.n_uniform = n_traj;
    a.key0 = (uint32_t)(seed & 0xFFFFFFFFu);
    a.key1 = (uint32_t)(seed >> 32);
    a.step0 = (uint32_t)step0;
    a.k_steps = k_steps;
    a.obs_every = 1;
    a.max_words = lattice_words((uint32_t)L);
    a.bits = L % 64 != 0 ? 1u : 0u;
    a.paired = a.single.paired;
    a.traj = static_cast<uint8_t*>(traj);
    a.traj_chain_bytes = (2ull * k_steps + 1ull) * a.max_words * sizeof(uint64_t);
    hipError_t e = batch_kernel_attributes(batch_lds_bytes(a.max_words, threads));
    if (e != hipSuccess)
        return e;
    return launch_batch_chains(a, n_traj, threads, st);
}

hipError_t launch_single_chain_lds(void* sigma, void* tau, int32_t L, bool int8_io, double J, double q,
                                   uint64_t seed, uint32_t stream, uint64_t step0, uint32_t k_steps, int64_t* obs,
                                   uint32_t obs_every, uint32_t flags, uint32_t threads, hipStream_t st) {
    BatchArgs a;
    std::memset(&a, 0, sizeof a);
    a.counter = nullptr;
    threshold_table(J, q, a.single.T);
    a.single.paired = thresholds_paired(a.single.T) && !(flags & SD_FLAG_GENERAL_COMPARE) ? 1u : 0u;
    a.single.L = (uint32_t)L;
    a.single.stream = stream;
    set_divisors(a.single, (uint32_t)L);
    a.single_sig = static_cast<uint8_t*>(sigma);
    a.single_tau = static_cast<uint8_t*>(tau);
    a.traces = obs;
    a.key0 = (uint32_t)(seed & 0xFFFFFFFFu);
    a.key1 = (uint32_t)(seed >> 32);
    a.step0 = (uint32_t)step0;
    a.k_steps = k_steps;
    a.obs_every = obs_every ? obs_every : 1u;
    a.rng_xor = (flags & SD_FLAG_COMPLEMENT_RNG) ? 0xFFFFFFFFu : 0u;
    a.max_words = lattice_words((uint32_t)L);
    a.bits = L % 64 != 0 ? 1u : 0u;
    a.int8_io = int8_io ? 1u : 0u;
    a.paired = a.single.paired;
    hipError_t e = batch_kernel_attributes(batch_lds_bytes(a.max_words, threads));
    if (e != hipSuccess)
        return e;
    return launch_batch_chains(a, 1, threads, st);
}

}  // namespace sd

using namespace sd;

extern "C" {

sd_status sd_batch_plan_create(sd_batch_plan** plan_out, const sd_chain_desc* chains, int32_t n_chains, int32_t layout,
                               uint64_t seed, uint32_t k_steps, uint32_t obs_every, uint32_t flags,
                               const char* tune_cache_path) {
    if (!plan_out || !chains || n_chains <= 0)
        return fail(SD_EINVAL, "sd_batch_plan_create: need an output handle and at least one chain");
    *plan_out = nullptr;
    if (layout != SD_P64 && layout != SD_I8)
        return fail(SD_EUNSUPPORTED, "sd_batch_plan_create: layout must be SD_P64 or SD_I8");
    if (k_steps >= (1u << 29))
        return fail(SD_EINVAL, "sd_batch_plan_create: k_steps must be below 2^29");
    if (flags & ~(SD_FLAG_COMPLEMENT_RNG | SD_FLAG_MOMENTS | SD_FLAG_GENERAL_COMPARE))
        return fail(SD_EINVAL, "sd_batch_plan_create: unknown flags");
    if ((flags & SD_FLAG_MOMENTS) && !obs_every)
        return fail(SD_EINVAL, "sd_batch_plan_create: SD_FLAG_MOMENTS needs obs_every > 0");
    for (int32_t c = 0; c < n_chains; ++c) {   // every descriptor before any device query
        const sd_chain_desc& in = chains[c];
        if (in.L < 8 || in.L > 65535 || in.L % 8 != 0 || !std::isfinite(in.J) || !std::isfinite(in.q))
            return fail(SD_EINVAL, "sd_batch_plan_create: chain %d needs finite J, q and L a multiple of 8", c);
    }
    int device = 0;
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess)
        return hip_fail(e, "sd_batch_plan_create");
    int max_lds = 0, n_cu = 0;
    e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess)
        return hip_fail(e, "sd_batch_plan_create");

    sd_batch_plan* p = new (std::nothrow) sd_batch_plan();
    if (!p)
        return fail(SD_ENOSPACE, "sd_batch_plan_create: out of host memory");
    p->device = device;
    p->n_chains = n_chains;
    p->layout = layout;
    p->seed = seed;
    p->k_steps = k_steps;
    p->obs_every = obs_every;
    p->n_rec = obs_every ? k_steps / obs_every : 0u;
    p->flags = flags;
    p->descs.resize((size_t)n_chains);

    // buckets by (L, compare form): largest L first, paired before the
    // six-class form (only under SD_FLAG_GENERAL_COMPARE)
    std::map<std::pair<uint32_t, uint32_t>, std::vector<uint32_t>, std::greater<std::pair<uint32_t, uint32_t>>> by_L;
    size_t off = 0;
    for (int32_t c = 0; c < n_chains; ++c) {
        const sd_chain_desc& in = chains[c];
        if (in.L < 8 || in.L > 65535 || in.L % 8 != 0 || !std::isfinite(in.J) || !std::isfinite(in.q)) {
            delete p;
            return fail(SD_EINVAL, "sd_batch_plan_create: chain %d needs finite J, q and L a multiple of 8", c);
        }
        const size_t words = lattice_words((uint32_t)in.L);
        if (batch_lds_bytes((uint32_t)words, 64) > (size_t)max_lds) {
            delete p;
            return fail(SD_EUNSUPPORTED, "sd_batch_plan_create: chain %d (L=%d) does not fit in %d bytes of LDS", c,
                        in.L, max_lds);
        }
        ChainDesc& d = p->descs[(size_t)c];
        threshold_table(in.J, in.q, d.T);
        d.paired = thresholds_paired(d.T) && !(flags & SD_FLAG_GENERAL_COMPARE) ? 1u : 0u;
        d.L = (uint32_t)in.L;
        d.stream = in.stream;
        set_divisors(d, (uint32_t)in.L);
        const size_t bytes = lattice_bytes(in.L, layout);
        d.sig_offset = off;
        off = align_up(off + bytes);
        d.tau_offset = off;
        off = align_up(off + bytes);
        d.trace_offset = (flags & SD_FLAG_MOMENTS) ? (uint64_t)c * kMomentWords : (uint64_t)c * p->n_rec * 3u;
        by_L[std::make_pair((uint32_t)in.L, d.paired)].push_back((uint32_t)c);
    }
    p->lattice_total = off;

    std::vector<uint32_t> order;
    order.reserve((size_t)n_chains);
    for (auto& kv : by_L) {
        sd_batch_plan::Bucket bk;
        bk.L = kv.first.first;
        bk.paired = kv.first.second;
        bk.max_words = lattice_words(bk.L);
        bk.first = (uint32_t)order.size();
        bk.count = (uint32_t)kv.second.size();
        order.insert(order.end(), kv.second.begin(), kv.second.end());
        p->buckets.push_back(bk);
    }

    size_t max_words = 0;
    for (auto& bk : p->buckets)
        max_words = std::max(max_words, (size_t)bk.max_words);
    e = batch_kernel_attributes(batch_lds_bytes((uint32_t)max_words, kBatchMaxThreads));
    if (e == hipSuccess)
        e = hipMalloc(&p->d_descs, sizeof(ChainDesc) * p->descs.size());
    if (e == hipSuccess)
        e = hipMalloc(&p->d_order, sizeof(uint32_t) * order.size());
    if (e == hipSuccess)
        e = hipMalloc(&p->d_counters, sizeof(uint32_t) * p->buckets.size());
    if (e == hipSuccess)
        e = hipMalloc(&p->d_times, sizeof(unsigned long long) * 2 * p->buckets.size());
    if (e == hipSuccess)
        e = hipMemcpy(p->d_descs, p->descs.data(), sizeof(ChainDesc) * p->descs.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(p->d_order, order.data(), sizeof(uint32_t) * order.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipStreamCreateWithFlags(&p->capture, hipStreamNonBlocking);
    for (size_t b = 0; b < p->buckets.size() && e == hipSuccess; ++b) {
        hipStream_t s = nullptr;
        e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e == hipSuccess)
            p->side.push_back(s);
    }
    for (size_t i = 0; i < p->buckets.size() + 1 && e == hipSuccess; ++i) {
        hipEvent_t ev = nullptr;
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess)
            p->events.push_back(ev);
    }
    if (e != hipSuccess) {
        sd_batch_plan_destroy(p);
        return hip_fail(e, "sd_batch_plan_create");
    }

    // launch shape per bucket: cached / tuned block size, grid = resident blocks
    for (auto& bk : p->buckets) {
        uint32_t threads = autotune_batch_threads(tune_cache_path, bk.L, bk.paired, bk.count, p);
        const size_t lds = batch_lds_bytes(bk.max_words, threads);
        int per_cu = 0;
        e = batch_occupancy(threads, lds, bk.paired != 0, bk.L % 64u != 0, &per_cu);
        if (e != hipSuccess || per_cu < 1)
            per_cu = 1;
        uint64_t blocks = (uint64_t)per_cu * (uint64_t)n_cu;
        bk.threads = threads;
        bk.blocks = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(blocks, bk.count));
    }
    *plan_out = p;
    return SD_OK;
}

size_t sd_batch_lattice_bytes(const sd_batch_plan* plan) { return plan ? plan->lattice_total : 0; }

size_t sd_batch_trace_len(const sd_batch_plan* plan) {
    if (!plan)
        return 0;
    if (plan->flags & SD_FLAG_MOMENTS)
        return (size_t)plan->n_chains * kMomentWords;
    return (size_t)plan->n_chains * plan->n_rec * 3u;
}

int64_t sd_batch_chain_offset(const sd_batch_plan* plan, int32_t chain, int32_t which) {
    if (!plan || chain < 0 || chain >= plan->n_chains || (which != 0 && which != 1))
        return -1;
    const ChainDesc& d = plan->descs[(size_t)chain];
    return (int64_t)(which == 0 ? d.sig_offset : d.tau_offset);
}

sd_status sd_batch_launch_shape(const sd_batch_plan* plan, int32_t bucket, int32_t* L, int32_t* n_chains,
                                int32_t* threads, int32_t* blocks) {
    if (!plan || bucket < 0 || (size_t)bucket >= plan->buckets.size())
        return fail(SD_EINVAL, "sd_batch_launch_shape: no such bucket");
    const auto& bk = plan->buckets[(size_t)bucket];
    if (L) *L = (int32_t)bk.L;
    if (n_chains) *n_chains = (int32_t)bk.count;
    if (threads) *threads = (int32_t)bk.threads;
    if (blocks) *blocks = (int32_t)bk.blocks;
    return SD_OK;
}

sd_status sd_batch_init(sd_batch_plan* plan, void* lattices, int32_t kind, double p_up, void* hip_stream) {
    if (!plan || !lattices)
        return fail(SD_EINVAL, "sd_batch_init: null plan or lattices");
    for (int32_t c = 0; c < plan->n_chains; ++c) {
        const ChainDesc& d = plan->descs[(size_t)c];
        sd_status s = sd_init(static_cast<uint8_t*>(lattices) + d.sig_offset, (int32_t)d.L, plan->layout, kind, p_up,
                              plan->seed, d.stream, hip_stream);
        if (s != SD_OK)
            return s;
    }
    return SD_OK;
}

sd_status sd_batch_run(sd_batch_plan* plan, void* lattices, int64_t* traces, uint64_t step0, void* hip_stream) {
    if (!plan || !lattices)
        return fail(SD_EINVAL, "sd_batch_run: null plan or lattices");
    if (plan->n_rec && !traces)
        return fail(SD_EINVAL, "sd_batch_run: the plan records observables, traces must not be null");
    if (step0 + plan->k_steps > (1ull << 29))
        return fail(SD_EINVAL, "sd_batch_run: step indices must stay below 2^29");
    const uintptr_t a = reinterpret_cast<uintptr_t>(lattices);
    if (a % 16u)
        return fail(SD_EINVAL, "sd_batch_run: lattices must be 16-byte aligned");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    hipError_t e = hipSuccess;
    if (!(plan->have_graph && plan->g_lattices == lattices && plan->g_traces == traces && plan->g_step0 == step0)) {
        // capture on the plan's own stream (the caller's may be the legacy
        // default stream, which cannot be captured); the graph is then
        // launched on the caller's stream and ordered after its earlier work
        release_graph(plan);
        e = hipStreamBeginCapture(plan->capture, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess)
            return hip_fail(e, "sd_batch_run: begin capture");
        hipError_t ee = enqueue_batch(plan, lattices, traces, step0, plan->capture);
        e = hipStreamEndCapture(plan->capture, &plan->graph);
        if (ee != hipSuccess)
            e = ee;
        if (e == hipSuccess)
            e = hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            release_graph(plan);
            return hip_fail(e, "sd_batch_run: graph capture");
        }
        plan->have_graph = true;
        plan->g_lattices = lattices;
        plan->g_traces = traces;
        plan->g_step0 = step0;
    }
    e = hipGraphLaunch(plan->exec, st);
    plan->ran = plan->ran || e == hipSuccess;
    return e == hipSuccess ? SD_OK : hip_fail(e, "sd_batch_run: graph launch");
}

sd_status sd_batch_run_direct(sd_batch_plan* plan, void* lattices, int64_t* traces, uint64_t step0,
                              void* hip_stream) {
    if (!plan || !lattices)
        return fail(SD_EINVAL, "sd_batch_run_direct: null plan or lattices");
    if (plan->n_rec && !traces)
        return fail(SD_EINVAL, "sd_batch_run_direct: the plan records observables, traces must not be null");
    if (step0 + plan->k_steps > (1ull << 29))
        return fail(SD_EINVAL, "sd_batch_run_direct: step indices must stay below 2^29");
    if (reinterpret_cast<uintptr_t>(lattices) % 16u)
        return fail(SD_EINVAL, "sd_batch_run_direct: lattices must be 16-byte aligned");
    hipError_t e = enqueue_batch(plan, lattices, traces, step0, static_cast<hipStream_t>(hip_stream));
    plan->ran = plan->ran || e == hipSuccess;
    return e == hipSuccess ? SD_OK : hip_fail(e, "sd_batch_run_direct");
}

sd_status sd_batch_bucket_times(sd_batch_plan* plan, int32_t bucket, float* start_ms, float* end_ms) {
    if (!plan || bucket < 0 || (size_t)bucket >= plan->buckets.size() || !start_ms || !end_ms)
        return fail(SD_EINVAL, "sd_batch_bucket_times: no such bucket or null output");
    if (!plan->ran)
        return fail(SD_EINVAL, "sd_batch_bucket_times: no run of this plan yet");
    const size_t nb = plan->buckets.size();
    std::vector<unsigned long long> t(2 * nb);
    int dev = 0, khz = 0;
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess)
        e = hipMemcpy(t.data(), plan->d_times, sizeof(unsigned long long) * 2 * nb, hipMemcpyDeviceToHost);
    if (e == hipSuccess)
        e = hipGetDevice(&dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
    if (e != hipSuccess)
        return hip_fail(e, "sd_batch_bucket_times");
    if (khz <= 0)
        return fail(SD_EHIP, "sd_batch_bucket_times: the device reports no wall-clock rate");
    unsigned long long t0 = ~0ull;
    for (size_t b = 0; b < nb; ++b)
        t0 = std::min(t0, t[b]);
    const size_t b = (size_t)bucket;
    if (t[b] == ~0ull || t[nb + b] < t[b])
        return fail(SD_EHIP, "sd_batch_bucket_times: bucket %d left no time stamps", bucket);
    *start_ms = (float)((double)(t[b] - t0) / khz);
    *end_ms = (float)((double)(t[nb + b] - t0) / khz);
    return SD_OK;
}

void sd_batch_plan_destroy(sd_batch_plan* plan) {
    if (!plan)
        return;
    release_graph(plan);
    for (hipStream_t s : plan->side)
        (void)hipStreamDestroy(s);
    if (plan->capture)
        (void)hipStreamDestroy(plan->capture);
    for (hipEvent_t ev : plan->events)
        (void)hipEventDestroy(ev);
    if (plan->d_descs)
        (void)hipFree(plan->d_descs);
    if (plan->d_order)
        (void)hipFree(plan->d_order);
    if (plan->d_counters)
        (void)hipFree(plan->d_counters);
    if (plan->d_times)
        (void)hipFree(plan->d_times);
    delete plan;
}

}  // extern "C"
