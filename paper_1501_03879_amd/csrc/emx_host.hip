// Host runtime of the C ABI declared in include/emx.h: argument validation,
// handle-owned workspace, persistent-grid sizing and kernel dispatch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "batch_plan.hpp"
#include "emx_internal.hpp"
#include "nlem_group.hpp"
#include "nlem_table.hpp"

namespace emx {

// batch_host.hip
em_status_t batch_solve(em_context *ctx, hipStream_t stream, int64_t B, const float *a,
                        const float *w, const em_instance_t *inst, const em_options_t &o, float *z,
                        em_stats_t *stats);
em_status_t plain_solve(em_context *ctx, hipStream_t stream, int64_t B, const float *a,
                        const float *w, const em_instance_t *inst, const em_instance_t *inst_host,
                        const em_options_t &o, float *z, em_stats_t *stats);
em_status_t batch_wide_counts(em_context *ctx, hipStream_t s, int64_t B, const em_instance_t *inst,
                              unsigned int (&wide_counts)[kNumWideClasses]);

__global__ void reset_counters_kernel(unsigned int *c, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) c[i] = 0u;
}
}  // namespace emx

using namespace emx;

struct MultiGraph {
    std::vector<char> key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void *ws = nullptr;   // the graph's own queue-order scratch (kept with the graph)
};

// NLEM plans: (patch radius, points per lane, solver, FP16 storage) -> the
// solve kernel's schedule (nlem_plan_t without its source).
using PlanKey = std::tuple<int, int, int, int>;
struct NlemPlan {
    int wc = 0;         // coordinate waves
    int chunk = 0;      // queue positions per pop; 0 = the size rule
    int order = -1;     // longest-first order: -1 = the rule, 0 = off, 1 = on
    float arm = 1.0f;   // residual arm factor (>= 1)
    int check = 1;      // residual-check interval (1, 2, 4 or 8)
    int source = EM_PLAN_BUILTIN;
};
// Batch plans: (solver, FP16 points) -> routing of the sliced classes and arm factor.
using BatchPlanKey = std::pair<int, int>;
struct BatchPlan {
    uint64_t mask = 0;
    float arm = 1.0f;
    int check = 1;
    int host_counts = 0;
    int source = EM_PLAN_BUILTIN;
};

struct em_context {
    int device = 0;
    int num_cus = 0;
    std::string arch;                   // gcnArchName of the device (cache key)
    std::map<PlanKey, NlemPlan> plans;  // measured by nlem_autotune, loaded from the cache or set
    std::map<BatchPlanKey, BatchPlan> batch_plans;   // em_batch_autotune / cache / em_batch_plan_set
    int plan_epoch = 0;                 // bumped when a plan changes (invalidates the multi graph)
    unsigned int *counters = nullptr;  // kNumCounters work-queue heads
    int num_counters = 0;
    char last_error[512] = {0};         // message of the last failed call (fixed storage)
    std::map<const void *, int> occupancy;
    MultiGraph multi;
    // batch workspace (grown on demand)
    void *ws = nullptr;
    size_t ws_bytes = 0;
    // plain-path workspace
    void *plain_ws = nullptr;
    size_t plain_ws_bytes = 0;
    // class counts read back under a plan with host_counts (pinned, on first use)
    unsigned int *host_counts = nullptr;
    // side streams for concurrent shape-class launches (created on first use)
    hipStream_t side[kSideStreams] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[kSideStreams] = {};
    // nlem_denoise_noalloc: this device's address of the static scratch array
    // (set by em_create; null when the device index is beyond kScratchDevices)
    void *noalloc = nullptr;
    // em_kernel_timing: event pairs around the NLEM solve launches
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> tev;
    size_t tev_used = 0;
};

// Error messages go to the handle's fixed buffer (no allocation on any path).
static em_status_t fail(em_context *ctx, em_status_t st, const char *msg) {
    if (ctx) snprintf(ctx->last_error, sizeof(ctx->last_error), "%s", msg);
    return st;
}

static em_status_t hip_fail(em_context *ctx, hipError_t e, const char *what) {
    if (ctx) snprintf(ctx->last_error, sizeof(ctx->last_error), "%s: %s", what, hipGetErrorString(e));
    return EM_ERR_HIP;
}

#define EMX_HIP(ctx, call)                                  \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, #call); \
    } while (0)

namespace emx {

// Resident workgroups per CU of a kernel, cached per handle; with
// cache = false a kernel not yet cached is measured without being added
// (no host allocation: the entry point that allocates nothing uses this).
int blocks_per_cu(em_context *ctx, const void *fn, int threads, bool cache) {
    auto it = ctx->occupancy.find(fn);
    if (it != ctx->occupancy.end()) return it->second;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, threads, 0) != hipSuccess || nb < 1) nb = 1;
    if (cache) ctx->occupancy[fn] = nb;
    return nb;
}

int blocks_per_cu(em_context *ctx, const void *fn, int threads) { return blocks_per_cu(ctx, fn, threads, true); }

int ctx_num_cus(em_context *ctx) { return ctx->num_cus; }

// The handle's side streams (default priority, non-blocking) and their
// fork/join events, created on first use.
em_status_t ctx_side_streams(em_context *ctx, hipStream_t **side, hipEvent_t *fork, hipEvent_t **join) {
    if (!ctx->fork) {
        for (int i = 0; i < kSideStreams; ++i) {
            if (!ctx->side[i]) EMX_HIP(ctx, hipStreamCreateWithFlags(&ctx->side[i], hipStreamNonBlocking));
            if (!ctx->join[i]) EMX_HIP(ctx, hipEventCreateWithFlags(&ctx->join[i], hipEventDisableTiming));
        }
        EMX_HIP(ctx, hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming));
    }
    *side = ctx->side;
    *fork = ctx->fork;
    *join = ctx->join;
    return EM_OK;
}
int ctx_device(em_context *ctx) { return ctx->device; }

em_status_t ctx_error(em_context *ctx, em_status_t st, const char *msg) { return fail(ctx, st, msg); }

em_status_t ctx_hip_error(em_context *ctx, hipError_t e, const char *what) { return hip_fail(ctx, e, what); }

// Pinned host buffer of n class counts (allocated on first use).
unsigned int *ctx_host_counts(em_context *ctx, int n) {
    (void)n;   // kNumAllClasses + a few, well under the fixed size below
    if (!ctx->host_counts &&
        hipHostMalloc(reinterpret_cast<void **>(&ctx->host_counts), 256 * sizeof(unsigned int),
                      hipHostMallocDefault) != hipSuccess) {
        ctx->host_counts = nullptr;
    }
    return ctx->host_counts;
}

// The batch plan of a call: the handle's plan for the fixed-penalty EM-ADMM
// over a box and its point storage, else the built-in one.
BatchPlanView ctx_batch_plan(em_context *ctx, const em_options_t &o) {
    if (o.solver == EM_SOLVER_ADMM && o.set == EM_SET_BOX) {
        auto it = ctx->batch_plans.find(BatchPlanKey{EM_SOLVER_ADMM, o.points_f16 ? 1 : 0});
        if (it != ctx->batch_plans.end())
            return BatchPlanView{it->second.mask, it->second.arm, it->second.check, it->second.host_counts};
    }
    return BatchPlanView{0, 1.0f, 1, 0};
}

// Work-queue heads: a fixed pool owned by the handle.
unsigned int *ctx_counters(em_context *ctx, int n) {
    if (n > ctx->num_counters) return nullptr;
    return ctx->counters;
}

em_status_t ctx_reset_counters(em_context *ctx, hipStream_t s, unsigned int *c, int n) {
    hipLaunchKernelGGL(reset_counters_kernel, dim3((n + 255) / 256), dim3(256), 0, s, c, n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(ctx, e, "reset_counters launch");
    return EM_OK;
}

// Device workspace of at least `bytes` (grown by reallocation; previous
// contents are not preserved).  Synchronises the device before freeing.
void *ctx_workspace(em_context *ctx, size_t bytes, em_status_t *st) {
    *st = EM_OK;
    if (bytes <= ctx->ws_bytes) return ctx->ws;
    if (ctx->ws) {
        (void)hipDeviceSynchronize();
        (void)hipFree(ctx->ws);
        ctx->ws = nullptr;
        ctx->ws_bytes = 0;
    }
    size_t cap = bytes + bytes / 4 + 4096;
    if (hipMalloc(&ctx->ws, cap) != hipSuccess) {
        ctx->ws = nullptr;
        *st = fail(ctx, EM_ERR_OUT_OF_MEMORY, "workspace allocation failed");
        return nullptr;
    }
    ctx->ws_bytes = cap;
    return ctx->ws;
}

void *ctx_plain_workspace(em_context *ctx, size_t bytes, em_status_t *st) {
    *st = EM_OK;
    if (bytes <= ctx->plain_ws_bytes) return ctx->plain_ws;
    if (ctx->plain_ws) {
        (void)hipDeviceSynchronize();
        (void)hipFree(ctx->plain_ws);
        ctx->plain_ws = nullptr;
        ctx->plain_ws_bytes = 0;
    }
    size_t cap = bytes + 4096;
    if (hipMalloc(&ctx->plain_ws, cap) != hipSuccess) {
        ctx->plain_ws = nullptr;
        *st = fail(ctx, EM_ERR_OUT_OF_MEMORY, "plain workspace allocation failed");
        return nullptr;
    }
    ctx->plain_ws_bytes = cap;
    return ctx->plain_ws;
}

}  // namespace emx

// ---------------------------------------------------------------------------
// autotune cache: text lines in the file named by EMX_AUTOTUNE_CACHE,
//   nlem2 <arch> <patch radius> <points per lane> <solver> <fp16> <waves> <chunk> <order> <arm> <check>
//   batch <arch> <solver> <fp16> <routed classes, hex> <arm> <check> <host counts>
// (a missing check field reads as 1, a missing host-counts field as 0)
// and, from before the queue and arm fields existed,
//   nlem <arch> <patch radius> <points per lane> <solver> <waves>
// (both storages, built-in queue rules).  Later lines win; lines for another
// architecture, an uncompiled variant, values out of range or that do not
// parse are skipped.
// ---------------------------------------------------------------------------

static bool plan_values_ok(int chunk, int order, float arm, int check) {
    return chunk >= 0 && chunk <= 64 && order >= -1 && order <= 1 && std::isfinite(arm) && arm >= 1.0f &&
           (check == 1 || check == 2 || check == 4 || check == 8);
}

static constexpr uint64_t kAllWideClasses = ((uint64_t)1 << kNumWideClasses) - 1;

static void load_plan_cache(em_context *ctx) {
    const char *path = getenv("EMX_AUTOTUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = fopen(path, "r");
    if (!f) return;
    char line[256];
    while (fgets(line, sizeof(line), f)) {
        char kind[16], arch[64];
        int pr, m, solver, f16, wc, chunk, order, check = 1, hc = 0;
        float arm;
        unsigned long long mask;
        if (sscanf(line, "%15s %63s", kind, arch) != 2 || ctx->arch != arch) continue;
        if (strcmp(kind, "nlem2") == 0 &&
            sscanf(line, "%*s %*s %d %d %d %d %d %d %d %f %d", &pr, &m, &solver, &f16, &wc, &chunk, &order,
                   &arm, &check) >= 8) {
            if ((f16 == 0 || f16 == 1) && nlem_kernel(pr, m, wc, solver).fn &&
                plan_values_ok(chunk, order, arm, check))
                ctx->plans[PlanKey{pr, m, solver, f16}] = NlemPlan{wc, chunk, order, arm, check, EM_PLAN_CACHE};
        } else if (strcmp(kind, "nlem") == 0 &&
                   sscanf(line, "%*s %*s %d %d %d %d", &pr, &m, &solver, &wc) == 4) {
            if (nlem_kernel(pr, m, wc, solver).fn)
                for (int x = 0; x < 2; ++x)
                    ctx->plans[PlanKey{pr, m, solver, x}] = NlemPlan{wc, 0, -1, 1.0f, 1, EM_PLAN_CACHE};
        } else if (strcmp(kind, "batch") == 0 &&
                   sscanf(line, "%*s %*s %d %d %llx %f %d %d", &solver, &f16, &mask, &arm, &check, &hc) >= 4) {
            if (solver == EM_SOLVER_ADMM && (f16 == 0 || f16 == 1) && (mask & ~kAllWideClasses) == 0 &&
                plan_values_ok(0, -1, arm, check) && (hc == 0 || hc == 1))
                ctx->batch_plans[BatchPlanKey{solver, f16}] =
                    BatchPlan{(uint64_t)mask, arm, check, hc, EM_PLAN_CACHE};
        }
    }
    fclose(f);
}

static void append_cache_line(const char *text) {
    const char *path = getenv("EMX_AUTOTUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = fopen(path, "a");
    if (!f) return;
    fputs(text, f);
    fclose(f);
}

static void append_plan_cache(const em_context *ctx, const PlanKey &k, const NlemPlan &p) {
    char line[256];
    snprintf(line, sizeof(line), "nlem2 %s %d %d %d %d %d %d %d %.9g %d\n", ctx->arch.c_str(),
             std::get<0>(k), std::get<1>(k), std::get<2>(k), std::get<3>(k), p.wc, p.chunk, p.order,
             (double)p.arm, p.check);
    append_cache_line(line);
}

static void append_batch_plan_cache(const em_context *ctx, const BatchPlanKey &k, const BatchPlan &p) {
    char line[256];
    snprintf(line, sizeof(line), "batch %s %d %d %llx %.9g %d %d\n", ctx->arch.c_str(), k.first, k.second,
             (unsigned long long)p.mask, (double)p.arm, p.check, p.host_counts);
    append_cache_line(line);
}

// ---------------------------------------------------------------------------
// handle
// ---------------------------------------------------------------------------

static constexpr int kNumCounters = 512;

// ---------------------------------------------------------------------------
// Scratch of nlem_denoise_noalloc: a static device array, one copy per GPU,
// held until the process ends.  Layout: the work-queue head (first 256
// bytes), then the longest-first order scratch of up to
// EM_NOALLOC_MAX_PIXELS pixels (nlem_order_bytes).  Host code never passes
// the array's name to a kernel (on the host it is only a stand-in symbol):
// em_create looks up its device address once per device with the device
// current and every use goes through that address.
// ---------------------------------------------------------------------------
static constexpr size_t kScratchHeadBytes = 256;
static constexpr size_t kScratchBytes =
    kScratchHeadBytes + (size_t)EM_NOALLOC_MAX_PIXELS * (sizeof(int32_t) + 1) + 4096;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static constexpr int kScratchDevices = 64;
static void *g_scratch_addr[kScratchDevices] = {};
static std::mutex g_scratch_mu;

// The device address of `scratch` on `device` (the current device), looked
// up on the first call for that device.  *addr = null for device indices
// beyond kScratchDevices.
static hipError_t scratch_address(int device, void **addr) {
    *addr = nullptr;
    if (device < 0 || device >= kScratchDevices) return hipSuccess;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_addr[device] = p;
    }
    *addr = g_scratch_addr[device];
    return hipSuccess;
}

extern "C" em_status_t em_create(em_handle_t *handle, int device) {
    if (!handle) return EM_ERR_INVALID_ARG;
    *handle = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess) return EM_ERR_HIP;
    if (device < 0 || device >= ndev) return EM_ERR_INVALID_ARG;
    if (hipSetDevice(device) != hipSuccess) return EM_ERR_HIP;
    em_context *ctx = new (std::nothrow) em_context();
    if (!ctx) return EM_ERR_OUT_OF_MEMORY;
    ctx->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
        delete ctx;
        return EM_ERR_HIP;
    }
    ctx->num_cus = prop.multiProcessorCount;
    ctx->arch = prop.gcnArchName;
    {
        std::string a = ctx->arch;
        const size_t colon = a.find(':');
        if (colon != std::string::npos) ctx->arch = a.substr(0, colon);
    }
    load_plan_cache(ctx);
    if (scratch_address(device, &ctx->noalloc) != hipSuccess) {
        delete ctx;
        return EM_ERR_HIP;
    }
    if (hipMalloc(&ctx->counters, kNumCounters * sizeof(unsigned int)) != hipSuccess) {
        delete ctx;
        return EM_ERR_OUT_OF_MEMORY;
    }
    if (hipMemset(ctx->counters, 0, kNumCounters * sizeof(unsigned int)) != hipSuccess) {
        (void)hipFree(ctx->counters);
        delete ctx;
        return EM_ERR_HIP;
    }
    ctx->num_counters = kNumCounters;
    *handle = ctx;
    return EM_OK;
}

extern "C" em_status_t em_destroy(em_handle_t h) {
    if (!h) return EM_OK;
    (void)hipSetDevice(h->device);
    (void)hipDeviceSynchronize();
    if (h->multi.exec) (void)hipGraphExecDestroy(h->multi.exec);
    if (h->multi.graph) (void)hipGraphDestroy(h->multi.graph);
    if (h->multi.ws) (void)hipFree(h->multi.ws);
    if (h->counters) (void)hipFree(h->counters);
    if (h->ws) (void)hipFree(h->ws);
    if (h->plain_ws) (void)hipFree(h->plain_ws);
    if (h->host_counts) (void)hipHostFree(h->host_counts);
    for (int i = 0; i < kSideStreams; ++i) {
        if (h->side[i]) (void)hipStreamDestroy(h->side[i]);
        if (h->join[i]) (void)hipEventDestroy(h->join[i]);
    }
    if (h->fork) (void)hipEventDestroy(h->fork);
    for (auto &p : h->tev) {
        (void)hipEventDestroy(p.first);
        (void)hipEventDestroy(p.second);
    }
    delete h;
    return EM_OK;
}

extern "C" const char *em_status_string(em_status_t s) {
    switch (s) {
        case EM_OK: return "EM_OK";
        case EM_ERR_INVALID_ARG: return "EM_ERR_INVALID_ARG";
        case EM_ERR_UNSUPPORTED: return "EM_ERR_UNSUPPORTED";
        case EM_ERR_OUT_OF_MEMORY: return "EM_ERR_OUT_OF_MEMORY";
        case EM_ERR_HIP: return "EM_ERR_HIP";
    }
    return "EM_ERR_UNKNOWN";
}

extern "C" const char *em_last_error(em_handle_t h) { return h ? h->last_error : ""; }

extern "C" em_status_t em_sync(em_handle_t h, void *stream) {
    if (!h) return EM_ERR_INVALID_ARG;
    hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(h, e, "hipStreamSynchronize");
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(h, e, "asynchronous error");
    return EM_OK;
}

// ---------------------------------------------------------------------------
// NLEM
// ---------------------------------------------------------------------------

// The primal residual costs three VALU operations per point coordinate, so
// it is evaluated only on iterations that follow one whose dual residual was
// already within kArmFactor * tol * D (both must be within tol * D to stop).
static constexpr float kArmFactor = 1.0f;

// Queues shorter than this many rounds of the resident grid run, in
// tolerance mode, with the most coordinate waves compiled for the shape: the
// slowest pixels set the time of such a queue, and more waves per pixel
// finish each of them sooner.  Measured on 64x64 to 160x120 images against
// the default counts: 64x64 r2 R10 0.314 -> 0.165 ms, 64x64 r3 R7 0.491 ->
// 0.290 ms, 128x96 r2 R5 0.228 -> 0.206 ms; at a fixed iteration count
// (no tail) more waves were slower (64x64 r2 R5 T50 0.166 -> 0.175 ms).
static constexpr int kFewRounds = 4;

// The schedule of one NLEM launch: kernel (coordinate waves), queue
// positions per pop (0 = the size rule), queue order (-1 = the rule, 0 = off,
// 1 = on) and residual arm factor.
struct NlemSchedule {
    NlemKernelInfo k;
    int chunk;
    int order;
    float arm;
    int check;   // residual-check interval
};

static const NlemPlan *find_plan(const em_context *h, int pr, int m, int solver, int f16) {
    auto it = h->plans.find(PlanKey{pr, m, solver, f16 ? 1 : 0});
    return it == h->plans.end() ? nullptr : &it->second;
}

// Schedule for a shape, field by field: the environment override
// (EMX_NLEM_WC when that variant is compiled; EMX_NLEM_CHUNK and
// EMX_NLEM_ORDER act in queue_chunk and order_enabled), else the handle's
// plan, else the built-in default; without an override or plan, a short
// queue in tolerance mode (total pixels of the group >= 0 and below
// kFewRounds rounds) runs with the most coordinate waves compiled.
static NlemSchedule nlem_schedule(em_context *h, int pr, int m, int solver, int f16, int64_t total = -1,
                                  bool tolerance = false, bool cache = true) {
    const NlemPlan *plan = find_plan(h, pr, m, solver, f16);
    NlemSchedule r{NlemKernelInfo{nullptr, 0}, plan ? plan->chunk : 0, plan ? plan->order : -1,
                   plan ? plan->arm : kArmFactor, plan ? plan->check : 1};
    const char *env = getenv("EMX_NLEM_WC");
    if (env && *env) {
        r.k = nlem_kernel(pr, m, atoi(env), solver);
        if (r.k.fn) return r;
    }
    if (plan) {
        r.k = nlem_kernel(pr, m, plan->wc, solver);
        if (r.k.fn) return r;
    }
    r.k = nlem_kernel(pr, m, nlem_default_wc(pr, m, solver), solver);
    if (r.k.fn && tolerance && total >= 0 &&
        total < (int64_t)kFewRounds * h->num_cus * blocks_per_cu(h, r.k.fn, r.k.threads, cache)) {
        for (int wc = 4; wc > 0; --wc) {
            const NlemKernelInfo x = nlem_kernel(pr, m, wc, solver);
            if (x.fn) {
                if (x.threads > r.k.threads) r.k = x;
                break;
            }
        }
    }
    return r;
}

static em_status_t check_solver_params(em_context *ctx, float lo, float hi, float rho,
                                       int32_t max_iter, float tol) {
    if (!(rho > 0.0f) || !std::isfinite(rho)) return fail(ctx, EM_ERR_INVALID_ARG, "rho must be finite and > 0");
    if (max_iter < 0) return fail(ctx, EM_ERR_INVALID_ARG, "max_iter must be >= 0");
    if (!(tol >= 0.0f)) return fail(ctx, EM_ERR_INVALID_ARG, "tol must be >= 0 (not NaN)");
    if (std::isnan(lo) || std::isnan(hi) || lo > hi) return fail(ctx, EM_ERR_INVALID_ARG, "need lo <= hi");
    return EM_OK;
}

static em_status_t check_image(em_context *ctx, const nlem_image_t &im) {
    if (!im.img || !im.out) return fail(ctx, EM_ERR_INVALID_ARG, "img and out must be non-NULL");
    if (im.H < 1 || im.W < 1) return fail(ctx, EM_ERR_INVALID_ARG, "H and W must be >= 1");
    if (im.patch_radius < 0 || im.window_radius < 0)
        return fail(ctx, EM_ERR_INVALID_ARG, "radii must be >= 0");
    if (!(im.h_param > 0.0f) || !std::isfinite(im.h_param))
        return fail(ctx, EM_ERR_INVALID_ARG, "h must be finite and > 0");
    if (im.patch_radius > EM_MAX_PATCH_RADIUS || im.window_radius > EM_MAX_WINDOW_RADIUS)
        return fail(ctx, EM_ERR_UNSUPPORTED, "patch or window radius above the compiled limits");
    if (im.patch_radius >= im.H || im.patch_radius >= im.W)
        return fail(ctx, EM_ERR_INVALID_ARG, "patch radius must be < min(H, W)");
    if ((int64_t)im.H * im.W >= (int64_t)1 << 31) return fail(ctx, EM_ERR_UNSUPPORTED, "image too large");
    if ((const void *)im.out == im.img) return fail(ctx, EM_ERR_INVALID_ARG, "out must not alias img");
    return EM_OK;
}

static NlemImageDesc make_desc(const nlem_image_t &im) {
    NlemImageDesc d{};
    d.img = im.img;
    d.out = im.out;
    d.stats = im.stats;
    d.H = im.H;
    d.W = im.W;
    d.R = im.window_radius;
    d.is_f16 = im.img_is_f16 ? 1 : 0;
    const double h = im.h_param;
    d.k_h = (float)(1.4426950408889634 / (h * h));
    return d;
}

static void fill_common(NlemLaunch &L, const nlem_options_t &o) {
    L.max_iter = o.max_iter;
    L.inv_mu = (o.solver == NLEM_SOLVER_ADMM) ? 1.0f / o.rho : 0.0f;
    L.lo = o.lo;
    L.hi = o.hi;
    L.tau = o.tol * (o.hi - o.lo);
    L.tau_arm = kArmFactor * L.tau;
    L.init_nlm = (o.init == NLEM_INIT_NLM) ? 1 : 0;
    L.eps = o.eps;
}

static nlem_options_t admm_options(float lo, float hi, float rho, int32_t max_iter, float tol) {
    nlem_options_t o{};
    o.solver = NLEM_SOLVER_ADMM;
    o.init = NLEM_INIT_NOISY;
    o.lo = lo;
    o.hi = hi;
    o.rho = rho;
    o.eps = 1e-6f;
    o.max_iter = max_iter;
    o.tol = tol;
    return o;
}

static em_status_t check_options(em_context *ctx, const nlem_options_t *o) {
    if (!o) return fail(ctx, EM_ERR_INVALID_ARG, "options must be non-NULL");
    if (o->solver != NLEM_SOLVER_ADMM && o->solver != NLEM_SOLVER_IRLS)
        return fail(ctx, EM_ERR_INVALID_ARG, "bad solver");
    if (o->init != NLEM_INIT_NOISY && o->init != NLEM_INIT_NLM) return fail(ctx, EM_ERR_INVALID_ARG, "bad init");
    if (o->solver == NLEM_SOLVER_IRLS && (!(o->eps > 0.0f) || !std::isfinite(o->eps)))
        return fail(ctx, EM_ERR_INVALID_ARG, "eps must be finite and > 0");
    const float rho = (o->solver == NLEM_SOLVER_ADMM) ? o->rho : 1.0f;
    em_status_t st = check_solver_params(ctx, o->lo, o->hi, rho, o->max_iter, o->tol);
    if (st != EM_OK) return st;
    if (!std::isfinite(o->lo) || !std::isfinite(o->hi)) return fail(ctx, EM_ERR_INVALID_ARG, "nlem needs a finite box");
    return EM_OK;
}

static NlemLaunch make_launch(const NlemGroup &g, const nlem_image_t *images, const nlem_options_t &o,
                              unsigned int *counter) {
    NlemLaunch L;
    memset(&L, 0, sizeof(L));
    fill_common(L, o);
    L.count = (int)g.images.size();
    L.prefix[0] = 0;
    for (int k = 0; k < L.count; ++k) {
        const nlem_image_t &im = images[g.images[k]];
        L.img[k] = make_desc(im);
        L.prefix[k + 1] = L.prefix[k] + (int64_t)im.H * im.W;
    }
    L.counter = counter;
    L.chunk = 1;
    return L;
}

// Queue positions per atomic: about 24,576 point coordinates of work per
// pop (one pixel at d = 49, n = 441; up to 8 for small windows and patches),
// fewer when the queue would not give every resident workgroup enough
// chunks.  For pixels of at least 1,024 point coordinates (every shape from
// 3x3 patches with 11x11 windows up) at most 2 per pop and at least 5 chunks
// per workgroup: one global counter serves about 75 M pops/s, which capped
// medium images at one pixel per pop (400x300 r2 R5 1.76 ms, 0.99 ms with
// 2), while larger chunks only unbalanced the end of the queue (measured
// over 160x120 to 480x640 images with 3x3 to 7x7 patches and chunks of 1 to
// 8: 27.6 -> 25.0 ms summed, the best choice per case summing to 24.7 ms).
// Smaller pixels keep up to 8 per pop and 16 chunks per workgroup.
// EMX_NLEM_CHUNK (1..64), then a plan's chunk, override the rule.
static int queue_chunk(const NlemGroup &g, int64_t total, int64_t cap, int plan_chunk) {
    const char *env = getenv("EMX_NLEM_CHUNK");
    if (env && *env) {
        const int v = atoi(env);
        if (v >= 1 && v <= 64) return v;
    }
    if (plan_chunk >= 1 && plan_chunk <= 64) return plan_chunk;
    const int64_t side = 2 * (int64_t)g.pr + 1;
    const int64_t elems = side * side * (int64_t)g.m * 64;   // d times the window slots
    int64_t k = std::max<int64_t>(1, std::min<int64_t>(8, 24576 / std::max<int64_t>(1, elems)));
    int64_t min_chunks = 16;
    if (elems >= 1024) {
        k = std::min<int64_t>(k, 2);
        min_chunks = 5;
    }
    while (k > 1 && total < min_chunks * k * cap) --k;
    return (int)k;
}

// Longest-first queue order (see nlem_order.hip), on unless EMX_NLEM_ORDER=0;
// pointless at a fixed iteration count (tol = 0: every pixel then costs about
// the same), and for a queue not much longer than the resident workgroups
// (nearly every pixel starts at once, and the order kernels cost more than
// the tail they shorten): used from kOrderMinRounds rounds of the grid on.
// Measured on 64x64 to 320x240 images against a threshold of 8 rounds: 4
// rounds shortened most tails (64x64 r3 R10 0.557 -> 0.372 ms, 160x120 r2 R7
// 0.544 -> 0.375 ms) and lengthened two (128x96 r2 R7 0.236 -> 0.286 ms);
// ordering every queue lost more often.
static constexpr int kOrderMinRounds = 4;
// With patches of radius <= 2 (d <= 25) the standard deviation hardly
// predicts the iteration count (correlation 0.12-0.25 on a 128x96 image,
// against 0.84 at radius 3) and the counts have no long tail, so the order
// only shuffles the queue: that broke up clusters of slow pixels in queues of
// up to ~15 rounds (128x96 r2 R10 0.681 -> 0.448 ms) and cost time in longer
// ones (320x240 r2 R7 1.078 -> 1.370 ms); such queues are ordered below
// kOrderMaxRoundsSmallPatch rounds only.
static constexpr int kOrderMaxRoundsSmallPatch = 16;

// plan_order: a plan's choice (0 off, 1 on) or -1 for the rule below.
static bool use_order(bool enabled, int pr, int64_t total, int64_t cap, int plan_order) {
    if (!enabled || plan_order == 0) return false;
    if (plan_order == 1) return true;
    if (total < kOrderMinRounds * cap) return false;
    return pr >= 3 || total < kOrderMaxRoundsSmallPatch * cap;
}

static bool order_enabled(const nlem_options_t &o) {
    if (o.max_iter <= 0 || !(o.tol > 0.0f)) return false;
    const char *e = getenv("EMX_NLEM_ORDER");
    return !(e && e[0] == '0' && e[1] == '\0');
}

static int64_t group_pixels(const NlemGroup &g, const nlem_image_t *images) {
    int64_t t = 0;
    for (int i : g.images) t += (int64_t)images[i].H * images[i].W;
    return t;
}

// A launch takes the plan of FP16 storage when every image in it is FP16.
static int group_f16(const NlemGroup &g, const nlem_image_t *images) {
    for (int i : g.images)
        if (!images[i].img_is_f16) return 0;
    return g.images.empty() ? 0 : 1;
}

// Queue the order kernels of one launch (its pixel order lands in A.order).
static em_status_t queue_order(em_context *h, hipStream_t s, const NlemOrderArgs &A) {
    OrderKernel k[kOrderKernels];
    nlem_order_kernels(A, h->num_cus, k);
    for (const OrderKernel &x : k) {
        void *args[] = {const_cast<NlemOrderArgs *>(&A)};
        EMX_HIP(h, hipLaunchKernel(x.fn, dim3(x.grid), dim3(x.block), args, 0, s));
    }
    return EM_OK;
}

// Event pairs kept for em_kernel_timing before they must be read.
static constexpr size_t kMaxTimedLaunches = 4096;

// The event pair for the next timed launch on stream s, or none: timing is
// off, or s is being captured into a graph (events there would become graph
// nodes).
static em_status_t timing_pair(em_context *h, hipStream_t s, std::pair<hipEvent_t, hipEvent_t> **out) {
    *out = nullptr;
    if (!h->timing) return EM_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    EMX_HIP(h, hipStreamIsCapturing(s, &cs));
    if (cs != hipStreamCaptureStatusNone) return EM_OK;
    if (h->tev_used == h->tev.size()) {
        if (h->tev.size() >= kMaxTimedLaunches)
            return fail(h, EM_ERR_UNSUPPORTED, "em_kernel_timing: read the timings (em_kernel_timing_read) "
                                               "at least every 4096 launches");
        std::pair<hipEvent_t, hipEvent_t> p{nullptr, nullptr};
        EMX_HIP(h, hipEventCreate(&p.first));
        const hipError_t e = hipEventCreate(&p.second);
        if (e != hipSuccess) {
            (void)hipEventDestroy(p.first);
            return hip_fail(h, e, "hipEventCreate");
        }
        h->tev.push_back(p);
    }
    *out = &h->tev[h->tev_used];
    return EM_OK;
}

// Queue one persistent launch per (patch radius, points per lane) group of
// the images, each after the kernels that put its pixels in longest-first
// order (the first of them zeroes the work-queue head) or, without the
// order, a reset of the head.
static em_status_t nlem_run(em_context *h, hipStream_t s, int32_t count, const nlem_image_t *images,
                            const nlem_options_t &o) {
    auto groups = group_images(count, images);
    if ((int)groups.size() > h->num_counters) return fail(h, EM_ERR_UNSUPPORTED, "too many shape groups");
    em_status_t st = EM_OK;
    const bool ord = order_enabled(o);
    char *ws = nullptr;
    if (ord) {
        size_t bytes = 0;
        for (const NlemGroup &g : groups) bytes += nlem_order_bytes(group_pixels(g, images));
        ws = static_cast<char *>(ctx_workspace(h, bytes, &st));
        if (!ws) return st;
    }
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        const NlemGroup &g = groups[gi];
        const NlemSchedule sc = nlem_schedule(h, g.pr, g.m, o.solver, group_f16(g, images),
                                              group_pixels(g, images), o.max_iter > 0 && o.tol > 0.0f);
        const NlemKernelInfo k = sc.k;
        if (!k.fn) return fail(h, EM_ERR_UNSUPPORTED, "no compiled kernel for this shape and solver");
        NlemLaunch L = make_launch(g, images, o, h->counters + gi);
        L.tau_arm = sc.arm * L.tau;
        L.check_mask = sc.check - 1;
        const int64_t total = L.prefix[L.count];
        const int64_t cap = (int64_t)h->num_cus * blocks_per_cu(h, k.fn, k.threads);
        L.chunk = queue_chunk(g, total, cap, sc.chunk);
        if (use_order(ord, g.pr, total, cap, sc.order)) {
            const NlemOrderArgs A = nlem_order_args(L, g.pr, o.lo, o.hi, ws);
            st = queue_order(h, s, A);
            if (st != EM_OK) return st;
            L.order = A.order;
        } else {
            st = ctx_reset_counters(h, s, L.counter, 1);
            if (st != EM_OK) return st;
        }
        if (ord) ws += nlem_order_bytes(total);
        const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(total, cap));
        void *args[] = {&L};
        std::pair<hipEvent_t, hipEvent_t> *tp = nullptr;
        st = timing_pair(h, s, &tp);
        if (st != EM_OK) return st;
        if (tp) EMX_HIP(h, hipEventRecord(tp->first, s));
        EMX_HIP(h, hipLaunchKernel(k.fn, dim3(grid), dim3(k.threads), args, 0, s));
        if (tp) {
            EMX_HIP(h, hipEventRecord(tp->second, s));
            ++h->tev_used;
        }
    }
    return EM_OK;
}

extern "C" em_status_t em_kernel_timing(em_handle_t h, int32_t enable) {
    if (!h) return EM_ERR_INVALID_ARG;
    h->timing = enable != 0;
    h->tev_used = 0;
    return EM_OK;
}

extern "C" em_status_t em_kernel_timing_read(em_handle_t h, double *total_ms, int64_t *launches) {
    if (!h) return EM_ERR_INVALID_ARG;
    if (!total_ms || !launches) return fail(h, EM_ERR_INVALID_ARG, "total_ms and launches must be non-NULL");
    EMX_HIP(h, hipSetDevice(h->device));
    double sum = 0.0;
    for (size_t i = 0; i < h->tev_used; ++i) {
        EMX_HIP(h, hipEventSynchronize(h->tev[i].second));
        float ms = 0.0f;
        EMX_HIP(h, hipEventElapsedTime(&ms, h->tev[i].first, h->tev[i].second));
        sum += ms;
    }
    *total_ms = sum;
    *launches = (int64_t)h->tev_used;
    h->tev_used = 0;
    return EM_OK;
}

extern "C" em_status_t nlem_denoise(em_handle_t h, void *stream, const void *img, int32_t img_is_f16,
                                    int32_t H, int32_t W, int32_t patch_radius, int32_t window_radius,
                                    float h_param, float lo, float hi, float rho, int32_t max_iter,
                                    float tol, float *out, em_stats_t *stats) {
    if (!h) return EM_ERR_INVALID_ARG;
    nlem_image_t im{img, out, stats, H, W, patch_radius, window_radius, h_param, img_is_f16};
    em_status_t st = check_image(h, im);
    if (st != EM_OK) return st;
    const nlem_options_t o = admm_options(lo, hi, rho, max_iter, tol);
    st = check_options(h, &o);
    if (st != EM_OK) return st;
    EMX_HIP(h, hipSetDevice(h->device));
    return nlem_run(h, static_cast<hipStream_t>(stream), 1, &im, o);
}

extern "C" em_status_t nlem_denoise_noalloc(em_handle_t h, void *stream, const void *img, int32_t img_is_f16,
                                            int32_t H, int32_t W, int32_t patch_radius, int32_t window_radius,
                                            float h_param, float lo, float hi, float rho, int32_t max_iter,
                                            float tol, float *out, em_stats_t *stats) {
    if (!h) return EM_ERR_INVALID_ARG;
    nlem_image_t im{img, out, stats, H, W, patch_radius, window_radius, h_param, img_is_f16};
    em_status_t st = check_image(h, im);
    if (st != EM_OK) return st;
    const nlem_options_t o = admm_options(lo, hi, rho, max_iter, tol);
    st = check_options(h, &o);
    if (st != EM_OK) return st;
    const int64_t total = (int64_t)H * W;
    if (total > (int64_t)EM_NOALLOC_MAX_PIXELS)
        return fail(h, EM_ERR_UNSUPPORTED, "nlem_denoise_noalloc: H * W above EM_NOALLOC_MAX_PIXELS");
    if (!h->noalloc) return fail(h, EM_ERR_UNSUPPORTED, "nlem_denoise_noalloc: no scratch for this device index");
    EMX_HIP(h, hipSetDevice(h->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const NlemGroup g{patch_radius, points_per_lane(window_radius), {}, 0};   // no images listed: no allocation
    const NlemSchedule sc = nlem_schedule(h, g.pr, g.m, NLEM_SOLVER_ADMM, img_is_f16 ? 1 : 0, total,
                                          max_iter > 0 && tol > 0.0f, /*cache=*/false);
    const NlemKernelInfo k = sc.k;
    if (!k.fn) return fail(h, EM_ERR_UNSUPPORTED, "no compiled kernel for this shape");
    char *scr = static_cast<char *>(h->noalloc);
    unsigned int *counter = reinterpret_cast<unsigned int *>(scr);
    NlemLaunch L;
    memset(&L, 0, sizeof(L));
    fill_common(L, o);
    L.tau_arm = sc.arm * L.tau;
    L.check_mask = sc.check - 1;
    L.count = 1;
    L.img[0] = make_desc(im);
    L.prefix[0] = 0;
    L.prefix[1] = total;
    L.counter = counter;
    const int64_t cap = (int64_t)h->num_cus * blocks_per_cu(h, k.fn, k.threads, /*cache=*/false);
    L.chunk = queue_chunk(g, total, cap, sc.chunk);
    if (use_order(order_enabled(o), g.pr, total, cap, sc.order)) {
        if (kScratchHeadBytes + nlem_order_bytes(total) > kScratchBytes)
            return fail(h, EM_ERR_UNSUPPORTED, "nlem_denoise_noalloc: order scratch too small");
        const NlemOrderArgs A = nlem_order_args(L, g.pr, o.lo, o.hi, scr + kScratchHeadBytes);
        st = queue_order(h, s, A);   // its first kernel clears the bucket counters and the head
        if (st != EM_OK) return st;
        L.order = A.order;
    } else {
        st = ctx_reset_counters(h, s, counter, 1);
        if (st != EM_OK) return st;
    }
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(total, cap));
    void *args[] = {&L};
    EMX_HIP(h, hipLaunchKernel(k.fn, dim3(grid), dim3(k.threads), args, 0, s));
    return EM_OK;
}

extern "C" em_status_t nlem_denoise_ex(em_handle_t h, void *stream, int32_t count,
                                       const nlem_image_t *images, const nlem_options_t *opt) {
    if (!h) return EM_ERR_INVALID_ARG;
    if (count < 0 || (count > 0 && !images)) return fail(h, EM_ERR_INVALID_ARG, "bad image list");
    for (int i = 0; i < count; ++i) {
        em_status_t st = check_image(h, images[i]);
        if (st != EM_OK) return st;
    }
    em_status_t st = check_options(h, opt);
    if (st != EM_OK) return st;
    if (count == 0) return EM_OK;
    EMX_HIP(h, hipSetDevice(h->device));
    return nlem_run(h, static_cast<hipStream_t>(stream), count, images, *opt);
}

extern "C" em_status_t nlm_denoise(em_handle_t h, void *stream, const void *img, int32_t img_is_f16,
                                   int32_t H, int32_t W, int32_t patch_radius, int32_t window_radius,
                                   float h_param, float *out) {
    if (!h) return EM_ERR_INVALID_ARG;
    nlem_image_t im{img, out, nullptr, H, W, patch_radius, window_radius, h_param, img_is_f16};
    em_status_t st = check_image(h, im);
    if (st != EM_OK) return st;
    // the NLM patch as the starting point and no iterations: its centre is NLM
    nlem_options_t o = admm_options(0.0f, 1.0f, 1.0f, 0, 0.0f);
    o.init = NLEM_INIT_NLM;
    EMX_HIP(h, hipSetDevice(h->device));
    return nlem_run(h, static_cast<hipStream_t>(stream), 1, &im, o);
}

// Mean time (ms) of `repeats` calls of fn on stream s after one warm-up call
// (synchronous).
template <class F>
static em_status_t time_calls(em_context *h, hipStream_t s, int repeats, F fn, float *ms) {
    em_status_t st = fn();   // warm-up (workspace, occupancy queries, code objects)
    if (st != EM_OK) return st;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    EMX_HIP(h, hipEventCreate(&e0));
    hipError_t e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int r = 0; r < repeats && st == EM_OK && e == hipSuccess; ++r) st = fn();
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st != EM_OK) return st;
    if (e != hipSuccess) return hip_fail(h, e, "autotune timing");
    *ms = t / (float)repeats;
    return EM_OK;
}

// A candidate after the first stage replaces the best plan only when it is
// faster by more than this fraction (run-to-run noise is ~0.5% here) than
// the best plan timed again right before it: paired timings, so that the
// clock ramping up during the search does not favour later candidates.
static constexpr float kTuneMargin = 0.01f;

extern "C" em_status_t nlem_autotune(em_handle_t h, void *stream, const nlem_image_t *image,
                                     const nlem_options_t *opt, int32_t repeats, int32_t *chosen) {
    if (!h) return EM_ERR_INVALID_ARG;
    if (!image) return fail(h, EM_ERR_INVALID_ARG, "image must be non-NULL");
    em_status_t st = check_image(h, *image);
    if (st != EM_OK) return st;
    st = check_options(h, opt);
    if (st != EM_OK) return st;
    if (repeats < 1) return fail(h, EM_ERR_INVALID_ARG, "repeats must be >= 1");
    EMX_HIP(h, hipSetDevice(h->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int pr = image->patch_radius, m = points_per_lane(image->window_radius);
    const PlanKey key{pr, m, opt->solver, image->img_is_f16 ? 1 : 0};
    const bool tolerance = opt->max_iter > 0 && opt->tol > 0.0f;
    const auto prev = h->plans.find(key);
    const bool had = prev != h->plans.end();
    const NlemPlan old = had ? prev->second : NlemPlan{};
    auto run = [&]() { return nlem_run(h, s, 1, image, *opt); };
    NlemPlan best;
    float best_ms = 0.0f;
    // margin 0: keep the fastest (first stage); otherwise time the best plan
    // again, then the candidate, and keep the candidate when faster by margin
    auto trial = [&](const NlemPlan &p, float margin) -> em_status_t {
        em_status_t r = EM_OK;
        if (margin > 0.0f) {
            h->plans[key] = best;
            r = time_calls(h, s, repeats, run, &best_ms);
            if (r != EM_OK) return r;
        }
        h->plans[key] = p;
        float ms = 0.0f;
        r = time_calls(h, s, repeats, run, &ms);
        if (r == EM_OK && (best.wc == 0 || ms < (1.0f - margin) * best_ms)) {
            best = p;
            best_ms = ms;
        }
        return r;
    };
    // 1: the tile shape (every compiled coordinate-wave count, built-in queue rules)
    for (int wc = 1; wc <= 4 && st == EM_OK; ++wc)
        if (nlem_kernel(pr, m, wc, opt->solver).fn) st = trial(NlemPlan{wc, 0, -1, 1.0f, 1, EM_PLAN_TUNED}, 0.0f);
    // 2: queue positions per pop; 3: queue order; 4: residual arm factor
    const int chunks[] = {1, 2, 4, 8};
    for (int c : chunks) {
        if (st != EM_OK || best.wc == 0) break;
        NlemPlan p = best;
        p.chunk = c;
        st = trial(p, kTuneMargin);
    }
    for (int ord = 0; tolerance && ord <= 1 && st == EM_OK && best.wc != 0; ++ord) {
        NlemPlan p = best;
        p.order = ord;
        st = trial(p, kTuneMargin);
    }
    const float arms[] = {1.5f, 2.0f, 3.0f};
    for (float a : arms) {
        if (!tolerance || opt->solver != NLEM_SOLVER_ADMM || st != EM_OK || best.wc == 0) break;
        NlemPlan p = best;
        p.arm = a;
        st = trial(p, kTuneMargin);
    }
    // 5: residual-check interval
    const int checks[] = {2, 4, 8};
    for (int c : checks) {
        if (!tolerance || opt->solver != NLEM_SOLVER_ADMM || st != EM_OK || best.wc == 0) break;
        NlemPlan p = best;
        p.check = c;
        st = trial(p, kTuneMargin);
    }
    if (st != EM_OK || best.wc == 0) {
        if (had) h->plans[key] = old;
        else h->plans.erase(key);
        return st != EM_OK ? st : fail(h, EM_ERR_UNSUPPORTED, "no compiled kernel for this shape and solver");
    }
    best.source = EM_PLAN_TUNED;
    h->plans[key] = best;
    ++h->plan_epoch;
    append_plan_cache(h, key, best);
    if (chosen) *chosen = best.wc;
    return EM_OK;
}

static em_status_t check_plan_shape(em_context *h, int32_t pr, int32_t wr, int32_t solver) {
    if (pr < 0 || pr > EM_MAX_PATCH_RADIUS || wr < 0 || wr > EM_MAX_WINDOW_RADIUS ||
        (solver != NLEM_SOLVER_ADMM && solver != NLEM_SOLVER_IRLS))
        return fail(h, EM_ERR_INVALID_ARG, "bad shape or solver");
    return EM_OK;
}

extern "C" em_status_t nlem_plan(em_handle_t h, int32_t patch_radius, int32_t window_radius,
                                 int32_t solver, int32_t *waves) {
    if (!h || !waves) return EM_ERR_INVALID_ARG;
    em_status_t st = check_plan_shape(h, patch_radius, window_radius, solver);
    if (st != EM_OK) return st;
    const int m = points_per_lane(window_radius);
    const NlemPlan *p = find_plan(h, patch_radius, m, solver, 0);
    *waves = p ? p->wc : nlem_default_wc(patch_radius, m, solver);
    return EM_OK;
}

extern "C" em_status_t nlem_plan_get(em_handle_t h, int32_t patch_radius, int32_t window_radius,
                                     int32_t solver, int32_t img_is_f16, nlem_plan_t *plan) {
    if (!h || !plan) return EM_ERR_INVALID_ARG;
    em_status_t st = check_plan_shape(h, patch_radius, window_radius, solver);
    if (st != EM_OK) return st;
    const int m = points_per_lane(window_radius);
    const NlemPlan *p = find_plan(h, patch_radius, m, solver, img_is_f16);
    const NlemPlan b = p ? *p : NlemPlan{nlem_default_wc(patch_radius, m, solver), 0, -1, 1.0f, 1, EM_PLAN_BUILTIN};
    *plan = nlem_plan_t{b.wc, b.chunk, b.order, b.arm, b.check, b.source};
    return EM_OK;
}

extern "C" em_status_t nlem_plan_set(em_handle_t h, int32_t patch_radius, int32_t window_radius,
                                     int32_t solver, int32_t img_is_f16, const nlem_plan_t *plan) {
    if (!h) return EM_ERR_INVALID_ARG;
    em_status_t st = check_plan_shape(h, patch_radius, window_radius, solver);
    if (st != EM_OK) return st;
    const int m = points_per_lane(window_radius);
    const PlanKey key{patch_radius, m, solver, img_is_f16 ? 1 : 0};
    if (!plan) {
        h->plans.erase(key);
    } else {
        if (!nlem_kernel(patch_radius, m, plan->waves, solver).fn)
            return fail(h, EM_ERR_INVALID_ARG, "waves: no compiled kernel of that count for the shape");
        if (!plan_values_ok(plan->chunk, plan->order, plan->arm_factor, plan->check_every))
            return fail(h, EM_ERR_INVALID_ARG,
                        "chunk 0..64, order -1..1, a finite arm_factor >= 1 and check_every 1, 2, 4 or 8");
        h->plans[key] = NlemPlan{plan->waves, plan->chunk, plan->order, plan->arm_factor, plan->check_every,
                                 EM_PLAN_SET};
    }
    ++h->plan_epoch;
    return EM_OK;
}

static bool same_key(const std::vector<char> &a, const std::vector<char> &b) {
    return a.size() == b.size() && memcmp(a.data(), b.data(), a.size()) == 0;
}

extern "C" em_status_t nlem_denoise_multi(em_handle_t h, void *stream, int32_t count,
                                          const nlem_image_t *images, float lo, float hi, float rho,
                                          int32_t max_iter, float tol) {
    if (!h) return EM_ERR_INVALID_ARG;
    if (count < 0 || (count > 0 && !images)) return fail(h, EM_ERR_INVALID_ARG, "bad image list");
    for (int i = 0; i < count; ++i) {
        em_status_t st = check_image(h, images[i]);
        if (st != EM_OK) return st;
    }
    const nlem_options_t o = admm_options(lo, hi, rho, max_iter, tol);
    em_status_t st = check_options(h, &o);
    if (st != EM_OK) return st;
    if (count == 0) return EM_OK;
    EMX_HIP(h, hipSetDevice(h->device));
    hipStream_t s = static_cast<hipStream_t>(stream);

    const bool ord = order_enabled(o);
    std::vector<char> key(sizeof(nlem_image_t) * count + 5 * sizeof(float) + 2 * sizeof(int));
    memcpy(key.data(), images, sizeof(nlem_image_t) * count);
    float params[5] = {lo, hi, rho, (float)max_iter, tol};
    memcpy(key.data() + sizeof(nlem_image_t) * count, params, sizeof(params));
    const int flags[2] = {h->plan_epoch, ord ? 1 : 0};
    memcpy(key.data() + sizeof(nlem_image_t) * count + sizeof(params), flags, sizeof(flags));

    if (!h->multi.exec || !same_key(key, h->multi.key)) {
        // the old graph may still run on some stream before its scratch goes
        if (h->multi.exec || h->multi.ws) (void)hipDeviceSynchronize();
        if (h->multi.exec) (void)hipGraphExecDestroy(h->multi.exec);
        if (h->multi.graph) (void)hipGraphDestroy(h->multi.graph);
        if (h->multi.ws) (void)hipFree(h->multi.ws);
        h->multi.exec = nullptr;
        h->multi.graph = nullptr;
        h->multi.ws = nullptr;
        h->multi.key.clear();
        auto groups = group_images(count, images);
        if ((int)groups.size() > h->num_counters) return fail(h, EM_ERR_UNSUPPORTED, "too many shape groups");
        if (ord) {
            size_t bytes = 0;
            for (const NlemGroup &g : groups) bytes += nlem_order_bytes(group_pixels(g, images));
            if (hipMalloc(&h->multi.ws, bytes) != hipSuccess) {
                h->multi.ws = nullptr;
                return fail(h, EM_ERR_OUT_OF_MEMORY, "queue-order scratch allocation failed");
            }
        }
        char *ws = static_cast<char *>(h->multi.ws);
        hipGraph_t graph;
        EMX_HIP(h, hipGraphCreate(&graph, 0));
        // one chain per group: [order: clear (and the head), count, scatter] or a reset of the head -> NLEM
        auto add = [&](hipGraphNode_t *node, const hipGraphNode_t *dep, const void *fn, dim3 grid, dim3 block,
                       void **args, const char *what) -> em_status_t {
            hipKernelNodeParams p{};
            p.func = const_cast<void *>(fn);
            p.gridDim = grid;
            p.blockDim = block;
            p.sharedMemBytes = 0;
            p.kernelParams = args;
            p.extra = nullptr;
            hipError_t e = hipGraphAddKernelNode(node, graph, dep, dep ? 1 : 0, &p);
            if (e != hipSuccess) {
                (void)hipGraphDestroy(graph);
                return hip_fail(h, e, what);
            }
            return EM_OK;
        };
        for (size_t gi = 0; gi < groups.size(); ++gi) {
            const NlemGroup &g = groups[gi];
            const NlemSchedule sc = nlem_schedule(h, g.pr, g.m, NLEM_SOLVER_ADMM, group_f16(g, images),
                                                  group_pixels(g, images), o.max_iter > 0 && o.tol > 0.0f);
            const NlemKernelInfo k = sc.k;
            if (!k.fn) {
                (void)hipGraphDestroy(graph);
                return fail(h, EM_ERR_UNSUPPORTED, "no compiled kernel for this shape");
            }
            unsigned int *counter = h->counters + gi;
            NlemLaunch L = make_launch(g, images, o, counter);
            L.tau_arm = sc.arm * L.tau;
            L.check_mask = sc.check - 1;
            hipGraphNode_t prev;
            const int64_t total = L.prefix[L.count];
            const int64_t cap = (int64_t)h->num_cus * blocks_per_cu(h, k.fn, k.threads);
            L.chunk = queue_chunk(g, total, cap, sc.chunk);
            if (use_order(ord, g.pr, total, cap, sc.order)) {
                // the first order kernel also zeroes the work-queue head
                const NlemOrderArgs A = nlem_order_args(L, g.pr, o.lo, o.hi, ws);
                OrderKernel ok[kOrderKernels];
                nlem_order_kernels(A, h->num_cus, ok);
                for (int i = 0; i < kOrderKernels; ++i) {
                    const OrderKernel &x = ok[i];
                    void *oargs[] = {const_cast<NlemOrderArgs *>(&A)};
                    hipGraphNode_t nn;
                    st = add(&nn, i ? &prev : nullptr, x.fn, dim3(x.grid), dim3(x.block), oargs,
                             "hipGraphAddKernelNode(order)");
                    if (st != EM_OK) return st;
                    prev = nn;
                }
                L.order = A.order;
            } else {
                int one = 1;
                void *rargs[] = {&counter, &one};
                st = add(&prev, nullptr, reinterpret_cast<const void *>(&reset_counters_kernel), dim3(1), dim3(64),
                         rargs, "hipGraphAddKernelNode(reset)");
                if (st != EM_OK) return st;
            }
            if (ord) ws += nlem_order_bytes(total);
            void *kargs[] = {&L};
            hipGraphNode_t knode;
            st = add(&knode, &prev, k.fn, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(total, cap))),
                     dim3(k.threads), kargs, "hipGraphAddKernelNode(nlem)");
            if (st != EM_OK) return st;
        }
        hipGraphExec_t exec;
        hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return hip_fail(h, e, "hipGraphInstantiate");
        }
        h->multi.graph = graph;
        h->multi.exec = exec;
        h->multi.key = key;
    }
    EMX_HIP(h, hipGraphLaunch(h->multi.exec, s));
    return EM_OK;
}

// ---------------------------------------------------------------------------
// batch and plain
// ---------------------------------------------------------------------------

static em_status_t check_batch_args(em_context *h, int64_t B, const float *a, const float *w,
                                    const em_instance_t *inst, float *z, float lo, float hi,
                                    float rho, int32_t max_iter, float tol, int32_t init) {
    if (B < 0) return fail(h, EM_ERR_INVALID_ARG, "B must be >= 0");
    if (B > 0 && (!a || !w || !inst || !z)) return fail(h, EM_ERR_INVALID_ARG, "NULL array with B > 0");
    if (B >= ((int64_t)1 << 31)) return fail(h, EM_ERR_UNSUPPORTED, "B too large");
    if (init != EM_INIT_GIVEN && init != EM_INIT_MAXW && init != EM_INIT_WMEAN)
        return fail(h, EM_ERR_INVALID_ARG, "bad init");
    return check_solver_params(h, lo, hi, rho, max_iter, tol);
}

extern "C" em_status_t em_solve_batch(em_handle_t h, void *stream, int64_t B, const float *a,
                                      const float *w, const em_instance_t *inst, float lo, float hi,
                                      float rho, int32_t max_iter, float tol, int32_t init, float *z,
                                      em_stats_t *stats) {
    if (!h) return EM_ERR_INVALID_ARG;
    em_status_t st = check_batch_args(h, B, a, w, inst, z, lo, hi, rho, max_iter, tol, init);
    if (st != EM_OK) return st;
    if (B == 0) return EM_OK;
    EMX_HIP(h, hipSetDevice(h->device));
    em_options_t o{};
    o.solver = EM_SOLVER_ADMM;
    o.init = init;
    o.lo = lo;
    o.hi = hi;
    o.rho = rho;
    o.eps = 1e-6f;
    o.max_iter = max_iter;
    o.tol = tol;
    return batch_solve(h, static_cast<hipStream_t>(stream), B, a, w, inst, o, z, stats);
}

extern "C" em_status_t em_solve_batch_ex(em_handle_t h, void *stream, int64_t B, const float *a,
                                         const float *w, const em_instance_t *inst,
                                         const em_options_t *opt, float *z, em_stats_t *stats) {
    if (!h) return EM_ERR_INVALID_ARG;
    if (!opt) return fail(h, EM_ERR_INVALID_ARG, "options must be non-NULL");
    const em_options_t &o = *opt;
    if (o.solver != EM_SOLVER_ADMM && o.solver != EM_SOLVER_IRLS && o.solver != EM_SOLVER_ADMM_ADAPTIVE &&
        o.solver != EM_SOLVER_ADMM_WEIGHTED && o.solver != EM_SOLVER_ADMM_FAST)
        return fail(h, EM_ERR_INVALID_ARG, "bad solver");
    if (o.solver == EM_SOLVER_ADMM_FAST && !(o.fast_eta > 0.0f && o.fast_eta < 1.0f))
        return fail(h, EM_ERR_INVALID_ARG, "fast_eta must be in (0, 1)");
    if (o.solver == EM_SOLVER_ADMM_FAST && o.set == EM_SET_BALL)
        return fail(h, EM_ERR_UNSUPPORTED, "the accelerated ADMM runs over boxes");
    if ((o.box_lo == nullptr) != (o.box_hi == nullptr))
        return fail(h, EM_ERR_INVALID_ARG, "box_lo and box_hi must both be NULL or both be set");
    if (o.solver == EM_SOLVER_IRLS && (!(o.eps > 0.0f) || !std::isfinite(o.eps)))
        return fail(h, EM_ERR_INVALID_ARG, "eps must be finite and > 0");
    if (o.solver == EM_SOLVER_ADMM_ADAPTIVE &&
        (o.adapt_every < 1 || !(o.adapt_ratio > 1.0f) || !(o.adapt_factor > 1.0f) ||
         !std::isfinite(o.adapt_ratio) || !std::isfinite(o.adapt_factor)))
        return fail(h, EM_ERR_INVALID_ARG, "adaptive penalty needs adapt_every >= 1, ratio > 1, factor > 1");
    if (o.set != EM_SET_BOX && o.set != EM_SET_BALL) return fail(h, EM_ERR_INVALID_ARG, "bad set");
    if (o.set == EM_SET_BALL && o.box_lo) return fail(h, EM_ERR_INVALID_ARG, "a ball takes no box arrays");
    if (o.set == EM_SET_BALL && o.solver == EM_SOLVER_ADMM_ADAPTIVE)
        return fail(h, EM_ERR_UNSUPPORTED, "the ball is supported with ADMM and IRLS");
    if (o.set == EM_SET_BALL && !o.ball_radius && !(o.radius >= 0.0f))
        return fail(h, EM_ERR_INVALID_ARG, "radius must be >= 0");
    const bool scalar_box = o.set == EM_SET_BOX && !o.box_lo;
    const float lo = scalar_box ? o.lo : 0.0f, hi = scalar_box ? o.hi : 0.0f;
    const float rho = (o.solver == EM_SOLVER_IRLS) ? 1.0f : o.rho;
    em_status_t st = check_batch_args(h, B, a, w, inst, z, lo, hi, rho, o.max_iter, o.tol, o.init);
    if (st != EM_OK) return st;
    if (B == 0) return EM_OK;
    EMX_HIP(h, hipSetDevice(h->device));
    return batch_solve(h, static_cast<hipStream_t>(stream), B, a, w, inst, o, z, stats);
}

extern "C" em_status_t em_batch_autotune(em_handle_t h, void *stream, int64_t B, const float *a,
                                         const float *w, const em_instance_t *inst, const em_options_t *opt,
                                         float *z, em_stats_t *stats, int32_t repeats, em_batch_plan_t *chosen) {
    if (!h) return EM_ERR_INVALID_ARG;
    if (!opt) return fail(h, EM_ERR_INVALID_ARG, "options must be non-NULL");
    if (repeats < 1) return fail(h, EM_ERR_INVALID_ARG, "repeats must be >= 1");
    if (opt->solver != EM_SOLVER_ADMM || opt->set != EM_SET_BOX)
        return fail(h, EM_ERR_UNSUPPORTED, "em_batch_autotune: the fixed-penalty EM-ADMM over a box");
    const BatchPlanKey key{EM_SOLVER_ADMM, opt->points_f16 ? 1 : 0};
    const auto prev = h->batch_plans.find(key);
    const bool had = prev != h->batch_plans.end();
    const BatchPlan old = had ? prev->second : BatchPlan{};
    h->batch_plans.erase(key);
    // validates the arguments like any call, before anything is timed
    em_status_t st = em_solve_batch_ex(h, stream, B, a, w, inst, opt, z, stats);
    if (st != EM_OK || B == 0) {
        if (had) h->batch_plans[key] = old;
        if (st == EM_OK && chosen) *chosen = em_batch_plan_t{old.mask, old.arm, old.check, old.host_counts, old.source};
        return st;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    unsigned int counts[kNumWideClasses];
    st = batch_wide_counts(h, s, B, inst, counts);
    auto run = [&]() { return em_solve_batch_ex(h, stream, B, a, w, inst, opt, z, stats); };
    BatchPlan best;
    float best_ms = 0.0f;
    bool have = false;
    auto trial = [&](const BatchPlan &p, float margin) -> em_status_t {
        em_status_t r = EM_OK;
        if (margin > 0.0f && have) {   // paired timing, as in nlem_autotune
            h->batch_plans[key] = best;
            r = time_calls(h, s, repeats, run, &best_ms);
            if (r != EM_OK) return r;
        }
        h->batch_plans[key] = p;
        float ms = 0.0f;
        r = time_calls(h, s, repeats, run, &ms);
        if (r == EM_OK && (!have || ms < (1.0f - margin) * best_ms)) {
            best = p;
            best_ms = ms;
            have = true;
        }
        return r;
    };
    if (st == EM_OK) st = trial(BatchPlan{0, 1.0f, 1, 0, EM_PLAN_TUNED}, 0.0f);
    // each populated sliced class in the generic classes, largest first
    int order[kNumWideClasses];
    int npop = 0;
    for (int k = 0; k < kNumWideClasses; ++k)
        if (counts[k] > 0) order[npop++] = k;
    std::sort(order, order + npop, [&](int x, int y) { return counts[x] > counts[y]; });
    for (int i = 0; i < npop && st == EM_OK; ++i) {
        BatchPlan p = best;
        p.mask |= (uint64_t)1 << order[i];
        st = trial(p, kTuneMargin);
    }
    const float arms[] = {1.5f, 2.0f, 3.0f};
    for (float arm : arms) {
        if (!(opt->tol > 0.0f) || opt->max_iter <= 0 || st != EM_OK) break;
        BatchPlan p = best;
        p.arm = arm;
        st = trial(p, kTuneMargin);
    }
    const int checks[] = {2, 4, 8};
    for (int c : checks) {
        if (!(opt->tol > 0.0f) || opt->max_iter <= 0 || st != EM_OK) break;
        BatchPlan p = best;
        p.check = c;
        st = trial(p, kTuneMargin);
    }
    if (st == EM_OK) {   // the dispatch: class counts read back, populated classes only
        BatchPlan p = best;
        p.host_counts = 1;
        st = trial(p, kTuneMargin);
    }
    if (st != EM_OK || !have) {
        if (had) h->batch_plans[key] = old;
        else h->batch_plans.erase(key);
        return st != EM_OK ? st : fail(h, EM_ERR_HIP, "em_batch_autotune: no timing");
    }
    best.source = EM_PLAN_TUNED;
    h->batch_plans[key] = best;
    append_batch_plan_cache(h, key, best);
    if (chosen) *chosen = em_batch_plan_t{best.mask, best.arm, best.check, best.host_counts, best.source};
    return EM_OK;
}

extern "C" em_status_t em_batch_plan_get(em_handle_t h, int32_t solver, int32_t points_f16,
                                         em_batch_plan_t *plan) {
    if (!h || !plan) return EM_ERR_INVALID_ARG;
    if (solver != EM_SOLVER_ADMM) return fail(h, EM_ERR_INVALID_ARG, "batch plans are for EM_SOLVER_ADMM");
    auto it = h->batch_plans.find(BatchPlanKey{EM_SOLVER_ADMM, points_f16 ? 1 : 0});
    const BatchPlan b = (it != h->batch_plans.end()) ? it->second : BatchPlan{};
    *plan = em_batch_plan_t{b.mask, b.arm, b.check, b.host_counts, b.source};
    return EM_OK;
}

extern "C" em_status_t em_batch_plan_set(em_handle_t h, int32_t solver, int32_t points_f16,
                                         const em_batch_plan_t *plan) {
    if (!h) return EM_ERR_INVALID_ARG;
    if (solver != EM_SOLVER_ADMM) return fail(h, EM_ERR_INVALID_ARG, "batch plans are for EM_SOLVER_ADMM");
    const BatchPlanKey key{EM_SOLVER_ADMM, points_f16 ? 1 : 0};
    if (!plan) {
        h->batch_plans.erase(key);
        return EM_OK;
    }
    if ((plan->generic_classes & ~kAllWideClasses) != 0)
        return fail(h, EM_ERR_INVALID_ARG, "generic_classes: bits above the sliced classes");
    if (!plan_values_ok(0, -1, plan->arm_factor, plan->check_every) ||
        (plan->host_counts != 0 && plan->host_counts != 1))
        return fail(h, EM_ERR_INVALID_ARG,
                    "arm_factor must be finite and >= 1, check_every 1, 2, 4 or 8, host_counts 0 or 1");
    h->batch_plans[key] =
        BatchPlan{plan->generic_classes, plan->arm_factor, plan->check_every, plan->host_counts, EM_PLAN_SET};
    return EM_OK;
}

extern "C" em_status_t em_solve_plain(em_handle_t h, void *stream, int64_t B, const float *a,
                                      const float *w, const em_instance_t *inst,
                                      const em_instance_t *inst_host, float lo, float hi, float rho,
                                      int32_t max_iter, float tol, int32_t init, float *z,
                                      em_stats_t *stats) {
    if (!h) return EM_ERR_INVALID_ARG;
    em_status_t st = check_batch_args(h, B, a, w, inst, z, lo, hi, rho, max_iter, tol, init);
    if (st != EM_OK) return st;
    if (B > 0 && !inst_host) return fail(h, EM_ERR_INVALID_ARG, "inst_host is required");
    if (B == 0) return EM_OK;
    EMX_HIP(h, hipSetDevice(h->device));
    em_options_t o{};
    o.solver = EM_SOLVER_ADMM;
    o.init = init;
    o.lo = lo;
    o.hi = hi;
    o.rho = rho;
    o.max_iter = max_iter;
    o.tol = tol;
    return plain_solve(h, static_cast<hipStream_t>(stream), B, a, w, inst, inst_host, o, z, stats);
}

extern "C" em_status_t em_solve_plain_ex(em_handle_t h, void *stream, int64_t B, const float *a,
                                         const float *w, const em_instance_t *inst,
                                         const em_instance_t *inst_host, const em_options_t *opt,
                                         float *z, em_stats_t *stats) {
    if (!h) return EM_ERR_INVALID_ARG;
    if (!opt) return fail(h, EM_ERR_INVALID_ARG, "options must be non-NULL");
    const em_options_t &o = *opt;
    if (o.solver == EM_SOLVER_IRLS || o.solver == EM_SOLVER_ADMM_ADAPTIVE || o.solver == EM_SOLVER_ADMM_WEIGHTED)
        return fail(h, EM_ERR_UNSUPPORTED, "this solver runs in em_solve_batch_ex");
    if (o.solver != EM_SOLVER_ADMM && o.solver != EM_SOLVER_ADMM_FAST)
        return fail(h, EM_ERR_INVALID_ARG, "bad solver");
    if (o.set == EM_SET_BALL) return fail(h, EM_ERR_UNSUPPORTED, "the ball runs in em_solve_batch_ex");
    if (o.points_f16) return fail(h, EM_ERR_UNSUPPORTED, "FP16 points run in em_solve_batch_ex");
    if (o.set != EM_SET_BOX) return fail(h, EM_ERR_INVALID_ARG, "bad set");
    if ((o.box_lo == nullptr) != (o.box_hi == nullptr))
        return fail(h, EM_ERR_INVALID_ARG, "box_lo and box_hi must both be NULL or both be set");
    if (o.solver == EM_SOLVER_ADMM_FAST && !(o.fast_eta > 0.0f && o.fast_eta < 1.0f))
        return fail(h, EM_ERR_INVALID_ARG, "fast_eta must be in (0, 1)");
    const float lo = o.box_lo ? 0.0f : o.lo, hi = o.box_lo ? 0.0f : o.hi;
    em_status_t st = check_batch_args(h, B, a, w, inst, z, lo, hi, o.rho, o.max_iter, o.tol, o.init);
    if (st != EM_OK) return st;
    if (B > 0 && !inst_host) return fail(h, EM_ERR_INVALID_ARG, "inst_host is required");
    if (B == 0) return EM_OK;
    EMX_HIP(h, hipSetDevice(h->device));
    return plain_solve(h, static_cast<hipStream_t>(stream), B, a, w, inst, inst_host, o, z, stats);
}
