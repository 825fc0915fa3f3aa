// Batched persistent launch of the fused forward / loss / adjoint tiles for
// many images of different sizes and filter parameters.
//
// Work items live in a device list: every forward tile of every image
// (longest first), then one SSD-loss reduction per image, then every adjoint
// tile (longest first).  A fixed grid of workgroups, one per compute unit,
// pulls item indices from an atomic counter.  Loss and adjoint items first
// wait until all forward tiles of their image have been counted done; since
// those tiles were handed out earlier to workgroups that never wait on later
// items, the waits always end.  Each wait is nevertheless bounded: on
// overrun a flag is raised (bf_batch_check) and the kernel still drains.
#include <algorithm>
#include <vector>

#include "bf_tile.h"

namespace bf {

enum ItemKind { kItemFwd = 0, kItemLoss = 1, kItemBwd = 2 };

struct BatchItem {
    int img, kind, tile;
};

struct BatchDev {
    const TileArgs* jobs;    // 2 per image: forward, adjoint
    const BatchItem* items;
    int n_items;
    const int* fwd_tiles;    // per image
    const int* part_base;    // per image: first loss partial
    const float* loss_part;
    float* loss;             // per image, or NULL
    unsigned* counters;      // [0] next item, [1] overrun flag, [2 + i] forward tiles done
    unsigned spin_limit;
};

constexpr int kBatchCounters0 = 2;

__global__ void bf_batch_reset(unsigned* counters, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        counters[i] = 0u;
}

__global__ void __launch_bounds__(kTileThreads)
bf_batch_kernel(const BatchDev d) {
    extern __shared__ __align__(16) float smem[];
    __shared__ __align__(16) int item_sh;
    const int t = threadIdx.x;
    for (;;) {
        if (t == 0) item_sh = (int)atomicAdd(&d.counters[0], 1u);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(item_sh);   // wave-uniform
        __syncthreads();
        if (it >= d.n_items) break;   // uniform: every wave leaves here
        BatchItem w = d.items[it];
        w.img = __builtin_amdgcn_readfirstlane(w.img);
        w.kind = __builtin_amdgcn_readfirstlane(w.kind);
        w.tile = __builtin_amdgcn_readfirstlane(w.tile);
        if (w.kind != kItemFwd) {
            if (t == 0) {
                const unsigned need = (unsigned)d.fwd_tiles[w.img];
                unsigned spins = 0;
                while (__hip_atomic_load(&d.counters[kBatchCounters0 + w.img], __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT) < need) {
                    if (++spins > d.spin_limit) {
                        atomicOr(&d.counters[1], 1u);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(4);
                }
            }
            __syncthreads();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        if (w.kind == kItemFwd) {
            tile_body<kForward, true>(d.jobs[2 * w.img], w.tile, smem);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __syncthreads();
            if (t == 0) atomicAdd(&d.counters[kBatchCounters0 + w.img], 1u);
        } else if (w.kind == kItemLoss) {
            if (t == 0 && d.loss) {
                double s = 0.0;
                const int b = d.part_base[w.img], nt = d.fwd_tiles[w.img];
                for (int k = 0; k < nt; ++k) s += (double)d.loss_part[b + k];
                d.loss[w.img] = (float)s;
            }
        } else {
            tile_body<kBackward, false>(d.jobs[2 * w.img + 1], w.tile, smem);
        }
        __syncthreads();
    }
}

}  // namespace bf

using namespace bf;

struct bf_batch_plan {
    int n = 0;
    std::vector<RangeParams> rp;
    std::vector<SpatialParams> sp;
    std::vector<TileGeom> gf, gb;
    std::vector<bf_image_desc> desc;
    std::vector<int> fwd_tiles, part_base;
    std::vector<size_t> aux_off;   // per image: offset of its P, Q planes in aux_d
    int total_parts = 0;
    int n_items = 0;
    int grid = 0;
    size_t lds = 0;
    bool bound = false;
    // device allocations (owned)
    TileArgs* jobs_d = nullptr;
    BatchItem* items_d = nullptr;
    int* fwd_tiles_d = nullptr;
    int* part_base_d = nullptr;
    float* loss_part_d = nullptr;
    unsigned* counters_d = nullptr;
    float* aux_d = nullptr;        // forward -> adjoint sums P, Q of every image
    float* loss = nullptr;
    StreamBatch* sb = nullptr;     // the streamed passes instead of the persistent kernel
};

static void free_plan(bf_batch_plan* p) {
    if (!p) return;
    stream_batch_destroy(p->sb);
    (void)hipFree(p->jobs_d);
    (void)hipFree(p->items_d);
    (void)hipFree(p->fwd_tiles_d);
    (void)hipFree(p->part_base_d);
    (void)hipFree(p->loss_part_d);
    (void)hipFree(p->counters_d);
    (void)hipFree(p->aux_d);
    delete p;
}

template <typename T>
static bf_status dev_alloc(T** ptr, size_t count) {
    if (hipMalloc((void**)ptr, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) {
        *ptr = nullptr;
        set_error("hipMalloc of %zu bytes failed", count * sizeof(T));
        return BF_ENOMEM;
    }
    return BF_OK;
}

static bool capturing() {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(nullptr, &cs) != hipSuccess) return false;
    return cs != hipStreamCaptureStatusNone;
}

extern "C" {

bf_status bf_batch_plan_create(const bf_image_desc* descs, int32_t n, bf_batch_plan** plan) {
    return bf_batch_plan_create_ex(descs, n, BF_PATH_AUTO, plan);
}

bf_status bf_batch_plan_create_ex(const bf_image_desc* descs, int32_t n, int32_t path,
                                  bf_batch_plan** plan) {
    if (!plan) {
        set_error("plan is NULL");
        return BF_EINVAL;
    }
    *plan = nullptr;
    if (!descs || n <= 0) {
        set_error("need n > 0 image descriptors");
        return BF_EINVAL;
    }
    if (path != BF_PATH_AUTO && path != BF_PATH_FUSED && path != BF_PATH_STREAMED) {
        set_error("path=%d is not one of BF_PATH_AUTO, BF_PATH_FUSED, BF_PATH_STREAMED", path);
        return BF_EINVAL;
    }
    if (path != BF_PATH_FUSED) {
        // the streamed passes: every image within their limits (AUTO), or
        // forced; tile overrides are ignored on this path
        std::vector<RangeParams> rp(n);
        std::vector<SpatialParams> sp(n);
        std::vector<int64_t> H(n), W(n);
        bool all = true;
        for (int i = 0; i < n; ++i) {
            const bf_image_desc& d = descs[i];
            bf_status st = BF_OK;
            if (d.H <= 0 || d.W <= 0 || d.H > (1 << 20) || d.W > (1 << 20)) {
                set_error("image %d: bad size %lld x %lld", i, (long long)d.H, (long long)d.W);
                st = BF_EINVAL;
            } else if ((st = make_spatial(&d.spatial, &sp[i])) == BF_OK &&
                       (st = make_range((double)d.T, (double)d.sigma_r, d.N, &rp[i])) == BF_OK &&
                       d.trunc_tol != 0.0f) {
                st = truncate_pairs(&rp[i], sp[i], (double)d.T, (double)d.trunc_tol, nullptr);
            }
            if (st != BF_OK) return st;
            H[i] = d.H;
            W[i] = d.W;
            all = all && stream_batch_supported(d.H, d.W, sp[i], rp[i].npairs);
        }
        if (all) {
            bf_batch_plan* p = new bf_batch_plan();
            p->n = n;
            p->desc.assign(descs, descs + n);
            const bf_status st = stream_batch_create(n, H.data(), W.data(), rp.data(), sp.data(),
                                                     &p->sb);
            if (st != BF_OK) {
                free_plan(p);
                return st;
            }
            *plan = p;
            return BF_OK;
        }
        if (path == BF_PATH_STREAMED) {
            set_error("an image of the batch is outside the streamed passes' limits");
            return BF_EUNSUPPORTED;
        }
    }
    bf_batch_plan* p = new bf_batch_plan();
    p->n = n;
    p->rp.resize(n);
    p->sp.resize(n);
    p->gf.resize(n);
    p->gb.resize(n);
    p->desc.assign(descs, descs + n);
    p->fwd_tiles.resize(n);
    p->part_base.resize(n);
    p->aux_off.resize(n);
    size_t aux_total = 0;
    for (int i = 0; i < n; ++i) {
        const bf_image_desc& d = descs[i];
        bf_status st;
        if (d.H <= 0 || d.W <= 0 || d.H > (1 << 20) || d.W > (1 << 20)) {
            set_error("image %d: bad size %lld x %lld", i, (long long)d.H, (long long)d.W);
            st = BF_EINVAL;
        } else if ((st = make_spatial(&d.spatial, &p->sp[i])) == BF_OK &&
                   (st = make_range((double)d.T, (double)d.sigma_r, d.N, &p->rp[i])) == BF_OK &&
                   (d.trunc_tol == 0.0f ||
                    (st = truncate_pairs(&p->rp[i], p->sp[i], (double)d.T, (double)d.trunc_tol,
                                         nullptr)) == BF_OK) &&
                   (st = plan_tiles(kForward, d.H, d.W, p->sp[i], d.tile_h, d.tile_w,
                                    &p->gf[i])) == BF_OK) {
            st = plan_tiles(kBackward, d.H, d.W, p->sp[i], d.bwd_tile_h, d.bwd_tile_w, &p->gb[i]);
        }
        if (st != BF_OK) {
            free_plan(p);
            return st;
        }
        p->fwd_tiles[i] = p->gf[i].tiles_x * p->gf[i].tiles_y;
        p->aux_off[i] = aux_total;
        aux_total += 2 * (size_t)d.H * d.W;
        p->part_base[i] = p->total_parts;
        p->total_parts += p->fwd_tiles[i];
        p->lds = std::max(p->lds, std::max(p->gf[i].lds_bytes, p->gb[i].lds_bytes));
    }
    p->lds = std::max<size_t>(p->lds, kTileThreads * sizeof(double));
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        set_error("cannot query the device");
        free_plan(p);
        return BF_EDEVICE;
    }
    p->grid = std::max(cus, 1);
    bf_status st;
    if ((st = dev_alloc(&p->jobs_d, 2 * (size_t)n)) != BF_OK ||
        (st = dev_alloc(&p->fwd_tiles_d, (size_t)n)) != BF_OK ||
        (st = dev_alloc(&p->part_base_d, (size_t)n)) != BF_OK ||
        (st = dev_alloc(&p->loss_part_d, (size_t)p->total_parts)) != BF_OK ||
        (st = dev_alloc(&p->counters_d, (size_t)kBatchCounters0 + n)) != BF_OK ||
        (st = dev_alloc(&p->aux_d, aux_total)) != BF_OK) {
        free_plan(p);
        return st;
    }
    size_t max_items = (size_t)p->total_parts + n;
    for (int i = 0; i < n; ++i) max_items += (size_t)p->gb[i].tiles_x * p->gb[i].tiles_y;
    if ((st = dev_alloc(&p->items_d, max_items)) != BF_OK) {
        free_plan(p);
        return st;
    }
    if (hipMemcpy(p->fwd_tiles_d, p->fwd_tiles.data(), n * sizeof(int), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(p->part_base_d, p->part_base.data(), n * sizeof(int), hipMemcpyHostToDevice) !=
            hipSuccess) {
        set_error("upload of the plan tables failed");
        free_plan(p);
        return BF_EDEVICE;
    }
    *plan = p;
    return BF_OK;
}

bf_status bf_batch_bind(bf_batch_plan* p, const float* const* f, const float* const* target,
                        float* const* out, float* const* eta, float* const* grad_f, float* loss) {
    if (!p || !f || !out) {
        set_error("plan, f and out are required");
        return BF_EINVAL;
    }
    if (capturing()) {
        set_error("bf_batch_bind uploads tables and cannot run during stream capture");
        return BF_ECAPTURE;
    }
    const bool bwd = grad_f != nullptr;
    if (bwd && (!target || !eta)) {
        set_error("the adjoint needs target and eta");
        return BF_EINVAL;
    }
    const int n = p->n;
    if (p->sb) {
        for (int i = 0; i < n; ++i) {
            const bf_image_desc& d = p->desc[i];
            const int64_t bytes = d.H * d.W * (int64_t)sizeof(float);
            if (!f[i] || !out[i] || (bwd && (!grad_f[i] || !target[i] || !eta[i])) ||
                overlaps(f[i], out[i], bytes) || (eta && overlaps(out[i], eta[i], bytes)) ||
                (bwd && (overlaps(grad_f[i], f[i], bytes) || overlaps(grad_f[i], out[i], bytes)))) {
                set_error("image %d: missing or overlapping buffers", i);
                return BF_EINVAL;
            }
        }
        const bf_status st = stream_batch_bind(p->sb, f, target, out, eta, grad_f, loss);
        p->bound = st == BF_OK;
        return st;
    }
    std::vector<TileArgs> jobs(2 * (size_t)n);
    struct Cost {
        double c;
        BatchItem w;
    };
    std::vector<Cost> fw, bw;
    for (int i = 0; i < n; ++i) {
        const bf_image_desc& d = p->desc[i];
        const int64_t bytes = d.H * d.W * (int64_t)sizeof(float);
        if (!f[i] || !out[i] || (bwd && (!grad_f[i] || !target[i] || !eta[i])) ||
            overlaps(f[i], out[i], bytes) || (eta && overlaps(out[i], eta[i], bytes)) ||
            (bwd && (overlaps(grad_f[i], f[i], bytes) || overlaps(grad_f[i], out[i], bytes)))) {
            set_error("image %d: missing or overlapping buffers", i);
            return BF_EINVAL;
        }
        TileArgs& a = jobs[2 * i];
        a = TileArgs{};
        a.f = f[i];
        a.out = out[i];
        a.eta = eta ? eta[i] : nullptr;
        a.target = target ? target[i] : nullptr;
        a.loss_part = target ? p->loss_part_d + p->part_base[i] : nullptr;
        a.aux = bwd ? p->aux_d + p->aux_off[i] : nullptr;
        fill_tile_args(a, d.H, d.W, p->rp[i], p->sp[i], p->gf[i], kForward);
        // a tile's time is set by its channel steps (every wave runs the whole
        // line program whatever its active lanes)
        const double fc = (double)a.nsteps;
        for (int k = 0; k < p->fwd_tiles[i]; ++k) fw.push_back({fc, {i, kItemFwd, k}});
        TileArgs& b = jobs[2 * i + 1];
        b = TileArgs{};
        if (bwd) {
            b.f = f[i];
            b.out = grad_f[i];
            b.fout = out[i];
            b.feta = eta[i];
            b.gout = nullptr;
            b.target = target[i];
            b.paux = p->aux_d + p->aux_off[i];
            fill_tile_args(b, d.H, d.W, p->rp[i], p->sp[i], p->gb[i], kBackward);
            const double bc = (double)b.nsteps;
            const int nb = p->gb[i].tiles_x * p->gb[i].tiles_y;
            for (int k = 0; k < nb; ++k) bw.push_back({bc, {i, kItemBwd, k}});
        }
    }
    auto by_cost = [](const Cost& x, const Cost& y) {
        return x.c > y.c || (x.c == y.c && (x.w.img < y.w.img ||
                                            (x.w.img == y.w.img && x.w.tile < y.w.tile)));
    };
    std::stable_sort(fw.begin(), fw.end(), by_cost);
    std::stable_sort(bw.begin(), bw.end(), by_cost);
    std::vector<BatchItem> items;
    items.reserve(fw.size() + n + bw.size());
    for (const Cost& c : fw) items.push_back(c.w);
    if (target)
        for (int i = 0; i < n; ++i) items.push_back({i, kItemLoss, 0});
    for (const Cost& c : bw) items.push_back(c.w);
    if (hipMemcpy(p->jobs_d, jobs.data(), jobs.size() * sizeof(TileArgs), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(p->items_d, items.data(), items.size() * sizeof(BatchItem),
                  hipMemcpyHostToDevice) != hipSuccess) {
        set_error("upload of the batch tables failed");
        return BF_EDEVICE;
    }
    p->n_items = (int)items.size();
    p->loss = loss;
    p->bound = true;
    return BF_OK;
}

bf_status bf_batch_launch(bf_batch_plan* p, void* stream) {
    if (!p || !p->bound) {
        set_error("plan missing or not bound");
        return BF_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    if (p->sb) return stream_batch_launch(p->sb, s);
    const int nc = kBatchCounters0 + p->n;
    hipLaunchKernelGGL(bf_batch_reset, dim3((nc + 255) / 256), dim3(256), 0, s, p->counters_d, nc);
    BatchDev d;
    d.jobs = p->jobs_d;
    d.items = p->items_d;
    d.n_items = p->n_items;
    d.fwd_tiles = p->fwd_tiles_d;
    d.part_base = p->part_base_d;
    d.loss_part = p->loss_part_d;
    d.loss = p->loss;
    d.counters = p->counters_d;
    d.spin_limit = 1u << 26;
    (void)hipFuncSetAttribute((const void*)bf_batch_kernel,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)p->lds);
    const int grid = std::min(p->grid, std::max(p->n_items, 1));
    hipLaunchKernelGGL(bf_batch_kernel, dim3(grid), dim3(kTileThreads), p->lds, s, d);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("batch launch failed: %s", hipGetErrorString(e));
        return BF_EDEVICE;
    }
    return BF_OK;
}

bf_status bf_batch_launch_stage(bf_batch_plan* p, int32_t stage, void* stream) {
    if (!p || !p->bound) {
        set_error("plan missing or not bound");
        return BF_EINVAL;
    }
    if (!p->sb) {
        if (stage != 0) {
            set_error("the persistent fused-tile batch has the single stage 0");
            return BF_EINVAL;
        }
        return bf_batch_launch(p, stream);
    }
    return stream_batch_stage(p->sb, stage, (hipStream_t)stream);
}

int32_t bf_batch_plan_path(const bf_batch_plan* p) {
    if (!p) return -1;
    return p->sb ? BF_PATH_STREAMED : BF_PATH_FUSED;
}

bf_status bf_batch_check(bf_batch_plan* p) {
    if (!p) {
        set_error("plan is NULL");
        return BF_EINVAL;
    }
    unsigned flags[2] = {0, 0};
    if (p->sb) {   // no bounded waits on this path
        if (hipDeviceSynchronize() != hipSuccess) {
            set_error("device error: %s", hipGetErrorString(hipGetLastError()));
            return BF_EDEVICE;
        }
        return BF_OK;
    }
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(flags, p->counters_d, sizeof(flags), hipMemcpyDeviceToHost) != hipSuccess) {
        set_error("device error: %s", hipGetErrorString(hipGetLastError()));
        return BF_EDEVICE;
    }
    if (flags[1]) {
        set_error("a batch wait hit its bound; results are invalid");
        return BF_EDEVICE;
    }
    return BF_OK;
}

void bf_batch_plan_destroy(bf_batch_plan* p) { free_plan(p); }

}  // extern "C"
