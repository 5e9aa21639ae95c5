// sc_batch.hip -- batched execution of many independent Shan-Chen lattices.
//
// Three launch forms advance the members of a batch by an epoch of K steps:
//   PER_LATTICE : one launch per lattice per step (the plain baseline);
//   FUSED       : one launch per step covering every member's tiles, the K
//                 launches captured once into a HIP graph and replayed;
//   PERSISTENT  : one launch per epoch; co-resident blocks claim tiles from a
//                 per-step counter and meet at a grid barrier between steps.
// All three run TileStep::run for every tile, so a lattice evolves bitwise
// the same alone or in any batch.  D2Q9 and D3Q19 members share a launch:
// D2Q9 tiles are NT x 1, D3Q19 tiles TX19 x TY19 with TX19 * TY19 = NT.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/lbm_sc.h"
#include "sc_internal.h"
#include "sc_runtime.h"

using namespace sc;

namespace {

// Clears the barrier words and claim counters of a persistent launch (a
// kernel, so that the clear may sit inside a captured graph).  The timeout
// flag is left alone: it stays set until the host has seen it.
__global__ void k_zero_u32(unsigned* p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        if (i != SYNC_TIMEOUT) p[i] = 0u;
}

struct BatchCfg {
    int nt, tx19, ty19;
};
static const BatchCfg kBatchCfgs[] = {{256, 64, 4}, {256, 32, 8}, {256, 16, 16}, {128, 32, 4},
                                      {512, 64, 8}, {512, 32, 16}};

bool cfg_supported(int nt, int tx19, int ty19) {
    for (const BatchCfg& c : kBatchCfgs)
        if (c.nt == nt && c.tx19 == tx19 && c.ty19 == ty19) return true;
    return false;
}

struct Member {
    lbm_sc* h;
    long long remaining;
};

// One kernel policy group's (precision, forcing, relaxation) device tables and cached graph.
struct Group {
    BatchDesc* d_desc = nullptr;
    size_t desc_cap = 0;
    WorkItem* d_work = nullptr;
    size_t work_cap = 0;
    unsigned* d_sync = nullptr;
    size_t sync_cap = 0;
    BatchDesc* h_desc = nullptr;  // pinned staging
    WorkItem* h_work = nullptr;
    hipEvent_t staged = nullptr;  // last upload from the staging buffers
    hipGraphExec_t gexec = nullptr;
    int g_mode = -1, g_nwork = -1, g_k = -1, g_grid = -1;
    unsigned g_spin = 0;
    // launch shape of the last epoch (captured or launched directly)
    int l_mode = -1, l_nwork = -1, l_k = -1, l_grid = -1;
    unsigned l_spin = 0;
    bool pers_used = false;       // a persistent launch may have set the timeout flag
};

}  // namespace

struct lbm_batch {
    size_t budget = 0, used = 0;
    std::vector<unsigned char> na_host;  // host staging of the allocation-free run
    hipEvent_t na_staged = nullptr;      // its last upload
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = 0;
    std::vector<Member> members;
    int nt = 256, tx19 = 64, ty19 = 4;
    int mb9 = 0, mb19 = 0;  // 0: each member's own march chunk
    unsigned spin_limit = kSpinLimit;  // grid-barrier polls before a persistent launch gives up
    Group grp[kPolicies];   // one per kernel policy (precision, forcing, relaxation)
    int err = 0;
};

namespace {

#define BCALL(b, expr)                    \
    do {                                  \
        hipError_t e_ = (expr);           \
        if (e_ != hipSuccess) {           \
            (b)->err = LBM_EDEVICE;       \
            return LBM_EDEVICE;           \
        }                                 \
    } while (0)

void free_group(Group& g) {
    if (g.gexec) (void)hipGraphExecDestroy(g.gexec);
    if (g.staged) {
        (void)hipEventSynchronize(g.staged);
        (void)hipEventDestroy(g.staged);
    }
    (void)hipFree(g.d_desc);
    (void)hipFree(g.d_work);
    (void)hipFree(g.d_sync);
    (void)hipHostFree(g.h_desc);
    (void)hipHostFree(g.h_work);
    g = Group();
}

int ensure(lbm_batch* b, Group& g, size_t ndesc, size_t nwork, int ksteps) {
    if (!g.staged) BCALL(b, hipEventCreateWithFlags(&g.staged, hipEventDisableTiming));
    // the staging buffers may still feed an upload in flight
    BCALL(b, hipEventSynchronize(g.staged));
    if (ndesc > g.desc_cap) {
        size_t cap = std::max<size_t>(ndesc, 2 * g.desc_cap);
        (void)hipFree(g.d_desc);
        (void)hipHostFree(g.h_desc);
        g.d_desc = nullptr;
        g.h_desc = nullptr;
        BCALL(b, hipMalloc(&g.d_desc, cap * sizeof(BatchDesc)));
        BCALL(b, hipHostMalloc(&g.h_desc, cap * sizeof(BatchDesc), 0));
        g.desc_cap = cap;
        if (g.gexec) (void)hipGraphExecDestroy(g.gexec);
        g.gexec = nullptr;
    }
    if (nwork > g.work_cap) {
        size_t cap = std::max<size_t>(nwork, 2 * g.work_cap);
        (void)hipFree(g.d_work);
        (void)hipHostFree(g.h_work);
        g.d_work = nullptr;
        g.h_work = nullptr;
        BCALL(b, hipMalloc(&g.d_work, cap * sizeof(WorkItem)));
        BCALL(b, hipHostMalloc(&g.h_work, cap * sizeof(WorkItem), 0));
        g.work_cap = cap;
        if (g.gexec) (void)hipGraphExecDestroy(g.gexec);
        g.gexec = nullptr;
    }
    const size_t nsync = SYNC_CTR + (size_t)ksteps;
    if (nsync > g.sync_cap) {
        size_t cap = std::max<size_t>(nsync, 2 * g.sync_cap);
        (void)hipFree(g.d_sync);
        g.d_sync = nullptr;
        BCALL(b, hipMalloc(&g.d_sync, cap * sizeof(unsigned)));
        // a fresh timeout flag (the per-launch clear keeps it); enqueued
        // before any capture begins
        BCALL(b, hipMemsetAsync(g.d_sync, 0, cap * sizeof(unsigned), b->stream));
        g.sync_cap = cap;
        if (g.gexec) (void)hipGraphExecDestroy(g.gexec);
        g.gexec = nullptr;
    }
    return LBM_OK;
}

// Waits for the batch's stream and reads the (sticky) timeout flag of every
// group that ran a persistent launch.  A give-up leaves the members half
// advanced: the batch and every member handle then report LBM_ETIMEOUT (the
// handles accept only destroy).  Returns LBM_OK, LBM_ETIMEOUT or LBM_EDEVICE.
int check_timeout(lbm_batch* b) {
    if (hipStreamSynchronize(b->stream) != hipSuccess) {
        b->err = LBM_EDEVICE;
        return LBM_EDEVICE;
    }
    bool hit = false;
    for (Group& g : b->grp) {
        if (!g.d_sync || !g.pers_used) continue;
        unsigned flag = 0;
        if (hipMemcpy(&flag, g.d_sync + SYNC_TIMEOUT, sizeof(unsigned), hipMemcpyDeviceToHost) !=
            hipSuccess) {
            b->err = LBM_EDEVICE;
            return LBM_EDEVICE;
        }
        hit = hit || flag != 0;
    }
    if (hit) {
        b->err = LBM_ETIMEOUT;
        for (Member& m : b->members) m.h->err = LBM_ETIMEOUT;
        return LBM_ETIMEOUT;
    }
    return LBM_OK;
}

int member_mb(const lbm_batch* b, const lbm_sc* h) {
    const int o = h->Q == 9 ? b->mb9 : b->mb19;
    return o > 0 ? o : h->mb;
}

// Descriptors and work list of one kernel policy group for an epoch: one
// descriptor per member (both buffer parities, its tile and march chunk in
// the batch's block shape) and its (member, tile, chunk) work items, the
// largest-cost items first.
void build_tables(lbm_batch* b, const std::vector<int>& idx, const std::vector<int>& ksteps,
                  std::vector<BatchDesc>& descs, std::vector<WorkItem>& works) {
    struct Item {
        WorkItem w;
        double cost;
    };
    std::vector<Item> items;
    descs.assign(idx.size(), BatchDesc{});
    for (size_t m = 0; m < idx.size(); ++m) {
        lbm_sc* h = b->members[idx[m]].h;
        const int save_tx = h->tx, save_ty = h->ty, save_mb = h->mb;
        h->tx = h->Q == 9 ? b->nt : b->tx19;
        h->ty = h->Q == 9 ? 1 : b->ty19;
        h->mb = member_mb(b, h);
        BatchDesc& d = descs[m];
        memset(&d, 0, sizeof(d));
        d.sp[0] = sc_step_params(h, 0);
        d.sp[1] = sc_step_params(h, 1);
        h->tx = save_tx;
        h->ty = save_ty;
        h->mb = save_mb;
        d.Q = h->Q;
        d.base_parity = h->cur;
        d.steps = ksteps[m];
        const StepParams& sp = d.sp[0];
        const double per = (double)h->Q * (h->Q == 9 ? b->nt : b->tx19 * b->ty19) *
                           (double)sp.mb;
        for (int c = 0; c < sp.nchunks; ++c)
            for (int ty = 0; ty < sp.nty; ++ty)
                for (int tx = 0; tx < sp.ntx; ++tx) {
                    const int planes = std::min(sp.mb, sp.NM - c * sp.mb);
                    items.push_back({{(int)m, tx, ty, c}, per * planes / sp.mb + 1e-9 * m});
                }
    }
    std::stable_sort(items.begin(), items.end(),
                     [](const Item& a, const Item& c) { return a.cost > c.cost; });
    works.resize(items.size());
    for (size_t i = 0; i < items.size(); ++i) works[i] = items[i].w;
}

// Enqueues one epoch of the members of one kernel policy group.
int run_group(lbm_batch* b, int pol, const std::vector<int>& idx, const std::vector<int>& ksteps,
              int K, int mode) {
    Group& g = b->grp[pol];
    std::vector<BatchDesc> descs;
    std::vector<WorkItem> items;
    build_tables(b, idx, ksteps, descs, items);
    const int nwork = (int)items.size();
    int rc = ensure(b, g, descs.size(), items.size(), K);
    if (rc) return rc;
    memcpy(g.h_desc, descs.data(), descs.size() * sizeof(BatchDesc));
    memcpy(g.h_work, items.data(), (size_t)nwork * sizeof(WorkItem));
    BCALL(b, hipMemcpyAsync(g.d_desc, g.h_desc, descs.size() * sizeof(BatchDesc),
                            hipMemcpyHostToDevice, b->stream));
    BCALL(b, hipMemcpyAsync(g.d_work, g.h_work, (size_t)nwork * sizeof(WorkItem),
                            hipMemcpyHostToDevice, b->stream));
    BCALL(b, hipEventRecord(g.staged, b->stream));

    BatchStepFn sf = nullptr;
    BatchPersFn pf = nullptr;
    const bool ok = batch_kernels(pol, b->nt, b->tx19, b->ty19, &sf, &pf);
    if (!ok) return LBM_EINVAL;

    int grid = nwork;
    if (mode == LBM_BATCH_PERSISTENT) {
        int per_cu = 0, dev = 0;
        BCALL(b, hipGetDevice(&dev));
        hipDeviceProp_t prop;
        BCALL(b, hipGetDeviceProperties(&prop, dev));
        BCALL(b, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)pf, b->nt, 0));
        if (per_cu < 1) return LBM_EDEVICE;
        grid = std::min(std::min(nwork, per_cu * prop.multiProcessorCount), kMaxPersistentBlocks);
    }
    // the epoch's launches (into a capture, or straight onto the stream)
    auto enqueue = [&]() -> hipError_t {
        hipError_t le = hipSuccess;
        if (mode == LBM_BATCH_FUSED) {
            for (int k = 0; k < K && le == hipSuccess; ++k) {
                hipLaunchKernelGGL(sf, dim3(nwork), dim3(b->nt), 0, b->stream, g.d_desc, g.d_work,
                                   nwork, k);
                le = hipGetLastError();
            }
        } else {
            hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(256), 0, b->stream, g.d_sync, SYNC_CTR + K);
            le = hipGetLastError();
            if (le == hipSuccess) {
                hipLaunchKernelGGL(pf, dim3(grid), dim3(b->nt), 0, b->stream, g.d_desc, g.d_work,
                                   nwork, K, g.d_sync, b->spin_limit);
                le = hipGetLastError();
            }
        }
        return le;
    };
    if (mode == LBM_BATCH_PERSISTENT) g.pers_used = true;
    // replay the cached graph when the launch shape is unchanged (the tables
    // are rewritten in place, so the captured arguments stay valid)
    const bool cached = g.gexec && g.g_mode == mode && g.g_nwork == nwork && g.g_k == K &&
                        g.g_grid == grid && g.g_spin == b->spin_limit;
    const bool repeat = g.l_mode == mode && g.l_nwork == nwork && g.l_k == K && g.l_grid == grid &&
                        g.l_spin == b->spin_limit;
    g.l_mode = mode;
    g.l_nwork = nwork;
    g.l_k = K;
    g.l_grid = grid;
    g.l_spin = b->spin_limit;
    if (!cached && !repeat) {
        // a launch shape not seen in the last epoch (the members changed):
        // launch directly, since capturing and instantiating a graph costs
        // about a millisecond of host time while the device waits; the graph
        // is captured once the shape repeats
        const hipError_t le = enqueue();
        if (le != hipSuccess) {
            b->err = LBM_EDEVICE;
            return LBM_EDEVICE;
        }
        return LBM_OK;
    }
    if (!cached) {
        if (g.gexec) (void)hipGraphExecDestroy(g.gexec);
        g.gexec = nullptr;
        hipGraph_t graph = nullptr;
        BCALL(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        const hipError_t le = enqueue();
        hipError_t ee = hipStreamEndCapture(b->stream, &graph);
        if (le != hipSuccess || ee != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            b->err = LBM_EDEVICE;
            return LBM_EDEVICE;
        }
        hipError_t ie = hipGraphInstantiate(&g.gexec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ie != hipSuccess) {
            g.gexec = nullptr;
            b->err = LBM_EDEVICE;
            return LBM_EDEVICE;
        }
        g.g_mode = mode;
        g.g_nwork = nwork;
        g.g_k = K;
        g.g_grid = grid;
        g.g_spin = b->spin_limit;
    }
    BCALL(b, hipGraphLaunch(g.gexec, b->stream));
    return LBM_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free run (lbm_batch_run_noalloc).  The fused form's descriptor
// table and work list go to a fixed device array instead of buffers the batch
// allocates.  Every GPU the library runs on holds its own copy of the array
// until the process ends; host code reaches it only through the address
// hipGetSymbolAddress returns for the device (the array's name is a host-side
// stand-in, not a device address).
// ---------------------------------------------------------------------------
constexpr int kNoAllocMaxMembers = 1024;   // members of one kernel policy group
constexpr int kNoAllocMaxWork = 1 << 18;   // work items of one kernel policy group
constexpr size_t kNoAllocDescBytes =
    ((size_t)kNoAllocMaxMembers * sizeof(BatchDesc) + 255) / 256 * 256;
constexpr size_t kNoAllocScratchBytes =
    kNoAllocDescBytes + (size_t)kNoAllocMaxWork * sizeof(WorkItem);
static_assert(kNoAllocScratchBytes <= (5u << 20), "scratch stays a few MB");

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's scratch array, looked up once per device with
// that device current (the caller has set it).
int scratch_address(int dev, unsigned char** out) {
    if (dev < 0 || dev >= kMaxDevices) return LBM_EINVAL;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
            return LBM_EDEVICE;
        g_scratch_ptr[dev] = ptr;
    }
    *out = static_cast<unsigned char*>(g_scratch_ptr[dev]);
    return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_batch_create(lbm_batch** out, size_t hbm_budget, void* stream) {
    if (!out) return LBM_EINVAL;
    *out = nullptr;
    lbm_batch* b = new (std::nothrow) lbm_batch();
    if (!b) return LBM_ENOMEM;
    b->budget = hbm_budget;
    if (hipGetDevice(&b->device) != hipSuccess) {
        delete b;
        return LBM_EDEVICE;
    }
    if (stream) {
        b->stream = static_cast<hipStream_t>(stream);
    } else {
        if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
            delete b;
            return LBM_EDEVICE;
        }
        b->own_stream = true;
    }
    if (hipEventCreateWithFlags(&b->na_staged, hipEventDisableTiming) != hipSuccess) {
        if (b->own_stream) (void)hipStreamDestroy(b->stream);
        delete b;
        return LBM_EDEVICE;
    }
    *out = b;
    return LBM_OK;
}

int lbm_batch_add(lbm_batch* b, lbm_sc* h, long long steps) {
    if (!b || !h || steps < 0) return LBM_EINVAL;
    if (b->err) return b->err;
    if (h->err) return h->err;
    if (!h->inited) return LBM_ESTATE;
    if (h->batch) return LBM_EINVAL;
    if (b->budget && b->used + h->mem_bytes > b->budget) return LBM_EBUDGET;
    (void)hipSetDevice(b->device);
    // the handle's own queued work (initialisation) precedes batch work
    if (hipStreamSynchronize(h->stream) != hipSuccess) return LBM_EDEVICE;
    h->batch = b;
    b->used += h->mem_bytes;
    b->members.push_back({h, steps});
    return LBM_OK;
}

int lbm_batch_remove(lbm_batch* b, lbm_sc* h) {
    if (!b || !h) return LBM_EINVAL;
    for (size_t i = 0; i < b->members.size(); ++i)
        if (b->members[i].h == h) {
            (void)hipSetDevice(b->device);
            const int rc = b->err ? b->err : check_timeout(b);
            h->batch = nullptr;
            b->used -= h->mem_bytes;
            b->members.erase(b->members.begin() + i);
            return rc;
        }
    return LBM_EINVAL;
}

int lbm_batch_run(lbm_batch* b, int epoch_steps, int mode) {
    if (!b || epoch_steps < 0) return LBM_EINVAL;
    if (b->err) return b->err;
    if (mode != LBM_BATCH_PER_LATTICE && mode != LBM_BATCH_FUSED && mode != LBM_BATCH_PERSISTENT)
        return LBM_EINVAL;
    if (epoch_steps == 0) return LBM_OK;
    (void)hipSetDevice(b->device);
    std::vector<int> idx[kPolicies], ks[kPolicies];
    for (size_t i = 0; i < b->members.size(); ++i) {
        Member& m = b->members[i];
        if (m.remaining <= 0 || m.h->err) continue;
        const int k = (int)std::min<long long>(m.remaining, epoch_steps);
        const int pol = sc_policy(m.h->p);
        idx[pol].push_back((int)i);
        ks[pol].push_back(k);
    }
    if (mode == LBM_BATCH_PER_LATTICE) {
        for (int pol = 0; pol < kPolicies; ++pol)
            for (size_t m = 0; m < idx[pol].size(); ++m) {
                lbm_sc* h = b->members[idx[pol][m]].h;
                lbm_batch* keep = h->batch;
                const int rc = sc_enqueue_steps(h, ks[pol][m], b->stream, false);
                h->batch = keep;
                if (rc) {
                    b->err = rc;
                    return rc;
                }
                // sc_enqueue_steps already advanced parity and step count
                b->members[idx[pol][m]].remaining -= ks[pol][m];
            }
        return LBM_OK;
    }
    for (int pol = 0; pol < kPolicies; ++pol) {
        if (idx[pol].empty()) continue;
        const int K = *std::max_element(ks[pol].begin(), ks[pol].end());
        const int rc = run_group(b, pol, idx[pol], ks[pol], K, mode);
        if (rc) return rc;
        for (size_t m = 0; m < idx[pol].size(); ++m) {
            Member& mm = b->members[idx[pol][m]];
            mm.h->cur ^= (ks[pol][m] & 1);
            mm.h->steps += ks[pol][m];
            mm.remaining -= ks[pol][m];
        }
    }
    return LBM_OK;
}

int lbm_batch_run_noalloc(lbm_batch* b, int epoch_steps, int mode) {
    if (!b || epoch_steps < 0) return LBM_EINVAL;
    if (b->err) return b->err;
    if (mode == LBM_BATCH_PER_LATTICE) return lbm_batch_run(b, epoch_steps, mode);  // launches only
    if (mode != LBM_BATCH_FUSED) return LBM_EINVAL;
    if (epoch_steps == 0) return LBM_OK;
    (void)hipSetDevice(b->device);
    unsigned char* scr = nullptr;
    int rc = scratch_address(b->device, &scr);
    if (rc) return rc;
    std::vector<int> idx[kPolicies], ks[kPolicies];
    for (size_t i = 0; i < b->members.size(); ++i) {
        Member& m = b->members[i];
        if (m.remaining <= 0 || m.h->err) continue;
        const int k = (int)std::min<long long>(m.remaining, epoch_steps);
        const int pol = sc_policy(m.h->p);
        idx[pol].push_back((int)i);
        ks[pol].push_back(k);
    }
    // every group's tables first: a batch beyond the scratch limits is
    // refused before anything is enqueued
    std::vector<BatchDesc> descs[kPolicies];
    std::vector<WorkItem> works[kPolicies];
    for (int pol = 0; pol < kPolicies; ++pol) {
        if (idx[pol].empty()) continue;
        build_tables(b, idx[pol], ks[pol], descs[pol], works[pol]);
        if (descs[pol].size() > (size_t)kNoAllocMaxMembers ||
            works[pol].size() > (size_t)kNoAllocMaxWork)
            return LBM_ETOOBIG;
    }
    for (int pol = 0; pol < kPolicies; ++pol) {
        if (idx[pol].empty()) continue;
        BatchStepFn sf = nullptr;
        BatchPersFn pf = nullptr;
        if (!batch_kernels(pol, b->nt, b->tx19, b->ty19, &sf, &pf)) return LBM_EINVAL;
        const size_t dbytes = descs[pol].size() * sizeof(BatchDesc);
        const size_t wbytes = works[pol].size() * sizeof(WorkItem);
        // the staging buffer may still feed the previous upload
        BCALL(b, hipEventSynchronize(b->na_staged));
        if (b->na_host.size() < kNoAllocScratchBytes) b->na_host.resize(kNoAllocScratchBytes);
        memcpy(b->na_host.data(), descs[pol].data(), dbytes);
        memcpy(b->na_host.data() + kNoAllocDescBytes, works[pol].data(), wbytes);
        // one group's tables at a time: the upload of the next group is
        // stream-ordered after this group's kernels
        BCALL(b, hipMemcpyAsync(scr, b->na_host.data(), dbytes, hipMemcpyHostToDevice, b->stream));
        BCALL(b, hipMemcpyAsync(scr + kNoAllocDescBytes, b->na_host.data() + kNoAllocDescBytes,
                                wbytes, hipMemcpyHostToDevice, b->stream));
        BCALL(b, hipEventRecord(b->na_staged, b->stream));
        const BatchDesc* d_desc = reinterpret_cast<const BatchDesc*>(scr);
        const WorkItem* d_work = reinterpret_cast<const WorkItem*>(scr + kNoAllocDescBytes);
        const int nwork = (int)works[pol].size();
        const int K = *std::max_element(ks[pol].begin(), ks[pol].end());
        for (int k = 0; k < K; ++k) {
            hipLaunchKernelGGL(sf, dim3(nwork), dim3(b->nt), 0, b->stream, d_desc, d_work, nwork, k);
            BCALL(b, hipGetLastError());
        }
        for (size_t m = 0; m < idx[pol].size(); ++m) {
            Member& mm = b->members[idx[pol][m]];
            mm.h->cur ^= (ks[pol][m] & 1);
            mm.h->steps += ks[pol][m];
            mm.remaining -= ks[pol][m];
        }
    }
    return LBM_OK;
}

int lbm_batch_poll(lbm_batch* b, lbm_sc** done, int max_done, int* n_done) {
    if (!b || !n_done || max_done < 0 || (max_done > 0 && !done)) return LBM_EINVAL;
    *n_done = 0;
    if (b->err) return b->err;
    (void)hipSetDevice(b->device);
    const int rc = check_timeout(b);
    if (rc) return rc;
    for (const Member& m : b->members)
        if (m.remaining <= 0 && *n_done < max_done) done[(*n_done)++] = m.h;
    return LBM_OK;
}

int lbm_batch_stats(const lbm_batch* b, int* members, size_t* bytes_used,
                    double* pending_site_updates) {
    if (!b) return LBM_EINVAL;
    if (members) *members = (int)b->members.size();
    if (bytes_used) *bytes_used = b->used;
    if (pending_site_updates) {
        double s = 0.0;
        for (const Member& m : b->members) s += (double)m.h->N * (double)std::max(0LL, m.remaining);
        *pending_site_updates = s;
    }
    return LBM_OK;
}

int lbm_batch_set_tiles(lbm_batch* b, int tx9, int tx19, int ty19, int mb9, int mb19) {
    if (!b) return LBM_EINVAL;
    const int nt = tx9 > 0 ? tx9 : b->nt;
    const int x19 = tx19 > 0 ? tx19 : b->tx19;
    const int y19 = ty19 > 0 ? ty19 : b->ty19;
    if (!cfg_supported(nt, x19, y19)) return LBM_EINVAL;
    if (mb9 < 0 || mb19 < 0) return LBM_EINVAL;
    b->nt = nt;
    b->tx19 = x19;
    b->ty19 = y19;
    b->mb9 = mb9;
    b->mb19 = mb19;
    for (Group& g : b->grp) {
        if (g.gexec) (void)hipGraphExecDestroy(g.gexec);
        g.gexec = nullptr;
    }
    return LBM_OK;
}

int lbm_batch_set_spin_limit(lbm_batch* b, unsigned spins) {
    if (!b) return LBM_EINVAL;
    b->spin_limit = spins ? spins : kSpinLimit;
    return LBM_OK;
}

int lbm_batch_destroy(lbm_batch* b) {
    if (!b) return LBM_OK;
    (void)hipSetDevice(b->device);
    const int rc = b->err ? b->err : check_timeout(b);
    for (Member& m : b->members) m.h->batch = nullptr;
    for (Group& g : b->grp) free_group(g);
    if (b->na_staged) (void)hipEventDestroy(b->na_staged);
    if (b->own_stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return rc == LBM_ETIMEOUT ? rc : LBM_OK;
}

}  // extern "C"
