// rti_batch.cpp -- batches of domains stepped together: per step one
// active-tile launch and one fused launch over a global table of every
// member's tiles (the members' own flags, buffers and parities), replayed
// from HIP graphs like a single domain.  Membership may change between steps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "rti_runtime.h"

using namespace rti_rt;

struct rti_batch {
    std::vector<rti_domain *> members;
    hipStream_t stream = nullptr;        // borrowed; every member's stream
    hipStream_t capture = nullptr;       // private, for graph capture
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    uint32_t flags = 0;
    int device = 0;
    int cu_count = 256;
    int bulk32 = -1;                     // precision of the members (-1: no member yet)
    // device tables (one allocation) and their host copies
    void *mem = nullptr;
    size_t mem_bytes = 0;
    BatchDev dev{};
    std::vector<int32_t> base;           // n + 1
    std::vector<uint16_t> tdom;          // global tile -> member
    std::vector<uint64_t> gen;           // members' generation when the tables were built
    std::vector<int> par;                // members' parity when the tables were built
    bool dirty = true;
    int flip = 0;                        // parity of the next step relative to par
    int64_t steps = 0;                   // batch steps since the tables were built
    unsigned long long cells_done = 0;   // computed cells carried over when the tables are rebuilt
    size_t nslot = 0;                    // computed-cell slots of the current tables
    int64_t cell_updates_all = 0;        // every member's cells times the steps it took in the batch
    bool overflowed = false;             // the global list's overflow flag was seen set (sticky)
};

namespace {

constexpr uint32_t kBatchFlags = RTI_FLAG_NO_GRAPH | RTI_FLAG_NO_ACTIVE | RTI_FLAG_PERSISTENT;
constexpr size_t kMaxMembers = 65535;    // member index is stored in 16 bits

void drop_graphs(rti_batch *B)
{
    for (int p = 0; p < 2; ++p) {
        if (B->exec[p]) (void)hipGraphExecDestroy(B->exec[p]);
        if (B->graph[p]) (void)hipGraphDestroy(B->graph[p]);
        B->exec[p] = nullptr;
        B->graph[p] = nullptr;
    }
}

// The tables are stale when membership changed, a member's tile tables or
// parameters changed (generation), or a member's parity no longer follows the
// batch (it cannot, as members are stepped only here, but cheap to check).
bool stale(const rti_batch *B)
{
    if (B->dirty) return true;
    for (size_t m = 0; m < B->members.size(); ++m) {
        const rti_domain *D = B->members[m];
        if (D->gen != B->gen[m] || D->cur != (B->par[m] ^ B->flip)) return true;
    }
    return false;
}

// Sum of the computed-cell slots of the current tables (synchronises).
int sum_cells(rti_batch *B, unsigned long long *out)
{
    std::vector<unsigned long long> part(B->nslot);
    if (B->nslot) {
        HIP_TRY(hipMemcpyAsync(part.data(), B->dev.cells_done, sizeof(unsigned long long) * B->nslot,
                               hipMemcpyDeviceToHost, B->stream));
        HIP_TRY(hipStreamSynchronize(B->stream));
    }
    unsigned long long t = 0;
    for (auto v : part) t += v;
    *out = t;
    return RTI_OK;
}

// The global list's overflow flag into the sticky host flag (synchronises);
// the tables' flag is cleared when they are rebuilt.
int read_overflow(rti_batch *B)
{
    if (!B->dev.status) return RTI_OK;
    int st = 0;
    HIP_TRY(hipMemcpyAsync(&st, B->dev.status + 1, sizeof st, hipMemcpyDeviceToHost, B->stream));
    HIP_TRY(hipStreamSynchronize(B->stream));
    if (st) B->overflowed = true;
    return RTI_OK;
}

int build_tables(rti_batch *B)
{
    HIP_TRY(hipStreamSynchronize(B->stream));
    if (int rc = read_overflow(B)) return rc;
    if (B->mem) {   // carry the computed-cells total over to the new tables
        unsigned long long t = 0;
        int rc = sum_cells(B, &t);
        if (rc) return rc;
        B->cells_done = t;
    }
    drop_graphs(B);
    const int n = (int)B->members.size();
    B->base.assign(n + 1, 0);
    for (int m = 0; m < n; ++m) B->base[m + 1] = B->base[m] + B->members[m]->dev.ntiles;
    const int ntiles = B->base[n];
    B->tdom.assign(ntiles, 0);
    for (int m = 0; m < n; ++m)
        std::fill(B->tdom.begin() + B->base[m], B->tdom.begin() + B->base[m + 1], (uint16_t)m);
    // global ring cells: member m's are rbase[m] .. rbase[m+1]-1
    std::vector<int32_t> rbase(n + 1, 0);
    for (int m = 0; m < n; ++m) rbase[m + 1] = rbase[m] + B->members[m]->dev.nring;
    const int nring = rbase[n];
    std::vector<uint16_t> rdom(std::max(nring, 1), 0);
    for (int m = 0; m < n; ++m) std::fill(rdom.begin() + rbase[m], rdom.begin() + rbase[m + 1], (uint16_t)m);
    std::vector<DomainDev> doms(n);
    std::vector<uint8_t> par(n);
    B->gen.assign(n, 0);
    B->par.assign(n, 0);
    for (int m = 0; m < n; ++m) {
        doms[m] = B->members[m]->dev;
        par[m] = (uint8_t)B->members[m]->cur;
        B->gen[m] = B->members[m]->gen;
        B->par[m] = B->members[m]->cur;
    }
    // layout: doms | base | tdom | par | list | lmeta | count | cells | rbase | rdom
    const size_t o_doms = 0;
    const size_t o_base = o_doms + align_up(sizeof(DomainDev) * std::max(n, 1), kAlign);
    const size_t o_tdom = o_base + align_up(sizeof(int32_t) * (n + 1), kAlign);
    const size_t o_par = o_tdom + align_up(sizeof(uint16_t) * std::max(ntiles, 1), kAlign);
    const size_t o_list = o_par + align_up((size_t)std::max(n, 1), kAlign);
    const size_t o_lmeta = o_list + align_up(sizeof(int32_t) * std::max(ntiles, 1), kAlign);
    const size_t o_count = o_lmeta + align_up(sizeof(int32_t) * std::max(ntiles, 1), kAlign);
    const size_t nslot = (size_t)(std::max(ntiles, 1) + 255) / 256;      // one per active-list workgroup
    const size_t o_cells = o_count + kAlign;
    const size_t o_rbase = o_cells + align_up(sizeof(unsigned long long) * nslot, kAlign);
    const size_t o_rdom = o_rbase + align_up(sizeof(int32_t) * (n + 1), kAlign);
    const size_t bytes = o_rdom + align_up(sizeof(uint16_t) * std::max(nring, 1), kAlign);
    if (bytes > B->mem_bytes) {
        if (B->mem) (void)hipFree(B->mem);
        B->mem = nullptr;
        B->mem_bytes = 0;
        hipError_t e = hipMalloc(&B->mem, bytes);
        if (e != hipSuccess) return fail(RTI_ENOMEM, "batch tables of %zu bytes: %s", bytes, hipGetErrorString(e));
        B->mem_bytes = bytes;
    }
    char *p = static_cast<char *>(B->mem);
    HIP_TRY(hipMemcpyAsync(p + o_doms, doms.data(), sizeof(DomainDev) * n, hipMemcpyHostToDevice, B->stream));
    HIP_TRY(hipMemcpyAsync(p + o_base, B->base.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, B->stream));
    if (ntiles)
        HIP_TRY(hipMemcpyAsync(p + o_tdom, B->tdom.data(), sizeof(uint16_t) * ntiles, hipMemcpyHostToDevice, B->stream));
    HIP_TRY(hipMemcpyAsync(p + o_par, par.data(), (size_t)n, hipMemcpyHostToDevice, B->stream));
    HIP_TRY(hipMemsetAsync(p + o_count, 0, 16, B->stream));                  // list counters, status
    HIP_TRY(hipMemsetAsync(p + o_cells, 0, sizeof(unsigned long long) * nslot, B->stream));
    HIP_TRY(hipMemcpyAsync(p + o_cells, &B->cells_done, sizeof B->cells_done, hipMemcpyHostToDevice, B->stream));
    HIP_TRY(hipMemcpyAsync(p + o_rbase, rbase.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, B->stream));
    if (nring)
        HIP_TRY(hipMemcpyAsync(p + o_rdom, rdom.data(), sizeof(uint16_t) * nring, hipMemcpyHostToDevice, B->stream));
    HIP_TRY(hipStreamSynchronize(B->stream));   // host vectors die on return
    BatchDev &bd = B->dev;
    bd.doms = reinterpret_cast<const DomainDev *>(p + o_doms);
    bd.base = reinterpret_cast<const int32_t *>(p + o_base);
    bd.tdom = reinterpret_cast<const uint16_t *>(p + o_tdom);
    bd.par = reinterpret_cast<const uint8_t *>(p + o_par);
    bd.list = reinterpret_cast<int32_t *>(p + o_list);
    bd.lmeta = reinterpret_cast<int32_t *>(p + o_lmeta);
    bd.count = reinterpret_cast<int32_t *>(p + o_count);
    bd.status = bd.count + 2;
    bd.cells_done = reinterpret_cast<unsigned long long *>(p + o_cells);
    bd.rbase = reinterpret_cast<const int32_t *>(p + o_rbase);
    bd.rdom = reinterpret_cast<const uint16_t *>(p + o_rdom);
    bd.nring = nring;
    B->nslot = nslot;
    bd.n = n;
    bd.ntiles = ntiles;
    B->flip = 0;
    B->steps = 0;
    B->dirty = false;
    return RTI_OK;
}

// The boundary fluxes of the members' masked children (after the fused launch).
hipError_t launch_member_injects(rti_batch *B, int flip, hipStream_t s)
{
    for (size_t m = 0; m < B->members.size(); ++m) {
        const rti_domain *D = B->members[m];
        if (D->dev.ninject == 0) continue;
        const hipError_t e = launch_inject(D->dev, B->par[m] ^ flip, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

int launch_batch_step(rti_batch *B, int flip, hipStream_t s)
{
    HIP_TRY(launch_active_batch(B->dev, flip, (B->flags & RTI_FLAG_NO_ACTIVE) ? 1 : 0, B->bulk32, s));
    HIP_TRY(launch_fused_batch(B->dev, flip, B->bulk32,
                               fused_grid(B->dev.ntiles, (B->flags & RTI_FLAG_PERSISTENT) != 0, B->cu_count), s));
    HIP_TRY(launch_member_injects(B, flip, s));
    return RTI_OK;
}

int build_graph(rti_batch *B, int flip)
{
    if (!B->capture) HIP_TRY(hipStreamCreateWithFlags(&B->capture, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(B->capture, hipStreamCaptureModeThreadLocal));
    int rc = RTI_OK;
    for (int k = 0; k < kGraphSteps && rc == RTI_OK; ++k) rc = launch_batch_step(B, (flip + k) & 1, B->capture);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(B->capture, &g);
    if (rc != RTI_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(RTI_EHIP, "hipStreamEndCapture failed: %s", hipGetErrorString(e));
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(RTI_EHIP, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
    }
    B->graph[flip] = g;
    B->exec[flip] = x;
    return RTI_OK;
}

// Members advance by n steps.
void advance(rti_batch *B, int64_t n)
{
    for (rti_domain *D : B->members) {
        D->steps += n;
        D->cur ^= (int)(n & 1);
        B->cell_updates_all += D->plan.cells * n;
    }
    B->steps += n;
}

int check_member(const rti_batch *B, const rti_domain *D)
{
    if (!D) return fail(RTI_EINVAL, "member is NULL");
    if (D->batch) return fail(RTI_ESTATE, "the domain already belongs to a batch");
    if (D->device != B->device) return fail(RTI_EINVAL, "the domain lives on device %d, the batch on %d", D->device, B->device);
    if (D->flags & RTI_FLAG_PHASED) return fail(RTI_EINVAL, "members use the fused kernel (no RTI_FLAG_PHASED)");
    if (D->diverged) return fail(RTI_EDIVERGED, "the domain diverged earlier");
    if (B->bulk32 >= 0 && D->dev.bulk32 != B->bulk32) return fail(RTI_EINVAL, "members share one precision");
    if (B->members.size() >= kMaxMembers) return fail(RTI_EINVAL, "a batch holds at most %zu members", kMaxMembers);
    return RTI_OK;
}

}  // namespace

void rti_rt::batch_forget_member(rti_batch *B, rti_domain *D)
{
    (void)hipStreamSynchronize(B->stream);
    auto it = std::find(B->members.begin(), B->members.end(), D);
    if (it != B->members.end()) B->members.erase(it);
    D->batch = nullptr;
    (void)reset_counts(D);          // its parity moved under the batch
    (void)hipStreamSynchronize(B->stream);
    D->stream = D->home_stream;
    B->dirty = true;
    drop_graphs(B);
}

extern "C" {

int rti_batch_create(rti_domain *const *members, int32_t n, void *hip_stream, uint32_t flags, rti_batch **out)
{
    try {
        if (!out) return fail(RTI_EINVAL, "out is NULL");
        *out = nullptr;
        if (n < 0 || (n > 0 && !members)) return fail(RTI_EINVAL, "members: %d entries", n);
        if (flags & ~kBatchFlags) return fail(RTI_EINVAL, "unknown batch flags 0x%x", flags);
        rti_batch *B = new rti_batch;
        B->stream = static_cast<hipStream_t>(hip_stream);
        B->flags = flags;
        hipError_t e = hipGetDevice(&B->device);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&B->cu_count, hipDeviceAttributeMultiprocessorCount, B->device);
        if (e != hipSuccess) {
            delete B;
            return fail(RTI_EHIP, "querying the device failed: %s", hipGetErrorString(e));
        }
        for (int32_t m = 0; m < n; ++m) {
            int rc = rti_batch_add(B, members[m]);
            if (rc) {
                rti_batch_destroy(B);
                return rc;
            }
        }
        *out = B;
        return RTI_OK;
    } catch (const std::bad_alloc &) {
        return fail(RTI_ENOMEM, "host allocation failed");
    } catch (...) {
        return fail(RTI_EINVAL, "unexpected exception");
    }
}

int rti_batch_add(rti_batch *B, rti_domain *D)
{
    try {
        if (!B) return fail(RTI_EINVAL, "batch is NULL");
        int rc = check_member(B, D);
        if (rc) return rc;
        if (D->stream != B->stream) {
            // adopt: the work queued on the member's own stream finishes first,
            // then everything of the member runs on the batch's stream
            HIP_TRY(hipStreamSynchronize(D->stream));
            D->stream = B->stream;
        }
        B->members.push_back(D);
        D->batch = B;
        B->bulk32 = D->dev.bulk32;
        B->dirty = true;
        return RTI_OK;
    } catch (const std::bad_alloc &) {
        return fail(RTI_ENOMEM, "host allocation failed");
    }
}

int rti_batch_remove(rti_batch *B, rti_domain *D)
{
    if (!B || !D) return fail(RTI_EINVAL, "NULL argument");
    if (D->batch != B) return fail(RTI_EINVAL, "the domain is not a member of this batch");
    batch_forget_member(B, D);
    if (B->members.empty()) B->bulk32 = -1;
    return RTI_OK;
}

int rti_batch_size(const rti_batch *B, int32_t *n)
{
    if (!B || !n) return fail(RTI_EINVAL, "NULL argument");
    *n = (int32_t)B->members.size();
    return RTI_OK;
}

int rti_batch_step(rti_batch *B, int64_t nsteps)
{
    try {
        if (!B) return fail(RTI_EINVAL, "batch is NULL");
        if (nsteps < 0) return fail(RTI_EINVAL, "nsteps %lld < 0", (long long)nsteps);
        if (B->members.empty() || nsteps == 0) return RTI_OK;
        for (const rti_domain *D : B->members)
            if (D->diverged) return fail(RTI_EDIVERGED, "a member diverged earlier");
        if (stale(B)) {
            int rc = build_tables(B);
            if (rc) return rc;
        }
        const bool graphs = !(B->flags & RTI_FLAG_NO_GRAPH);
        while (nsteps > 0) {
            if (graphs && nsteps >= kGraphSteps) {
                if (!B->exec[B->flip]) {
                    int rc = build_graph(B, B->flip);
                    if (rc) return rc;
                }
                HIP_TRY(hipGraphLaunch(B->exec[B->flip], B->stream));
                advance(B, kGraphSteps);
                nsteps -= kGraphSteps;
            } else {
                int rc = launch_batch_step(B, B->flip, B->stream);
                if (rc) return rc;
                B->flip ^= 1;
                advance(B, 1);
                nsteps -= 1;
            }
        }
        return RTI_OK;
    } catch (const std::bad_alloc &) {
        return fail(RTI_ENOMEM, "host allocation failed");
    } catch (...) {
        return fail(RTI_EINVAL, "unexpected exception");
    }
}

int rti_batch_sync(rti_batch *B)
{
    if (!B) return fail(RTI_EINVAL, "batch is NULL");
    HIP_TRY(hipStreamSynchronize(B->stream));
    if (int rc = read_overflow(B)) return rc;
    if (B->overflowed) return fail(RTI_EINTERNAL, "the batch's active-tile list overflowed on the device");
    for (rti_domain *D : B->members)
        if (int rc = check_status(D)) return rc;
    return RTI_OK;
}

int rti_batch_profile(rti_batch *B, int64_t nsteps, double *fused_ms, double *active_ms, double *active_cells)
{
    try {
        if (!B || nsteps < 1) return fail(RTI_EINVAL, "bad argument");
        if (B->members.empty()) return fail(RTI_ESTATE, "the batch is empty");
        if (stale(B)) {
            int rc = build_tables(B);
            if (rc) return rc;
        }
        hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
        for (auto &x : ev) HIP_TRY(hipEventCreate(&x));
        double sf = 0.0, sa = 0.0, sc = 0.0;
        int rc = RTI_OK;
        std::vector<int32_t> list;
        const int grid = fused_grid(B->dev.ntiles, (B->flags & RTI_FLAG_PERSISTENT) != 0, B->cu_count);
        for (int64_t k = 0; k < nsteps && !rc; ++k) {
            const int flip = B->flip;
            hipError_t e = hipEventRecord(ev[0], B->stream);
            if (e == hipSuccess)
                e = launch_active_batch(B->dev, flip, (B->flags & RTI_FLAG_NO_ACTIVE) ? 1 : 0, B->bulk32, B->stream);
            if (e == hipSuccess) e = hipEventRecord(ev[1], B->stream);
            if (e == hipSuccess) e = launch_fused_batch(B->dev, flip, B->bulk32, grid, B->stream);
            if (e == hipSuccess) e = launch_member_injects(B, flip, B->stream);
            if (e == hipSuccess) e = hipEventRecord(ev[2], B->stream);
            if (e == hipSuccess) e = hipEventSynchronize(ev[2]);
            float ta = 0.0f, tf = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ta, ev[0], ev[1]);
            if (e == hipSuccess) e = hipEventElapsedTime(&tf, ev[1], ev[2]);
            int cnt = 0;
            if (e == hipSuccess) e = hipMemcpy(&cnt, B->dev.count + flip, sizeof(int), hipMemcpyDeviceToHost);
            cnt = std::min(cnt, B->dev.ntiles);        // the list holds at most one entry per tile
            if (e == hipSuccess && cnt > 0) {
                list.resize(cnt);
                e = hipMemcpy(list.data(), B->dev.list, sizeof(int32_t) * cnt, hipMemcpyDeviceToHost);
            }
            if (e != hipSuccess) {
                rc = fail(RTI_EHIP, "batch profiling: %s", hipGetErrorString(e));
                break;
            }
            double cells = 0.0;
            for (int q = 0; q < cnt; ++q) {
                const int G = list[q];
                const int m = B->tdom[G];
                cells += B->members[m]->plan.tcells[G - B->base[m]];
            }
            sa += ta;
            sf += tf;
            sc += cells;
            B->flip ^= 1;
            advance(B, 1);
        }
        for (auto &x : ev) (void)hipEventDestroy(x);
        if (rc) return rc;
        if (fused_ms) *fused_ms = sf / nsteps;
        if (active_ms) *active_ms = sa / nsteps;
        if (active_cells) *active_cells = sc / nsteps;
        return RTI_OK;
    } catch (const std::bad_alloc &) {
        return fail(RTI_ENOMEM, "host allocation failed");
    } catch (...) {
        return fail(RTI_EINVAL, "unexpected exception");
    }
}

int rti_batch_cell_updates(rti_batch *B, int64_t *all, int64_t *computed)
{
    if (!B || !all || !computed) return fail(RTI_EINVAL, "NULL argument");
    unsigned long long done = B->cells_done;
    if (B->mem) {   // the device slots stay current until the tables are rebuilt
        int rc = sum_cells(B, &done);
        if (rc) return rc;
    }
    *all = B->cell_updates_all;
    *computed = (int64_t)done;
    return RTI_OK;
}

void rti_batch_destroy(rti_batch *B)
{
    if (!B) return;
    (void)hipStreamSynchronize(B->stream);
    for (rti_domain *D : B->members) {
        D->batch = nullptr;
        (void)reset_counts(D);      // its parity moved under the batch
    }
    (void)hipStreamSynchronize(B->stream);
    for (rti_domain *D : B->members) D->stream = D->home_stream;
    drop_graphs(B);
    if (B->capture) (void)hipStreamDestroy(B->capture);
    if (B->mem) (void)hipFree(B->mem);
    delete B;
}

}  // extern "C"
