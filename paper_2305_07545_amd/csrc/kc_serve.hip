// Serving form: a request loop over device-resident countBFs (the request
// and session model is documented with the kc_server entry points).
//
// A lane is a slot for one batch of requests in flight.  Each lane owns
// device staging for its batch (the reads of its requests at 4096-aligned
// bases with 'N' gaps, their raw CSR offsets one request after another, the
// combined offsets of the whole buffer, a small table and the per-request
// result words, mirrored to pinned host memory), a copy stream, a compute
// stream and a kc_batch of its own (its scratch).  Issuing a lane enqueues
// its host-to-device copies on its copy stream and everything else on its
// compute stream behind an event: every request's insert goes through one
// kc_batch_insert call (whose large sets run on side lanes of their own),
// then the classifications.  Lanes run concurrently, so requests admitted
// while other batches are on the device overlap them.  A session's requests
// stay in submission order: a lane that takes a request of a session whose
// previous request is still in flight on another lane first waits for that
// session's event, recorded after each of its requests.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>
#include <deque>
#include <new>
#include <unordered_map>
#include <vector>

#include "kc_handle.hpp"
#include "kc_kernels.hpp"
#include "kmerco.h"

namespace {

using kcapi::dev_alloc;
using kcapi::dev_free;

constexpr uint32_t kRes = 8;  // result words per request
enum : uint32_t { kResWindows = 0, kResBefore = 1, kResAfter = 2, kResTrust = 3, kResErr = 4 };
constexpr uint64_t kAlign = 4096;   // set alignment of the batched form
constexpr uint32_t kMaxLanes = 8;
constexpr uint32_t kMaxLaneRequests = 4096;

uint64_t align_up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// out[0] = 0; out[1 + p] = raw[p] + base of the request that raw entry p
// belongs to.  tab holds (raw_start, base) per request, raw_start ascending
// from 0; each request's raw offsets start with its own 0, which becomes the
// end of the (possibly empty) gap read before it.
__global__ void k_serve_rebase(const uint64_t *__restrict__ raw, uint64_t n_raw,
                               const uint64_t *__restrict__ tab, uint32_t n_req,
                               uint64_t *__restrict__ out) {
    const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0)
        out[0] = 0;
    if (p >= n_raw)
        return;
    uint32_t lo = 0, hi = n_req;  // tab[2 * lo] <= p < tab[2 * hi]
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (tab[2 * (uint64_t)mid] <= p)
            lo = mid;
        else
            hi = mid;
    }
    out[1 + p] = raw[p] + tab[2 * (uint64_t)lo + 1];
}

// res[i * kRes + field] = *src[i] (the sessions' running distinct counts)
__global__ void k_serve_snap(const uint64_t *const *__restrict__ src, uint32_t n,
                             uint64_t *__restrict__ res, uint32_t field) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        res[(uint64_t)i * kRes + field] = *src[i];
}

enum class SState { Waiting, Open, Failed, Closed };

struct Session {
    kc_layout layout{};
    uint32_t k = 0;
    uint64_t cap = 0;
    uint64_t bytes = 0;
    SState state = SState::Waiting;
    bool closing = false;
    uint64_t *words = nullptr;
    uint64_t *distinct = nullptr;
    uint64_t *counter = nullptr;  // running distinct count (device)
    kc_filter *f = nullptr;
    hipEvent_t done = nullptr;   // recorded after each of its requests
    std::deque<uint64_t> queue;  // submitted, not issued (tickets)
    uint32_t inflight = 0;
};

struct Req {
    kc_request q{};
    uint64_t n_bases = 0;
    kc_result res{};
};

struct Lane {
    uint8_t *reads = nullptr;
    uint64_t *raw = nullptr, *comb = nullptr, *tab = nullptr, *res = nullptr;
    uint64_t *tab_host = nullptr, *res_host = nullptr;  // pinned
    hipStream_t copy = nullptr, compute = nullptr;
    hipEvent_t copied = nullptr, done = nullptr;
    kc_batch *batch = nullptr;
    bool busy = false;
    std::vector<uint64_t> tickets;
    std::vector<uint8_t> classify;  // per ticket
};

}  // namespace

struct kc_server {
    int device = 0;
    kc_server_config cfg{};
    hipStream_t admin = nullptr;  // session set-up (clears, classify scratch)
    std::vector<Session> sessions;
    std::deque<uint32_t> waiting;  // sessions to admit, in open order
    std::deque<uint64_t> order;    // submitted, not issued, in arrival order
    std::unordered_map<uint64_t, Req> reqs;
    std::vector<Lane> lanes;
    uint64_t next_ticket = 1;
    uint64_t used = 0;
    uint64_t staging = 0;
    kc_server_stats st{};
    std::chrono::steady_clock::time_point t0;
};

namespace {

double now_s(const kc_server *s) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - s->t0).count();
}

uint64_t key_words(uint32_t k) { return k > 32 ? 2 : 1; }

// A session's device bytes: countBF, distinct list, its count, the direct
// path's per-counter entries when the countBF takes that path, and the
// classification scratch for its whole list.
uint64_t session_bytes(const kc_layout &L, uint32_t k, uint64_t cap) {
    const uint64_t tiles = kc::tiles(cap) + 1;
    return L.X * L.Y * 8 + cap * 8 * key_words(k) + 8 + kcapi::filter_private_bytes(L) +
           tiles * (3 * 4 + 3 * 8 + kc::kTile / 8) + 64;
}

void release(kc_server *s, Session &S) {
    if (S.f) {
        kc_destroy(S.f);
        S.f = nullptr;
    }
    if (S.done) {
        (void)hipEventDestroy(S.done);
        S.done = nullptr;
    }
    dev_free(S.words);
    dev_free(S.distinct);
    dev_free(S.counter);
    if (S.state == SState::Open)
        s->used -= S.bytes;
    S.state = SState::Closed;
}

// Allocate and clear a session on the admin stream; its event marks the
// clears, so that the first lane to take one of its requests waits for them.
kc_status admit_one(kc_server *s, Session &S) {
    if (!dev_alloc(&S.words, S.layout.X * S.layout.Y) ||
        !dev_alloc(&S.distinct, S.cap * key_words(S.k)) || !dev_alloc(&S.counter, 1))
        return KC_ENOMEM;
    if (kc::fill_u64(S.counter, 1, 0, s->admin) != hipSuccess)
        return KC_EDEVICE;
    // the handle knows its k from the start (classify requests before any
    // insert read keys of that width)
    kc_status st = kc_create_in(&S.layout, S.words, 1, S.k, nullptr, 0, 0, s->admin, &S.f);
    if (st != KC_OK)
        return st;
    // classification scratch for the session's whole list, so that a lane
    // never allocates (or waits) when it classifies
    kcapi::DeviceGuard g(s->device);
    if ((st = kcapi::ensure_scalars(*S.f->W)) != KC_OK ||
        (st = kcapi::ensure_tiles(*S.f->W, s->admin, S.cap)) != KC_OK)
        return st;
    if (hipEventCreateWithFlags(&S.done, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(S.done, s->admin) != hipSuccess)
        return KC_EDEVICE;
    return KC_OK;
}

void fail_queue(kc_server *s, Session &S, kc_status why) {
    const double t = now_s(s);
    for (uint64_t tk : S.queue) {
        for (auto it = s->order.begin(); it != s->order.end(); ++it)
            if (*it == tk) {
                s->order.erase(it);
                break;
            }
        Req &R = s->reqs[tk];
        R.res.status = why;
        R.res.done = 1;
        R.res.t_issue = R.res.t_done = t;
        s->st.requests_done++;
    }
    S.queue.clear();
}

void admit(kc_server *s) {
    while (!s->waiting.empty()) {
        Session &S = s->sessions[s->waiting.front()];
        if (S.state != SState::Waiting) {
            s->waiting.pop_front();
            continue;
        }
        if (s->used + S.bytes > s->cfg.memory_budget)
            return;  // in order: later sessions wait behind this one
        s->waiting.pop_front();
        kc_status st = admit_one(s, S);
        if (st != KC_OK) {
            dev_free(S.words);
            dev_free(S.distinct);
            dev_free(S.counter);
            if (S.f) {
                kc_destroy(S.f);
                S.f = nullptr;
            }
            S.state = SState::Failed;
            if (S.done) {
                (void)hipEventDestroy(S.done);
                S.done = nullptr;
            }
            fail_queue(s, S, st);
            continue;
        }
        S.state = SState::Open;
        s->used += S.bytes;
    }
}

void maybe_release(kc_server *s, Session &S) {
    if (S.closing && S.state == SState::Open && S.inflight == 0 && S.queue.empty())
        release(s, S);
}

uint32_t retire(kc_server *s) {
    uint32_t n = 0;
    for (Lane &L : s->lanes) {
        if (!L.busy)
            continue;
        hipError_t e = hipEventQuery(L.done);
        if (e == hipErrorNotReady)
            continue;
        const double t = now_s(s);
        for (size_t i = 0; i < L.tickets.size(); i++) {
            Req &R = s->reqs[L.tickets[i]];
            Session &S = s->sessions[R.q.session];
            const uint64_t *r = L.res_host + i * kRes;
            if (e != hipSuccess) {
                R.res.status = KC_EDEVICE;
            } else if (R.res.status == KC_OK) {
                R.res.n_windows = r[kResWindows];
                R.res.distinct_first = r[kResBefore];
                R.res.n_new = r[kResAfter] - r[kResBefore];
                if (r[kResAfter] > S.cap)
                    R.res.status = KC_ERANGE;
                if (L.classify[i]) {
                    R.res.n_trust = r[kResTrust];
                    R.res.n_err = r[kResErr];
                    if (r[kResAfter] > R.q.class_cap)
                        R.res.status = KC_ERANGE;
                }
            }
            R.res.t_done = t;
            R.res.done = 1;
            S.inflight--;
            n++;
        }
        for (uint64_t tk : L.tickets)
            maybe_release(s, s->sessions[s->reqs[tk].q.session]);
        L.busy = false;
        L.tickets.clear();
        L.classify.clear();
    }
    s->st.requests_done += n;
    return n;
}

// Enqueue one lane: copies on its copy stream, calls on its compute stream.
kc_status issue_lane(kc_server *s, Lane &L, std::vector<uint64_t> &picked) {
    const std::vector<uint64_t> &all = picked;
    const uint32_t n = (uint32_t)all.size();
    L.classify.assign(n, 0);
    // layout of the lane buffers: each inserting request's reads at a
    // 4096-aligned base, its raw offsets after the previous request's
    std::vector<uint64_t> base(n), rawpos(n);
    uint64_t pos = 0, raw = 0;
    uint32_t n_ins = 0;
    for (uint32_t i = 0; i < n; i++) {
        const Req &R = s->reqs[all[i]];
        base[i] = align_up(pos);
        rawpos[i] = raw;
        const bool ins = R.q.op & KC_OP_INSERT;
        pos = base[i] + (ins ? R.n_bases : 0);
        raw += ins ? R.q.n_reads + 1 : 0;
        n_ins += ins;
    }
    // the lane buffers: lane_bases + lane_requests * kAlign bases, lane_reads
    // + lane_requests raw offsets (+1 combined)
    if (n > s->cfg.lane_requests ||
        pos > s->cfg.lane_bases + (uint64_t)s->cfg.lane_requests * kAlign ||
        raw > s->cfg.lane_reads + s->cfg.lane_requests) {
        for (uint64_t tk : all)
            s->reqs[tk].res.status = KC_EINVAL;  // not reachable through issue()
        L.tickets = all;
        L.busy = true;
        for (uint64_t tk : all)
            s->sessions[s->reqs[tk].q.session].inflight++;
        (void)hipEventRecord(L.done, L.compute);
        return KC_EINVAL;
    }
    uint64_t *tab = L.tab_host;  // (raw_start, base) per request, then counter pointers
    for (uint32_t i = 0; i < n; i++) {
        tab[2 * i] = rawpos[i];
        tab[2 * i + 1] = base[i];
        tab[2 * n + i] = (uint64_t)(uintptr_t)s->sessions[s->reqs[all[i]].q.session].counter;
    }
    hipError_t e = hipSuccess;
    uint64_t end = 0;
    for (uint32_t i = 0; i < n && e == hipSuccess; i++) {
        const Req &R = s->reqs[all[i]];
        if (!(R.q.op & KC_OP_INSERT))
            continue;
        if (base[i] > end)
            e = hipMemsetAsync(L.reads + end, 'N', base[i] - end, L.copy);
        if (e == hipSuccess && R.n_bases)
            e = hipMemcpyAsync(L.reads + base[i], R.q.reads_host, R.n_bases,
                               hipMemcpyHostToDevice, L.copy);
        if (e == hipSuccess)
            e = hipMemcpyAsync(L.raw + rawpos[i], R.q.offsets_host,
                               (R.q.n_reads + 1) * sizeof(uint64_t), hipMemcpyHostToDevice,
                               L.copy);
        end = base[i] + R.n_bases;
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(L.tab, tab, 3 * (uint64_t)n * sizeof(uint64_t), hipMemcpyHostToDevice,
                           L.copy);
    if (e == hipSuccess)
        e = hipEventRecord(L.copied, L.copy);
    if (e == hipSuccess)
        e = hipStreamWaitEvent(L.compute, L.copied, 0);
    // each session's previous request (on any lane) and its admission
    for (uint32_t i = 0; i < n && e == hipSuccess; i++)
        e = hipStreamWaitEvent(L.compute, s->sessions[s->reqs[all[i]].q.session].done, 0);
    const uint64_t *const *ctrs = (const uint64_t *const *)(L.tab + 2 * n);
    const uint32_t tb = 256, grid_n = (n + tb - 1) / tb;
    if (e == hipSuccess)
        e = kc::fill_u64(L.res, (uint64_t)n * kRes, 0, L.compute);
    if (e == hipSuccess) {
        k_serve_snap<<<grid_n, tb, 0, L.compute>>>(ctrs, n, L.res, kResBefore);
        e = hipGetLastError();
    }
    kc_status st = e == hipSuccess ? KC_OK : KC_EDEVICE;
    if (st == KC_OK && n_ins > 0) {
        // one batched call for every insert of the lane: the combined CSR has
        // one (gap) read before each request plus its reads
        const uint64_t blocks = (raw + tb - 1) / tb;
        k_serve_rebase<<<(uint32_t)blocks, tb, 0, L.compute>>>(L.raw, raw, L.tab, n, L.comb);
        st = hipGetLastError() == hipSuccess ? KC_OK : KC_EDEVICE;
        std::vector<kc_set> sets;
        for (uint32_t i = 0; i < n; i++) {
            const Req &R = s->reqs[all[i]];
            if (!(R.q.op & KC_OP_INSERT))
                continue;
            const Session &S = s->sessions[R.q.session];
            kc_set q;
            std::memset(&q, 0, sizeof q);
            q.filter = S.f;
            q.first_base = base[i];
            q.n_bases = R.n_bases;
            q.k = S.k;
            q.distinct_dev = S.distinct;
            q.distinct_cap = S.cap;
            q.n_distinct_dev = S.counter;
            q.n_windows_dev = L.res + (uint64_t)i * kRes + kResWindows;
            sets.push_back(q);
        }
        if (st == KC_OK)
            st = kc_batch_insert(L.batch, sets.data(), (uint32_t)sets.size(), L.reads, L.comb,
                                 raw, pos, 0, L.compute);
        s->st.batched_requests += sets.size();
    }
    for (uint32_t i = 0; i < n && st == KC_OK; i++) {
        const Req &R = s->reqs[all[i]];
        if (!(R.q.op & KC_OP_CLASSIFY))
            continue;
        const Session &S = s->sessions[R.q.session];
        L.classify[i] = 1;
        const uint64_t cap = S.cap < R.q.class_cap ? S.cap : R.q.class_cap;
        st = kc_classify(S.f, S.distinct, S.counter, cap, R.q.tau, R.q.trust_dev,
                         L.res + (uint64_t)i * kRes + kResTrust, R.q.err_dev,
                         L.res + (uint64_t)i * kRes + kResErr, L.compute);
    }
    if (st == KC_OK) {
        k_serve_snap<<<grid_n, tb, 0, L.compute>>>(ctrs, n, L.res, kResAfter);
        e = hipGetLastError();
        for (uint32_t i = 0; i < n && e == hipSuccess; i++)
            e = hipEventRecord(s->sessions[s->reqs[all[i]].q.session].done, L.compute);
        if (e == hipSuccess)
            e = hipMemcpyAsync(L.res_host, L.res, (uint64_t)n * kRes * sizeof(uint64_t),
                               hipMemcpyDeviceToHost, L.compute);
        if (e == hipSuccess)
            e = hipEventRecord(L.done, L.compute);
        if (e != hipSuccess)
            st = KC_EDEVICE;
    }
    const double t = now_s(s);
    for (uint32_t i = 0; i < n; i++) {
        Req &R = s->reqs[all[i]];
        R.res.t_issue = t;
        s->sessions[R.q.session].inflight++;
    }
    L.tickets = all;
    L.busy = true;
    s->st.batches++;
    if (n > s->st.max_batch)
        s->st.max_batch = n;
    if (st != KC_OK) {
        // the lane's work may be partly enqueued: wait for it, then report
        (void)hipStreamSynchronize(L.compute);
        for (uint32_t i = 0; i < n; i++) {
            s->reqs[all[i]].res.status = st;
            (void)hipEventRecord(s->sessions[s->reqs[all[i]].q.session].done, L.compute);
        }
        (void)hipEventRecord(L.done, L.compute);
    }
    return st;
}

void issue(kc_server *s) {
    for (Lane &L : s->lanes) {
        if (L.busy)
            continue;
        std::vector<uint64_t> picked;
        std::vector<uint32_t> in_batch;
        uint64_t bases = 0, reads = 0;
        for (uint64_t tk : s->order) {
            if (picked.size() >= s->cfg.lane_requests)
                break;
            const Req &R = s->reqs[tk];
            const Session &S = s->sessions[R.q.session];
            if (S.state != SState::Open || S.queue.empty() || S.queue.front() != tk)
                continue;
            bool dup = false;
            for (uint32_t id : in_batch)
                dup |= id == R.q.session;
            if (dup)
                continue;
            // unpadded sums: the lane buffer has kAlign bytes of room per
            // request for alignment in whatever order issue_lane lays them out
            const bool ins = R.q.op & KC_OP_INSERT;
            const uint64_t nb = ins ? bases + R.n_bases : bases;
            const uint64_t nr = ins ? reads + R.q.n_reads + 1 : reads;
            if (nb > s->cfg.lane_bases || nr > s->cfg.lane_reads + s->cfg.lane_requests)
                continue;
            bases = nb;
            reads = nr;
            picked.push_back(tk);
            in_batch.push_back(R.q.session);
        }
        if (picked.empty())
            return;
        for (uint64_t tk : picked) {
            Session &S = s->sessions[s->reqs[tk].q.session];
            S.queue.pop_front();
            for (auto it = s->order.begin(); it != s->order.end(); ++it)
                if (*it == tk) {
                    s->order.erase(it);
                    break;
                }
        }
        (void)issue_lane(s, L, picked);
        uint32_t busy = 0;
        for (const Lane &M : s->lanes)
            busy += M.busy;
        if (busy > s->st.lanes_in_flight_max)
            s->st.lanes_in_flight_max = busy;
    }
}

// Wait for everything the server has enqueued.
bool sync_all(kc_server *s) {
    bool ok = !s->admin || hipStreamSynchronize(s->admin) == hipSuccess;
    for (Lane &L : s->lanes) {
        if (L.copy)
            ok &= hipStreamSynchronize(L.copy) == hipSuccess;
        if (L.compute)
            ok &= hipStreamSynchronize(L.compute) == hipSuccess;
    }
    return ok;
}

void free_lane(Lane &L) {
    dev_free(L.reads);
    dev_free(L.raw);
    dev_free(L.comb);
    dev_free(L.tab);
    dev_free(L.res);
    if (L.tab_host)
        (void)hipHostFree(L.tab_host);
    if (L.res_host)
        (void)hipHostFree(L.res_host);
    if (L.copied)
        (void)hipEventDestroy(L.copied);
    if (L.done)
        (void)hipEventDestroy(L.done);
    if (L.batch)
        kc_batch_destroy(L.batch);
    if (L.copy)
        (void)hipStreamDestroy(L.copy);
    if (L.compute)
        (void)hipStreamDestroy(L.compute);
    L = Lane{};
}

}  // namespace

extern "C" {

kc_status kc_server_create(const kc_server_config *cfg, kc_server **out) {
    if (!out)
        return KC_EINVAL;
    *out = nullptr;
    if (!cfg || cfg->lanes < 1 || cfg->lanes > kMaxLanes || cfg->lane_requests < 1 ||
        cfg->lane_requests > kMaxLaneRequests || cfg->lane_bases < 1 || cfg->lane_reads < 1)
        return KC_EINVAL;
    kc_server *s = new (std::nothrow) kc_server();
    if (!s)
        return KC_ENOMEM;
    s->cfg = *cfg;
    s->t0 = std::chrono::steady_clock::now();
    kc_status st = KC_OK;
    // every stream at the default priority
    if (hipGetDevice(&s->device) != hipSuccess ||
        hipStreamCreateWithFlags(&s->admin, hipStreamNonBlocking) != hipSuccess)
        st = KC_EDEVICE;
    const uint64_t nb = cfg->lane_bases + (uint64_t)cfg->lane_requests * kAlign;
    const uint64_t nr = cfg->lane_reads + cfg->lane_requests;
    s->lanes.resize(cfg->lanes);
    for (Lane &L : s->lanes) {
        if (st != KC_OK)
            break;
        if (!dev_alloc(&L.reads, nb) || !dev_alloc(&L.raw, nr) || !dev_alloc(&L.comb, nr + 1) ||
            !dev_alloc(&L.tab, 3ull * cfg->lane_requests) ||
            !dev_alloc(&L.res, (uint64_t)kRes * cfg->lane_requests) ||
            hipHostMalloc((void **)&L.tab_host, 3ull * cfg->lane_requests * sizeof(uint64_t),
                          hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void **)&L.res_host,
                          (uint64_t)kRes * cfg->lane_requests * sizeof(uint64_t),
                          hipHostMallocDefault) != hipSuccess)
            st = KC_ENOMEM;
        else if (hipEventCreateWithFlags(&L.copied, hipEventDisableTiming) != hipSuccess ||
                 hipEventCreateWithFlags(&L.done, hipEventDisableTiming) != hipSuccess ||
                 hipStreamCreateWithFlags(&L.copy, hipStreamNonBlocking) != hipSuccess ||
                 hipStreamCreateWithFlags(&L.compute, hipStreamNonBlocking) != hipSuccess)
            st = KC_EDEVICE;
        else
            st = kc_batch_create(&L.batch);
        s->staging += nb + (2 * nr + 1 + 3ull * cfg->lane_requests +
                            (uint64_t)kRes * cfg->lane_requests) * sizeof(uint64_t);
    }
    if (st != KC_OK) {
        kc_server_destroy(s);
        return st;
    }
    *out = s;
    return KC_OK;
}

void kc_server_destroy(kc_server *s) {
    if (!s)
        return;
    kcapi::DeviceGuard g(s->device);
    sync_all(s);
    for (Session &S : s->sessions)
        if (S.state == SState::Open)
            release(s, S);
    for (Lane &L : s->lanes)
        free_lane(L);
    if (s->admin)
        (void)hipStreamDestroy(s->admin);
    delete s;
}

kc_status kc_server_open(kc_server *s, const kc_layout *layout, uint32_t k,
                         uint64_t distinct_cap, uint32_t *session) {
    if (!s || !session || !layout || !kcapi::valid_layout(layout) || k < 1 || k > 64)
        return KC_EINVAL;
    Session S;
    S.layout = *layout;
    S.k = k;
    S.cap = distinct_cap;
    S.bytes = session_bytes(*layout, k, distinct_cap);
    if (S.bytes > s->cfg.memory_budget)
        return KC_ENOMEM;
    *session = (uint32_t)s->sessions.size();
    s->sessions.push_back(std::move(S));
    s->waiting.push_back(*session);
    kcapi::DeviceGuard g(s->device);
    admit(s);
    return KC_OK;
}

kc_status kc_server_close(kc_server *s, uint32_t session) {
    if (!s || session >= s->sessions.size())
        return KC_EINVAL;
    Session &S = s->sessions[session];
    if (S.closing || S.state == SState::Closed)
        return KC_ESTATE;
    S.closing = true;
    kcapi::DeviceGuard g(s->device);
    if (S.state == SState::Waiting && S.queue.empty()) {
        S.state = SState::Closed;
    } else {
        maybe_release(s, S);
    }
    admit(s);
    return KC_OK;
}

kc_status kc_server_submit(kc_server *s, const kc_request *req, uint64_t *ticket) {
    if (!s || !req || !ticket || req->session >= s->sessions.size() || req->reserved != 0)
        return KC_EINVAL;
    Session &S = s->sessions[req->session];
    if (S.closing || S.state == SState::Closed || S.state == SState::Failed)
        return KC_ESTATE;
    const uint32_t op = req->op;
    if (op == 0 || (op & ~(KC_OP_INSERT | KC_OP_CLASSIFY)) != 0)
        return KC_EINVAL;
    Req R;
    R.q = *req;
    if (op & KC_OP_INSERT) {
        if (!req->offsets_host || (req->n_reads > 0 && !req->reads_host))
            return KC_EINVAL;
        const uint64_t *o = req->offsets_host;
        if (o[0] != 0)
            return KC_EINVAL;
        for (uint64_t i = 0; i < req->n_reads; i++)
            if (o[i + 1] < o[i])
                return KC_EINVAL;
        R.n_bases = o[req->n_reads];
        if (R.n_bases > s->cfg.lane_bases || req->n_reads > s->cfg.lane_reads)
            return KC_ERANGE;
    }
    if ((op & KC_OP_CLASSIFY) && (!req->trust_dev || !req->err_dev))
        return KC_EINVAL;
    R.res.t_submit = now_s(s);
    const uint64_t tk = s->next_ticket++;
    s->reqs.emplace(tk, R);
    *ticket = tk;
    S.queue.push_back(tk);
    s->order.push_back(tk);
    return KC_OK;
}

kc_status kc_server_pump(kc_server *s, uint32_t *n_done) {
    if (!s)
        return KC_EINVAL;
    kcapi::DeviceGuard g(s->device);
    const uint32_t n = retire(s);
    admit(s);
    issue(s);
    if (n_done)
        *n_done = n;
    return KC_OK;
}

kc_status kc_server_wait(kc_server *s, uint64_t ticket) {
    if (!s || (ticket != 0 && s->reqs.find(ticket) == s->reqs.end()))
        return KC_EINVAL;
    for (;;) {
        kc_status st = kc_server_pump(s, nullptr);
        if (st != KC_OK)
            return st;
        Lane *busy = nullptr;
        for (Lane &L : s->lanes)
            if (L.busy && !busy)
                busy = &L;
        if (ticket != 0 ? s->reqs[ticket].res.done != 0 : (s->order.empty() && !busy))
            return KC_OK;
        if (!busy)  // nothing runs and nothing could be issued: the rest waits
            return KC_ESTATE;  // for session memory that only a close releases
        kcapi::DeviceGuard g(s->device);
        (void)hipEventSynchronize(busy->done);
    }
}

kc_status kc_server_result(const kc_server *s, uint64_t ticket, kc_result *out) {
    if (!s || !out)
        return KC_EINVAL;
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end())
        return KC_EINVAL;
    *out = it->second.res;
    return KC_OK;
}

kc_status kc_server_release(kc_server *s, uint64_t ticket) {
    if (!s)
        return KC_EINVAL;
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end())
        return KC_EINVAL;
    if (!it->second.res.done)
        return KC_ESTATE;
    s->reqs.erase(it);
    return KC_OK;
}

kc_status kc_server_read_distinct(kc_server *s, uint32_t session, uint64_t first, uint64_t n,
                                  uint64_t *dst_host) {
    if (!s || session >= s->sessions.size() || (n > 0 && !dst_host))
        return KC_EINVAL;
    Session &S = s->sessions[session];
    if (S.state != SState::Open)
        return KC_ESTATE;
    kcapi::DeviceGuard g(s->device);
    if (!sync_all(s))
        return KC_EDEVICE;
    uint64_t nd = 0;
    if (hipMemcpy(&nd, S.counter, sizeof nd, hipMemcpyDeviceToHost) != hipSuccess)
        return KC_EDEVICE;
    const uint64_t have = nd < S.cap ? nd : S.cap;
    if (first > have || n > have - first)
        return KC_ERANGE;
    const uint64_t w = key_words(S.k);
    if (n && hipMemcpy(dst_host, S.distinct + first * w, n * w * sizeof(uint64_t),
                       hipMemcpyDeviceToHost) != hipSuccess)
        return KC_EDEVICE;
    return KC_OK;
}

kc_status kc_server_read_words(kc_server *s, uint32_t session, uint64_t *dst_host) {
    if (!s || session >= s->sessions.size() || !dst_host)
        return KC_EINVAL;
    Session &S = s->sessions[session];
    if (S.state != SState::Open)
        return KC_ESTATE;
    kcapi::DeviceGuard g(s->device);
    if (!sync_all(s))
        return KC_EDEVICE;
    if (hipMemcpy(dst_host, S.words, S.layout.X * S.layout.Y * sizeof(uint64_t),
                  hipMemcpyDeviceToHost) != hipSuccess)
        return KC_EDEVICE;
    return KC_OK;
}

kc_status kc_server_stats_get(const kc_server *s, kc_server_stats *out) {
    if (!s || !out)
        return KC_EINVAL;
    *out = s->st;
    out->session_bytes = s->used;
    out->staging_bytes = s->staging;
    out->sessions_open = out->sessions_waiting = 0;
    for (const Session &S : s->sessions) {
        out->sessions_open += S.state == SState::Open;
        out->sessions_waiting += S.state == SState::Waiting;
    }
    return KC_OK;
}

double kc_server_now(const kc_server *s) { return s ? now_s(s) : 0.0; }

}  // extern "C"
