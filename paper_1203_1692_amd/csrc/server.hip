// Serving loop: FIFO admission by device-memory footprint and free slots,
// tree builds and culls of many requests in shared launches (rounds),
// batched leaf-GEMM launches across requests on one GEMM stream, squaring
// chains kept on the device.
//
// Rounds (requests of depth 1..8, every serving size): the steps waiting
// for their build and cull are gathered into one round on a prep stream ps
// (two rounds in flight, one per prep stream):
//   ps: [wait for the GEMMs enqueued so far, when a chain step is in it] ->
// keep flags of the output trees -> every tree's leaf norms -> the pyramids
// -> the pack of the leaves that some kept product can read (tau > 0: a leaf
// with fl64(s max(||A||^2, ||B||^2)) < tau^2 never passes the product test,
// Sec. II.C; its norm stays, so task sets, roots and C are those of the
// dense trees) -> the culls of all plans, tier by tier -> one readback of
// every plan's counts and roots -> record the round's event.  About 15 launches
// for up to 16 requests, where one request alone took 10 to 18.  Once the
// host sees the event, the round's requests join the next GEMM batch; a
// chain request's next step joins the next round.
//
// Other depths run each step on their slot's stream (slot stream ss, GEMM
// stream gs):
//   ss: build tree(s) -> root norm to pinned host -> cull -> task counts to
//       pinned host -> record ev_cull
//   gs: a batch of requests whose ev_cull has completed (the host polls it,
//       so a long build or cull never holds up the GEMM stream) -> one launch
//       per kernel kind -> record ev_done
//   chain step s -> s+1, enqueued at once after the GEMM:
//   ss: wait ev_done -> build the tree of X_{s+1} from C and step s's
//       schedule over the arena space of X_s's tree -> cull -> ... (no host
//       round trip).  Only the leaves of C that step s's kept products reach
//       are read (the others are zero), and the GEMM of every step before
//       the last writes only the blocks that have products.
// The host only watches ev_done of a request's last product.
//
// Memory: each slot owns one device arena (trees + task arena of its current
// request, carved at fixed offsets), kept across requests and grown when a
// larger request lands on the slot, so the steady state allocates nothing.
// The arenas together never exceed the server's budget.
#include <math.h>
#include <pthread.h>
#include <sys/prctl.h>
#include <string.h>
#include <time.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "runtime.hpp"

using namespace spamm;

namespace {

constexpr int kMaxSlots = 64;
constexpr int kMaxChain = 64;
constexpr size_t kMaxQueue = 65536;
// GEMM batches allowed on the GEMM stream at once; requests culled while
// the stream is full wait and join the next batch.
constexpr int kInflightBatches = 2;
// rounds in flight, each on a prep stream of its own: a round is a chain of
// short launches, so two overlap on the chip; a new round takes every step
// waiting at the time (up to kMaxRound)
constexpr int kRounds = 2;
// idle scheduler passes that yield before it sleeps between polls
constexpr int kSpinPasses = 16;

struct StepOut {                   // one step's cull readback: its plan's leafK[0..5)
    uint64_t K[2];                 // HIGH / LOW leaf products
    uint64_t sub;                  // (sub-leaf products; not used by the server)
    double root[2];                // ||X_s||_F^2 of the step's left and right trees
};
static_assert(sizeof(StepOut) == 5 * sizeof(uint64_t), "plan leafK layout");

struct Pinned {                    // per-slot readbacks (host-visible)
    StepOut step[kMaxChain];
};

struct Job {
    uint64_t ticket;
    spamm_request rq;
    size_t bytes;
    double t_submit;
    bool batched;                  // its steps go through rounds
};

// a batched request's step: waiting for a round, in one, culled
enum Phase : int { kIdle = 0, kPrep, kCulling, kReady };

struct Round {
    hipStream_t s = nullptr;       // the round's prep stream
    hipEvent_t ev = nullptr;
    uint64_t *dout = nullptr;      // device: 5 words per plan (launch_cull_round)
    uint64_t *hout = nullptr;      // pinned copy of dout
    std::vector<uint64_t> tickets; // the requests of the round, in plan order
    bool busy = false;
};

struct Active {
    Job job;
    int slot = -1;
    int steps = 1, step = 0;
    bool split = false, distinctB = false;
    spamm_tree *tA = nullptr, *tB = nullptr;
    spamm_plan *plan = nullptr;
    bool culled = false;           // this step's cull enqueued, its GEMM not yet
    bool batched = false;
    int phase = kIdle;             // batched requests
    bool final = false;            // nothing more to enqueue; done once ev_done passes
    int status = SPAMM_OK;
    double t_admit = 0.0;
};

bool bad_tol(double v) { return !(v >= 0.0) || isinf(v) || (v > 0.0 && v < 1e-150); }

int check_request(const spamm_request *r, size_t *bytes, bool *batched = nullptr)
{
    if (r == nullptr)
        return fail(SPAMM_E_INVAL, "request is NULL");
    if (r->A == nullptr || r->C == nullptr)
        return fail(SPAMM_E_INVAL, "A and C must be device pointers");
    if (r->n < 1)
        return fail(SPAMM_E_INVAL, "n = %lld < 1", (long long)r->n);
    if (r->leaf != 16 && r->leaf != 32 && r->leaf != 64)
        return fail(SPAMM_E_INVAL, "leaf = %d not in {16, 32, 64}", r->leaf);
    if (r->precision != SPAMM_PREC_FP32 && r->precision != SPAMM_PREC_SPLIT_BF16 &&
        r->precision != SPAMM_PREC_SPLIT_FP16 && r->precision != SPAMM_PREC_SPLIT_BF16X3)
        return fail(SPAMM_E_INVAL, "unknown precision %d", r->precision);
    const bool split = r->precision != SPAMM_PREC_FP32;
    if (split && r->leaf == 16)
        return fail(SPAMM_E_INVAL, "split precision needs leaf 32 or 64");
    if (bad_tol(r->tau))
        return fail(SPAMM_E_INVAL, "tau = %g must be 0 or in [1e-150, inf)", r->tau);
    if (split && bad_tol(r->low_tol))
        return fail(SPAMM_E_INVAL, "low_tol = %g must be 0 or in [1e-150, inf)", r->low_tol);
    if (split && bad_tol(r->low_rel))
        return fail(SPAMM_E_INVAL, "low_rel = %g must be 0 or in [1e-150, inf)", r->low_rel);
    if (split && r->low_tol > 0.0 && r->low_rel > 0.0)
        return fail(SPAMM_E_INVAL, "low_tol = %g and low_rel = %g: give one threshold",
                    r->low_tol, r->low_rel);
    if (r->chain_len < 0 || r->chain_len > kMaxChain)
        return fail(SPAMM_E_INVAL, "chain_len = %d outside 0..%d", r->chain_len, kMaxChain);
    if (r->chain_len > 0 && r->B != nullptr && r->B != r->A)
        return fail(SPAMM_E_INVAL, "a squaring chain takes B = NULL (or B = A)");
    int32_t d;
    int64_t np;
    int rc = tree_depth(r->n, r->leaf, &d, &np);
    if (rc)
        return rc;
    const bool distinctB = r->B != nullptr && r->B != r->A;
    *bytes = tree_device_bytes(r->n, r->leaf, tree_flags_for(r->precision)) * (distinctB ? 2 : 1) +
             plan_device_bytes(d, split) + (r->chain_len > 0 ? output_map_bytes(d) : 0);
    if (batched != nullptr)
        *batched = d >= 1 && d <= kRoundMaxDepth;
    return SPAMM_OK;
}

}  // namespace

struct spamm_server {
    int device = -1;
    size_t budget = 0;
    int nslots = 0;
    hipStream_t gemm = nullptr;
    Round rounds[kRounds];               // each with its prep stream
    hipStream_t ss[kMaxSlots] = {};
    hipEvent_t ev_cull[kMaxSlots] = {}, ev_done[kMaxSlots] = {};
    Pinned *pin = nullptr;
    std::deque<hipEvent_t> inflight;     // batch events on the GEMM stream
    std::vector<hipEvent_t> spare;       // idle batch events

    // shared with submit / poll (guarded by mu)
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Job> queue;
    std::unordered_set<uint64_t> live;   // queued or admitted
    std::unordered_map<uint64_t, spamm_result> done;
    size_t used = 0;                     // bytes held by the slot arenas
    void *arena[kMaxSlots] = {};
    size_t cap[kMaxSlots] = {};
    spamm_server_stats st{};
    bool busy[kMaxSlots] = {};
    uint64_t next_ticket = 1;
    bool stopping = false;
    double t_start = 0.0;          // host clock (us) when the scheduler started

    // scheduler thread only
    std::vector<Active> active;
    std::thread worker;
};

namespace {

// Enqueue the trees and the cull of the request's current step on its slot
// stream.  Step 0 reads A (and B); step s > 0 builds the tree of X_s from C
// and the plan `prev` of step s-1 that wrote it: only the leaves that step's
// kept products reached are read (the others are zero).
int start_step(spamm_server *S, Active &a, const spamm_plan *prev)
{
    hipStream_t ss = S->ss[a.slot];
    Pinned &P = S->pin[a.slot];
    const spamm_request &r = a.job.rq;
    const uint32_t flags = tree_flags_for(r.precision);
    // arena: [tree of A or X_s][tree of B, step 0 only][plan][output map, chains]
    char *base = (char *)S->arena[a.slot];
    const size_t tb = tree_device_bytes(r.n, r.leaf, flags);
    int rc;
    if (a.step == 0) {
        rc = tree_build_async(r.A, r.n, r.leaf, flags, ss, nullptr, &a.tA, base);
    } else {
        char *map = base + tb + plan_device_bytes(prev->depth, a.split);
        rc = tree_build_output_async(r.C, prev, flags, ss, &a.tA, base, map);
    }
    if (rc)
        return rc;
    if (a.step == 0 && a.distinctB) {
        if ((rc = tree_build_async(r.B, r.n, r.leaf, flags, ss, nullptr, &a.tB, base + tb)))
            return rc;
    } else {
        a.tB = a.tA;
    }
    spamm_opts o{};
    o.tau = r.tau;
    o.precision = r.precision;
    o.low_tol = a.split ? r.low_tol : 0.0;
    // a relative threshold is taken against this step's own roots on the device
    o.low_rel = a.split ? r.low_rel : 0.0;
    if ((rc = symbolic_async(a.tA, a.tB, &o, ss, base + (a.distinctB ? 2 : 1) * tb, &a.plan)))
        return rc;
    // kept counts and both roots in one copy (the cull writes them all)
    hipError_t e = hipMemcpyAsync(&P.step[a.step], a.plan->leafK, sizeof(StepOut),
                                  hipMemcpyDeviceToHost, ss);
    if (e == hipSuccess)
        e = hipEventRecord(S->ev_cull[a.slot], ss);
    if (e != hipSuccess)
        return hip_fail(e, "server step");
    a.culled = true;
    return SPAMM_OK;
}

// Order the slot stream after the step's GEMM (the next step overwrites the
// arena and reads C) and drop the step's handles; their buffers live in the
// slot arena.
void release_step(spamm_server *S, Active &a)
{
    hipStream_t ss = S->ss[a.slot];
    hipStreamWaitEvent(ss, S->ev_done[a.slot], 0);
    spamm_plan_free(a.plan);
    if (a.tB != nullptr && a.tB != a.tA)
        spamm_tree_free(a.tB);
    spamm_tree_free(a.tA);
    a.plan = nullptr;
    a.tA = a.tB = nullptr;
}

// After the GEMM of step s was enqueued: queue step s+1 or mark final.
void advance(spamm_server *S, Active &a)
{
    a.culled = false;
    a.phase = kIdle;
    if (a.step + 1 >= a.steps) {
        a.final = true;
        return;
    }
    if (a.batched) {
        // the next round builds step s+1 from C and this step's plan (kept
        // until then, with the step's trees)
        a.step += 1;
        a.phase = kPrep;
        return;
    }
    // step s+1 reads C and step s's schedule, and overwrites step s's trees:
    // the slot stream waits for the GEMM; the handles of step s go once step
    // s+1 is enqueued (their buffers live in the slot arena)
    hipStreamWaitEvent(S->ss[a.slot], S->ev_done[a.slot], 0);
    spamm_plan *prev = a.plan;
    spamm_tree *pA = a.tA, *pB = a.tB;
    a.plan = nullptr;
    a.tA = a.tB = nullptr;
    a.step += 1;
    int rc = start_step(S, a, prev);
    spamm_plan_free(prev);
    if (pB != nullptr && pB != pA)
        spamm_tree_free(pB);
    spamm_tree_free(pA);
    if (rc) {
        a.status = rc;
        a.final = true;
    }
}

// Gather every culled request into batched launches on the GEMM stream.
// Returns true if anything was launched.
bool launch_batches(spamm_server *S)
{
    while (!S->inflight.empty() && hipEventQuery(S->inflight.front()) == hipSuccess) {
        S->spare.push_back(S->inflight.front());
        S->inflight.pop_front();
    }
    bool any = false;
    std::vector<size_t> ready;
    for (size_t i = 0; i < S->active.size(); ++i) {
        Active &a = S->active[i];
        if (a.batched) {
            if (a.phase == kReady)
                ready.push_back(i);
            continue;
        }
        if (!a.culled)
            continue;
        const hipError_t q = hipEventQuery(S->ev_cull[a.slot]);
        if (q == hipSuccess) {
            ready.push_back(i);
        } else if (q != hipErrorNotReady) {
            // the build or cull on the slot stream failed: nothing more is
            // enqueued for this request, and it finishes with the error once
            // its slot stream has drained
            a.status = hip_fail(q, "request build / cull");
            a.culled = false;
            a.final = true;
            hipStreamSynchronize(S->ss[a.slot]);
            any = true;
        }
    }
    while (!ready.empty() && (int)S->inflight.size() < kInflightBatches) {
        // one batch: up to kMaxJobs requests of the first ready request's leaf size
        const int leaf = S->active[ready[0]].job.rq.leaf;
        std::vector<size_t> batch, rest;
        for (size_t i : ready)
            (S->active[i].job.rq.leaf == leaf && (int)batch.size() < kMaxJobs ? batch : rest)
                .push_back(i);
        ready.swap(rest);
        // jobs of each kernel kind (FP32 or BF16 split on 2 x 2 or 4 x 4
        // blocks, with FP32 or compensated HIGH products; FP16 split) go to
        // one launch
        constexpr int kKinds = 7;
        constexpr GemmKind kinds[kKinds] = {GemmKind::Fp32,      GemmKind::Split,
                                            GemmKind::SplitF16,  GemmKind::SplitWide,
                                            GemmKind::Wide32,    GemmKind::SplitX3,
                                            GemmKind::SplitWideX3};
        GemmJobs tabs[kKinds] = {};
        hipError_t e = hipSuccess;
        for (size_t i : batch) {
            Active &a = S->active[i];
            const GemmKind kind = plan_kind(a.plan);
            int slot = 0;
            while (slot + 1 < kKinds && kinds[slot] != kind)
                ++slot;
            GemmJobs &tab = tabs[slot];
            GemmJob &j = tab.job[tab.njobs++];
            plan_jobs(a.plan, a.job.rq.C, j);
            // a chain step before the last: the next tree reads only the
            // leaves this product reaches, so blocks without products need
            // not write their zeros
            j.skip_empty = a.step + 1 < a.steps ? 1 : 0;
            j.block0 = tab.nblocks;
            tab.nblocks += j.nblocks;
        }
        for (int k = 0; k < kKinds && e == hipSuccess; ++k)
            if (tabs[k].njobs > 0)
                e = launch_gemm_jobs(leaf, kinds[k], tabs[k], S->gemm);
        hipEvent_t bev = S->spare.back();
        if (e == hipSuccess)
            e = hipEventRecord(bev, S->gemm);
        if (e == hipSuccess) {
            S->spare.pop_back();
            S->inflight.push_back(bev);
            std::lock_guard<std::mutex> lock(S->mu);
            S->st.launches += 1;
            S->st.launched_products += (int64_t)batch.size();
            S->st.max_batch = std::max<int64_t>(S->st.max_batch, (int64_t)batch.size());
        }
        for (size_t i : batch) {
            Active &a = S->active[i];
            hipError_t f = e == hipSuccess ? hipEventRecord(S->ev_done[a.slot], S->gemm) : e;
            if (f != hipSuccess) {
                // nothing further is enqueued for this request; its resources
                // are released once the GEMM stream has drained
                a.status = hip_fail(f, "batched leaf GEMM");
                a.culled = false;
                a.phase = kIdle;
                a.final = true;
                hipStreamSynchronize(S->gemm);
                continue;
            }
            advance(S, a);
        }
        any = true;
    }
    return any;
}

Active *find_active(spamm_server *S, uint64_t ticket)
{
    for (Active &a : S->active)
        if (a.job.ticket == ticket)
            return &a;
    return nullptr;
}

// One round on R's prep stream for the requests S->active[pick[..]] (at most
// kMaxRound, all in phase kPrep).
void launch_round(spamm_server *S, Round &R, const std::vector<size_t> &pick)
{
    hipStream_t ps = R.s;
    bool chain = false;
    for (size_t i : pick)
        chain |= S->active[i].step > 0;
    // a chain step reads C and overwrites its previous trees: after every
    // GEMM enqueued so far (the GEMM stream runs in order)
    if (chain && !S->inflight.empty())
        hipStreamWaitEvent(ps, S->inflight.back(), 0);
    std::vector<RoundTree> trees;
    std::vector<const spamm_plan *> plans;
    std::vector<size_t> in;
    std::vector<spamm_plan *> old_plans;
    std::vector<spamm_tree *> old_trees;
    for (size_t i : pick) {
        Active &a = S->active[i];
        const spamm_request &r = a.job.rq;
        const uint32_t flags = tree_flags_for(r.precision);
        // arena: [tree of A or X_s][tree of B, step 0 only][plan][keep flags, chains]
        char *base = (char *)S->arena[a.slot];
        const size_t tb = tree_device_bytes(r.n, r.leaf, flags);
        spamm_plan *prev = a.step > 0 ? a.plan : nullptr;
        old_plans.push_back(a.plan);
        old_trees.push_back(a.tA);
        if (a.tB != a.tA)
            old_trees.push_back(a.tB);
        a.plan = nullptr;
        a.tA = a.tB = nullptr;
        int rc;
        if (a.step > 0) {
            uint32_t *keep = (uint32_t *)(base + tb + plan_device_bytes(prev->depth, a.split));
            rc = tree_prepare(r.n, r.leaf, flags, base, keep, ps, &a.tA);
            a.tB = a.tA;
        } else {
            rc = tree_prepare(r.n, r.leaf, flags, base, nullptr, ps, &a.tA);
            if (rc == SPAMM_OK && a.distinctB)
                rc = tree_prepare(r.n, r.leaf, flags, base + tb, nullptr, ps, &a.tB);
            else
                a.tB = a.tA;
        }
        spamm_opts o{};
        o.tau = r.tau;
        o.precision = r.precision;
        o.low_tol = a.split ? r.low_tol : 0.0;
        o.low_rel = a.split ? r.low_rel : 0.0;
        if (rc == SPAMM_OK)
            rc = plan_prepare(a.tA, a.tB, &o, ps, base + (a.distinctB ? 2 : 1) * tb, &a.plan);
        if (rc != SPAMM_OK) {
            a.status = rc;
            a.phase = kIdle;
            a.final = true;
            continue;
        }
        const double T2 = r.tau * r.tau;
        trees.push_back({a.tA, a.step == 0 ? r.A : r.C, prev, T2, a.tB});
        if (a.tB != a.tA)
            trees.push_back({a.tB, r.B, nullptr, T2, a.tA});
        plans.push_back(a.plan);
        in.push_back(i);
    }
    hipError_t e = hipSuccess;
    if (!in.empty()) {
        e = launch_build_round(trees.data(), (int)trees.size(), ps);
        if (e == hipSuccess)
            e = launch_cull_round(plans.data(), (int)plans.size(), R.dout, ps);
        if (e == hipSuccess)
            e = hipMemcpyAsync(R.hout, R.dout, sizeof(StepOut) * in.size(), hipMemcpyDeviceToHost,
                               ps);
        if (e == hipSuccess)
            e = hipEventRecord(R.ev, ps);
    }
    // the previous steps' handles (their buffers live in the slot arenas and
    // were read by the work just enqueued)
    for (spamm_plan *p : old_plans)
        spamm_plan_free(p);
    for (spamm_tree *t : old_trees)
        spamm_tree_free(t);
    if (e != hipSuccess) {
        const int rc = hip_fail(e, "round build / cull");
        hipStreamSynchronize(ps);
        for (size_t i : in) {
            S->active[i].status = rc;
            S->active[i].phase = kIdle;
            S->active[i].final = true;
        }
        return;
    }
    if (in.empty())
        return;
    R.busy = true;
    R.tickets.clear();
    {
        std::lock_guard<std::mutex> lock(S->mu);
        S->st.rounds += 1;
        S->st.round_steps += (int64_t)in.size();
    }
    for (size_t i : in) {
        R.tickets.push_back(S->active[i].job.ticket);
        S->active[i].phase = kCulling;
    }
}

// Rounds for every request waiting in phase kPrep, while round records are
// free.  Returns true if anything was launched.
bool form_rounds(spamm_server *S)
{
    bool any = false;
    for (Round &R : S->rounds) {
        if (R.busy)
            continue;
        std::vector<size_t> pick;
        for (size_t i = 0; i < S->active.size() && (int)pick.size() < kMaxRound; ++i)
            if (S->active[i].batched && S->active[i].phase == kPrep)
                pick.push_back(i);
        if (pick.empty())
            break;
        launch_round(S, R, pick);
        any = true;
    }
    return any;
}

// Completed rounds: their requests' counts and roots to the slots' step
// records, and on to the GEMM batches.
bool poll_rounds(spamm_server *S)
{
    bool any = false;
    for (Round &R : S->rounds) {
        if (!R.busy)
            continue;
        const hipError_t q = hipEventQuery(R.ev);
        if (q == hipErrorNotReady)
            continue;
        const int rc = q == hipSuccess ? SPAMM_OK : hip_fail(q, "round build / cull");
        if (q != hipSuccess)
            hipStreamSynchronize(R.s);
        for (size_t j = 0; j < R.tickets.size(); ++j) {
            Active *a = find_active(S, R.tickets[j]);
            if (a == nullptr)
                continue;
            if (rc == SPAMM_OK) {
                memcpy(&S->pin[a->slot].step[a->step], R.hout + 5 * j, sizeof(StepOut));
                a->phase = kReady;
            } else {
                a->status = rc;
                a->phase = kIdle;
                a->final = true;
            }
        }
        R.busy = false;
        R.tickets.clear();
        any = true;
    }
    return any;
}

// Post the result of a request whose last GEMM has passed (or that failed).
void finish(spamm_server *S, Active &a)
{
    release_step(S, a);
    const Pinned &P = S->pin[a.slot];
    spamm_result res;
    memset(&res, 0, sizeof res);
    res.status = a.status;
    res.steps = a.step + 1;
    if (res.status == SPAMM_OK) {
        for (int s = 0; s <= a.step; ++s) {
            const bool finite = isfinite(P.step[s].root[0]) && isfinite(P.step[s].root[1]);
            if (!finite) {
                res.status = SPAMM_E_NONFINITE;
                break;
            }
            if (a.job.rq.precision == SPAMM_PREC_SPLIT_BF16X3 &&
                (P.step[s].root[0] >= kX3MaxRoot2 || P.step[s].root[1] >= kX3MaxRoot2)) {
                res.status = SPAMM_E_RANGE;
                break;
            }
            res.tasks += (int64_t)(P.step[s].K[0] + P.step[s].K[1]);
            res.tasks_low += (int64_t)P.step[s].K[1];
        }
    }
    const double b = a.job.rq.leaf;
    res.flops = 2.0 * b * b * b * (double)res.tasks;
    const double t = now_us();
    res.queue_ms = (a.t_admit - a.job.t_submit) * 1e-3;
    res.latency_ms = (t - a.job.t_submit) * 1e-3;
    std::lock_guard<std::mutex> lock(S->mu);
    S->done[a.job.ticket] = res;
    S->st.completed += 1;
    S->live.erase(a.job.ticket);
    S->busy[a.slot] = false;
}

// Pick a free slot whose arena can hold `need` bytes, growing one (and
// releasing idle arenas) within the budget.  Called with S->mu held; -1 when
// the request has to wait.  Returns a HIP error through *err.  A new arena
// is allocated in the slot stream's order; for a batched request, whose
// rounds run on the prep streams, that stream is then synchronized (arenas
// grow rarely: the steady state reuses them).
int claim_slot(spamm_server *S, size_t need, bool batched, hipError_t *err)
{
    int fit = -1, big = -1;
    for (int i = 0; i < S->nslots; ++i) {
        if (S->busy[i])
            continue;
        if (S->cap[i] >= need && (fit < 0 || S->cap[i] < S->cap[fit]))
            fit = i;
        if (big < 0 || S->cap[i] > S->cap[big])
            big = i;
    }
    if (fit >= 0)
        return fit;
    if (big < 0)
        return -1;
    // release idle arenas (smallest first) until the grown arena fits
    while (S->used - S->cap[big] + need > S->budget) {
        int v = -1;
        for (int i = 0; i < S->nslots; ++i)
            if (!S->busy[i] && i != big && S->cap[i] > 0 && (v < 0 || S->cap[i] < S->cap[v]))
                v = i;
        if (v < 0)
            return -1;
        hipFreeAsync(S->arena[v], S->ss[v]);
        S->used -= S->cap[v];
        S->arena[v] = nullptr;
        S->cap[v] = 0;
    }
    if (S->arena[big] != nullptr) {
        hipFreeAsync(S->arena[big], S->ss[big]);
        S->used -= S->cap[big];
        S->arena[big] = nullptr;
        S->cap[big] = 0;
    }
    hipError_t e = dev_alloc_async(S->device, &S->arena[big], need, S->ss[big]);
    if (e == hipSuccess && batched)
        e = hipStreamSynchronize(S->ss[big]);
    if (e != hipSuccess) {
        S->arena[big] = nullptr;
        *err = e;
        return -1;
    }
    S->cap[big] = need;
    S->used += need;
    return big;
}

void scheduler(spamm_server *S)
{
    hipSetDevice(S->device);
    // short sleeps between polls stay short (the default slack is 50 us)
    prctl(PR_SET_TIMERSLACK, 2000UL, 0UL, 0UL, 0UL);
    int idle = 0;
    for (;;) {
        std::vector<Job> admitted;
        std::vector<int> slots;
        {
            std::unique_lock<std::mutex> lock(S->mu);
            if (S->active.empty() && S->queue.empty()) {
                if (S->stopping)
                    break;
                S->cv.wait(lock, [S] { return S->stopping || !S->queue.empty(); });
                continue;
            }
            while (!S->queue.empty()) {
                hipError_t err = hipSuccess;
                const int slot = claim_slot(S, S->queue.front().bytes, S->queue.front().batched,
                                            &err);
                if (slot < 0) {
                    if (err == hipSuccess)
                        break;
                    // the arena could not be allocated: fail this request
                    Job j = S->queue.front();
                    S->queue.pop_front();
                    spamm_result res;
                    memset(&res, 0, sizeof res);
                    res.status = hip_fail(err, "slot arena");
                    res.latency_ms = (now_us() - j.t_submit) * 1e-3;
                    S->done[j.ticket] = res;
                    S->live.erase(j.ticket);
                    S->st.completed += 1;
                    continue;
                }
                S->busy[slot] = true;
                S->st.admitted += 1;
                S->st.peak_used = std::max<uint64_t>(S->st.peak_used, S->used);
                int64_t nb = 0;
                for (int k = 0; k < S->nslots; ++k)
                    nb += S->busy[k] ? 1 : 0;
                S->st.peak_active = std::max<int64_t>(S->st.peak_active, nb);
                admitted.push_back(S->queue.front());
                slots.push_back(slot);
                S->queue.pop_front();
            }
        }
        bool progress = !admitted.empty();
        for (size_t i = 0; i < admitted.size(); ++i) {
            Active a;
            a.job = admitted[i];
            a.slot = slots[i];
            a.steps = std::max(1, a.job.rq.chain_len);
            a.split = a.job.rq.precision != SPAMM_PREC_FP32;
            a.distinctB = a.job.rq.B != nullptr && a.job.rq.B != a.job.rq.A;
            a.batched = a.job.batched;
            a.t_admit = now_us();
            if (a.batched) {
                a.phase = kPrep;          // the next round builds and culls it
            } else {
                int rc = start_step(S, a, nullptr);
                if (rc) {
                    a.status = rc;
                    a.culled = false;
                    a.final = true;
                }
            }
            S->active.push_back(a);
        }
        progress |= poll_rounds(S);
        progress |= launch_batches(S);
        progress |= form_rounds(S);
        for (size_t i = 0; i < S->active.size();) {
            Active &a = S->active[i];
            bool over = false;
            if (a.final) {
                hipError_t q = hipEventQuery(S->ev_done[a.slot]);
                if (q == hipSuccess) {
                    over = true;
                } else if (q != hipErrorNotReady) {
                    a.status = hip_fail(q, "request completion");
                    hipStreamSynchronize(S->gemm);
                    over = true;
                }
            }
            if (over) {
                finish(S, a);
                S->active.erase(S->active.begin() + (std::ptrdiff_t)i);
                progress = true;
            } else {
                ++i;
            }
        }
        // nothing moved: yield a few passes, then poll every ~10 us (the
        // GPU work being waited for takes tens of microseconds or more)
        if (progress) {
            idle = 0;
        } else if (++idle < kSpinPasses) {
            std::this_thread::yield();
        } else {
            std::this_thread::sleep_for(std::chrono::microseconds(8));
        }
    }
}

void release_server(spamm_server *S)
{
    if (S->gemm)
        hipStreamSynchronize(S->gemm);
    for (Round &R : S->rounds)
        if (R.s)
            hipStreamSynchronize(R.s);
    for (int i = 0; i < S->nslots; ++i)
        if (S->ss[i])
            hipStreamSynchronize(S->ss[i]);
    for (hipEvent_t e : S->inflight)
        hipEventDestroy(e);
    for (hipEvent_t e : S->spare)
        hipEventDestroy(e);
    for (int i = 0; i < kMaxSlots; ++i) {
        if (S->arena[i])
            hipFree(S->arena[i]);
        if (S->ev_cull[i])
            hipEventDestroy(S->ev_cull[i]);
        if (S->ev_done[i])
            hipEventDestroy(S->ev_done[i]);
        if (S->ss[i])
            hipStreamDestroy(S->ss[i]);
    }
    if (S->gemm)
        hipStreamDestroy(S->gemm);
    for (Round &R : S->rounds) {
        if (R.ev)
            hipEventDestroy(R.ev);
        if (R.s)
            hipStreamDestroy(R.s);
    }
    if (S->rounds[0].dout)
        hipFree(S->rounds[0].dout);
    if (S->rounds[0].hout)
        hipHostFree(S->rounds[0].hout);
    if (S->pin)
        hipHostFree(S->pin);
    delete S;
}

}  // namespace

extern "C" {

int spamm_request_footprint(const spamm_request *req, size_t *bytes)
{
    if (bytes == nullptr)
        return fail(SPAMM_E_INVAL, "bytes is NULL");
    return check_request(req, bytes);
}

int spamm_server_create(size_t hbm_budget, int32_t max_slots, spamm_server **out)
{
    if (out == nullptr)
        return fail(SPAMM_E_INVAL, "out is NULL");
    *out = nullptr;
    if (hbm_budget == 0)
        return fail(SPAMM_E_INVAL, "hbm_budget = 0");
    if (max_slots < 1 || max_slots > kMaxSlots)
        return fail(SPAMM_E_INVAL, "max_slots = %d outside 1..%d", max_slots, kMaxSlots);
    int dev, rc;
    if ((rc = prepare_device(&dev)))
        return rc;
    spamm_server *S = new (std::nothrow) spamm_server();
    if (S == nullptr)
        return fail(SPAMM_E_NOMEM, "host allocation failed");
    S->device = dev;
    S->budget = hbm_budget;
    S->nslots = max_slots;
    hipError_t e = hipStreamCreateWithFlags(&S->gemm, hipStreamNonBlocking);
    // round readbacks: 5 words per plan, kMaxRound plans per round
    const size_t rwords = 5 * (size_t)kMaxRound;
    uint64_t *dout = nullptr, *hout = nullptr;
    if (e == hipSuccess)
        e = hipMalloc((void **)&dout, sizeof(uint64_t) * rwords * kRounds);
    if (e == hipSuccess)
        S->rounds[0].dout = dout;
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&hout, sizeof(uint64_t) * rwords * kRounds,
                          hipHostMallocDefault);
    if (e == hipSuccess)
        S->rounds[0].hout = hout;
    for (int r = 0; r < kRounds && e == hipSuccess; ++r) {
        S->rounds[r].dout = dout + rwords * r;
        S->rounds[r].hout = hout + rwords * r;
        e = hipEventCreateWithFlags(&S->rounds[r].ev, hipEventDisableTiming);
        if (e == hipSuccess)
            e = hipStreamCreateWithFlags(&S->rounds[r].s, hipStreamNonBlocking);
    }
    for (int i = 0; i < max_slots && e == hipSuccess; ++i) {
        e = hipStreamCreateWithFlags(&S->ss[i], hipStreamNonBlocking);
        if (e == hipSuccess)
            e = hipEventCreateWithFlags(&S->ev_cull[i], hipEventDisableTiming);
        if (e == hipSuccess)
            e = hipEventCreateWithFlags(&S->ev_done[i], hipEventDisableTiming);
    }
    for (int i = 0; i < kInflightBatches && e == hipSuccess; ++i) {
        hipEvent_t ev = nullptr;
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess)
            S->spare.push_back(ev);
    }
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&S->pin, sizeof(Pinned) * (size_t)max_slots, hipHostMallocDefault);
    if (e != hipSuccess) {
        rc = hip_fail(e, "spamm_server_create");
        release_server(S);
        return rc;
    }
    memset(S->pin, 0, sizeof(Pinned) * (size_t)max_slots);
    try {
        S->t_start = now_us();
        S->worker = std::thread(scheduler, S);
    } catch (...) {
        release_server(S);
        return fail(SPAMM_E_HIP, "could not start the scheduler thread");
    }
    *out = S;
    return SPAMM_OK;
}

int spamm_submit(spamm_server *S, const spamm_request *req, uint64_t *ticket)
{
    if (S == nullptr || ticket == nullptr)
        return fail(SPAMM_E_INVAL, "NULL argument");
    size_t bytes = 0;
    bool batched = false;
    int rc = check_request(req, &bytes, &batched);
    if (rc)
        return rc;
    if (bytes > S->budget)
        return fail(SPAMM_E_NOMEM, "request needs %zu bytes, the server's budget is %zu", bytes,
                    S->budget);
    Job j;
    j.rq = *req;
    j.bytes = bytes;
    j.t_submit = now_us();
    j.batched = batched;
    {
        std::lock_guard<std::mutex> lock(S->mu);
        if (S->stopping)
            return fail(SPAMM_E_INVAL, "server is shutting down");
        if (S->queue.size() >= kMaxQueue)
            return fail(SPAMM_E_BUSY, "%zu requests queued", S->queue.size());
        j.ticket = S->next_ticket++;
        S->queue.push_back(j);
        S->live.insert(j.ticket);
        *ticket = j.ticket;
    }
    S->cv.notify_one();
    return SPAMM_OK;
}

int spamm_poll(spamm_server *S, uint64_t ticket, spamm_result *out)
{
    if (S == nullptr)
        return fail(SPAMM_E_INVAL, "server is NULL");
    std::lock_guard<std::mutex> lock(S->mu);
    auto it = S->done.find(ticket);
    if (it != S->done.end()) {
        if (out)
            *out = it->second;
        S->done.erase(it);
        return SPAMM_OK;
    }
    if (S->live.count(ticket))
        return SPAMM_PENDING;
    return fail(SPAMM_E_INVAL, "unknown ticket %llu", (unsigned long long)ticket);
}

int spamm_server_info(spamm_server *S, spamm_server_stats *out)
{
    if (S == nullptr || out == nullptr)
        return fail(SPAMM_E_INVAL, "NULL argument");
    std::lock_guard<std::mutex> lock(S->mu);
    *out = S->st;
    out->queued = (int64_t)S->queue.size();
    out->used = S->used;
    out->budget = S->budget;
    // the scheduler thread's own CPU clock: how busy the host side is
    out->sched_cpu_ms = 0.0;
    out->sched_wall_ms = (now_us() - S->t_start) * 1e-3;
    clockid_t cid;
    timespec ts;
    if (S->worker.joinable() &&
        pthread_getcpuclockid(S->worker.native_handle(), &cid) == 0 &&
        clock_gettime(cid, &ts) == 0)
        out->sched_cpu_ms = ts.tv_sec * 1e3 + ts.tv_nsec * 1e-6;
    return SPAMM_OK;
}

int spamm_server_destroy(spamm_server *S)
{
    if (S == nullptr)
        return SPAMM_OK;
    {
        std::lock_guard<std::mutex> lock(S->mu);
        S->stopping = true;
        for (const Job &j : S->queue)
            S->live.erase(j.ticket);
        S->queue.clear();
    }
    S->cv.notify_all();
    if (S->worker.joinable())
        S->worker.join();
    const int dev = S->device;
    int dev0 = -1;
    hipGetDevice(&dev0);
    if (dev0 != dev)
        hipSetDevice(dev);
    release_server(S);
    if (dev0 >= 0 && dev0 != dev)
        hipSetDevice(dev0);
    return SPAMM_OK;
}

}  // extern "C"
