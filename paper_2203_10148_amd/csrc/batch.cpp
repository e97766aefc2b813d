// Batched and served PiTSBiCG solves: many instances of Algorithm 1 (Sec. 3)
// advanced together on one GPU.
//
// Every instance runs the same control flow as pit_solve (the host decides
// after each reduction, with the same scalars and the same branches), split
// into phases that end at a reduction:
//   INIT      R = G^{-1} B, shadow R = P = R, <R,Rt>, <R,R>
//   A         P = R + beta(P - omega D) (deferred), D = G^{-1}F P, <D,Rt>
//   A_RESTART shadow R = P = R, <R,R>          (breakdown <D,Rt> = 0, then A again)
//   B         S = R - alpha D, K = G^{-1}F S, <K,S>, <K,K>, <S,S>
//   C         X += alpha P + omega S, R = S - omega K, <R,Rt>, <R,R>
//   W0        X += alpha P, R = S, shadow R = P = R, <R,R>   (omega = 0 restart)
//   FINAL     X out of the working layout
// An instance whose phase has completed is "ready"; every scheduling round
// gathers the ready 1D instances and issues their phases together on one of
// four streams: one launch per line shape for the fine applies (every slice of
// every listed instance), one per shape for the coarse sweeps (one workgroup
// per instance, so the sequential sweeps of different instances run on
// different CUs at the same time), one for the vector updates and one pair
// for the inner products.  A 2D instance runs its phases with its own
// launches on a stream of its own.  The device arithmetic per instance is the
// single-instance kernels' (shared device functions), so results do not
// depend on the company an instance keeps.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <functional>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "arena.hpp"
#include "ctx.hpp"

static_assert(pit::kArenaAlign == pit::kAlign, "arena granules keep workspaces aligned");

using namespace pit;

namespace {

constexpr int kLanes = 4;

enum Phase { PH_INIT, PH_A, PH_A_RESTART, PH_B, PH_C, PH_W0, PH_FINAL, PH_DONE };

struct Inst {
    pit_ctx *ctx = nullptr;
    int slot = -1;
    pit_solve_opts o{};
    const double *u0 = nullptr;
    double *Xout = nullptr;
    Phase ph = PH_INIT;
    bool in_flight = false;
    int red_pos = -1;  // position of this instance's reduction in its lane's results
    // Algorithm 1 state (names as in pit_solve)
    int k = 0, restarts = 0, matvecs = 0, status = PIT_ENOCONV, best_at = 0, n_fine = 0, n_coarse = 0;
    double rho = 0, nrm = 0, scale = 1, best = 0, alpha = 0, omega = 0, beta = 0;
    bool second_try = false;
    // deferred vector operations, issued at the head of the next phase in this order
    bool pend_p = false;        // P = R + beta (P - omega D)
    bool pend_xap = false;      // X += alpha P
    bool pend_rs = false;       // R = S
    bool pend_restart = false;  // shadow R = R, P = R
    std::vector<double> hist;
    // bookkeeping of the owner (batch call or server)
    double t_submit = 0, t_admit = 0, t_done = 0;
    uint64_t ticket = 0;
    size_t ws_off = 0, ws_bytes = 0;
    int hip_error = 0;
    int index = 0;
    double t_ready = 0, t_issue = 0;  // current phase, engine clock (for the trace)
    int lane = -1, group = 0;

    bool dim2() const { return ctx->dim2(); }
    long n() const { return ctx->ntc(); }
    double *v(int q) const { return ctx->vec(q); }
};

// Pinned host staging of one round's launch arguments, copied to the lane's
// device buffer with one transfer before the launches that read it.
struct Blob {
    char *h = nullptr;
    char *d = nullptr;
    size_t cap = 0, used = 0;
    template <class T>
    T *put(const T *src, size_t n)
    {
        used = (used + 15) & ~size_t(15);
        const size_t b = n * sizeof(T);
        if (used + b > cap) return nullptr;
        std::memcpy(h + used, src, b);
        T *dev = reinterpret_cast<T *>(d + used);
        used += b;
        return dev;
    }
};

struct Lane {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    Blob blob;
    RedOut *d_red = nullptr;
    RedOut *h_red = nullptr;
    std::vector<Inst *> members;
    bool busy = false;
    bool kind2d = false;
    uint64_t seq = 0;
};

struct ClassKey {
    int NT, C, a, b;
    bool operator<(const ClassKey &o) const
    {
        return std::tie(NT, C, a, b) < std::tie(o.NT, o.C, o.a, o.b);
    }
};

}  // namespace

namespace pit {

class Engine {
  public:
    explicit Engine(int max_slots) : max_(max_slots), t0_(std::chrono::steady_clock::now())
    {
        // PIT_BATCH_TRACE=<file>: one CSV line per completed phase (times in
        // ms on the engine's clock: ready, issued, seen complete by the host)
        if (const char *f = std::getenv("PIT_BATCH_TRACE")) {
            trace_ = std::fopen(f, "w");
            if (trace_) std::fprintf(trace_, "index,M,N,m,phase,lane,group,t_ready,t_issue,t_done\n");
        }
    }
    ~Engine()
    {
        release();
        if (trace_) std::fclose(trace_);
    }

    static size_t args_cap(int max_slots) { return 65536 + (size_t)max_slots * 640; }
    static size_t bytes(int max_slots)
    {
        return align_up((size_t)max_slots * sizeof(Inst1d)) +
               kLanes * (align_up(args_cap(max_slots)) + align_up((size_t)max_slots * sizeof(RedOut)));
    }

    int bind(char *dev, size_t nbytes)
    {
        if (nbytes < bytes(max_)) return PIT_ENOMEM;
        release();
        char *p = dev;
        d_inst_ = reinterpret_cast<Inst1d *>(p);
        p += align_up((size_t)max_ * sizeof(Inst1d));
        for (auto &L : lanes_) {
            PIT_HIP(hipStreamCreateWithFlags(&L.st, hipStreamNonBlocking));
            PIT_HIP(hipEventCreateWithFlags(&L.ev, hipEventDisableTiming));
            L.blob.cap = args_cap(max_);
            L.blob.d = p;
            p += align_up(L.blob.cap);
            PIT_HIP(hipHostMalloc(reinterpret_cast<void **>(&L.blob.h), L.blob.cap, hipHostMallocDefault));
            L.d_red = reinterpret_cast<RedOut *>(p);
            p += align_up((size_t)max_ * sizeof(RedOut));
            PIT_HIP(hipHostMalloc(reinterpret_cast<void **>(&L.h_red), (size_t)max_ * sizeof(RedOut),
                                  hipHostMallocDefault));
        }
        free_.clear();
        for (int i = max_ - 1; i >= 0; --i) free_.push_back(i);
        h_inst_.assign(max_, Inst1d{});
        bound_ = true;
        return PIT_OK;
    }

    bool bound() const { return bound_; }
    bool has_slot() const { return !free_.empty(); }
    bool idle() const { return active_.empty(); }
    int running() const { return (int)active_.size(); }

    // Make every lane wait for the work queued so far on `user`.
    int after(hipStream_t user)
    {
        hipEvent_t e;
        PIT_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        hipError_t r = hipEventRecord(e, user);
        for (auto &L : lanes_)
            if (r == hipSuccess) r = hipStreamWaitEvent(L.st, e, 0);
        (void)hipEventDestroy(e);
        PIT_HIP(r);
        return PIT_OK;
    }

    // Give a bound context's solve a slot; it starts at the next round.
    int admit(Inst *in)
    {
        if (free_.empty()) return PIT_ENOMEM;
        in->slot = free_.back();
        free_.pop_back();
        in->ph = PH_INIT;
        in->in_flight = false;
        in->t_ready = now();
        if (!in->dim2()) {
            const pit_ctx *c = in->ctx;
            Inst1d d{};
            d.tf = c->tab(c->lf, c->off_tf);
            if (c->fine32()) d.tf32 = c->tab32(c->lf, c->off_tf32);
            d.tc = c->tab(c->lc, c->off_tc);
            d.vec = c->vec(0);
            d.part = c->part();
            d.ld = c->ld;
            d.N = c->N;
            d.M = c->npts;
            d.m = c->m;
            d.c = c->coarse.substeps;
            d.bps = c->bps;
            d.w = c->w;
            d.pd = c->pd;
            d.pa = c->pa;
            d.pr = c->pr;
            d.periodic = c->pb.bc == PIT_PERIODIC ? 1 : 0;
            h_inst_[in->slot] = d;
        }
        active_.push_back(in);
        return PIT_OK;
    }

    // One scheduling round: collect finished phases, issue the ready ones.
    // Returns PIT_OK or PIT_EHIP; `progress` tells whether anything happened.
    int round(std::vector<Inst *> &finished, bool &progress)
    {
        progress = false;
        for (auto &L : lanes_) {
            if (!L.busy) continue;
            const hipError_t q = hipEventQuery(L.ev);
            if (q == hipErrorNotReady) continue;
            PIT_HIP(q);
            complete(L, finished);
            progress = true;
        }
        // Lanes: when both kinds are running, 1D rounds and 2D instances each
        // keep half of the lanes, so neither starves the other; otherwise
        // one kind may use all of them.
        bool has1 = false, has2 = false;
        for (const Inst *in : active_) (in->dim2() ? has2 : has1) = true;
        int busy1 = 0, busy2 = 0;
        for (const auto &L : lanes_)
            if (L.busy) (L.kind2d ? busy2 : busy1)++;
        const int cap1 = has2 ? kLanes / 2 : kLanes, cap2 = has1 ? kLanes / 2 : kLanes;
        // 1D instances: the ready ones in groups of similar expected phase
        // length (powers of two), so a short phase does not wait for the
        // longest sweep of the round; groups are merged down to the free lanes.
        std::map<int, std::vector<Inst *>, std::greater<int>> buckets;
        for (Inst *in : active_)
            if (!in->in_flight && !in->dim2()) buckets[(int)std::floor(std::log2(phase_us(in)))].push_back(in);
        std::vector<std::vector<Inst *>> groups;
        for (auto &kv : buckets) groups.push_back(std::move(kv.second));
        int free1 = 0;
        for (const auto &L : lanes_)
            if (!L.busy) free1++;
        free1 = std::min(free1, cap1 - busy1);
        while ((int)groups.size() > std::max(free1, 1)) {
            auto last = std::move(groups.back());
            groups.pop_back();
            groups.back().insert(groups.back().end(), last.begin(), last.end());
        }
        // a group larger than the cap gives its longest-phase members their own
        // smaller group when a stream is free for it
        const int gmax = group_cap();
        for (size_t gi = 0; gi < groups.size() && (int)groups.size() < free1; ++gi) {
            auto &gr = groups[gi];
            if ((int)gr.size() <= gmax) continue;
            std::stable_sort(gr.begin(), gr.end(), [](const Inst *a, const Inst *b) { return phase_us(a) > phase_us(b); });
            std::vector<Inst *> head(gr.begin(), gr.begin() + gmax);
            gr.erase(gr.begin(), gr.begin() + gmax);
            groups.insert(groups.begin() + gi, std::move(head));
        }
        if (free1 > 0) {
            for (auto &g : groups) {
                Lane *L = free_lane();
                if (!L) break;
                int rc = issue_batch(*L, g);
                if (rc) return rc;
                start(*L, g, false);
                progress = true;
            }
        }
        // 2D instances: one lane each
        for (Inst *in : active_) {
            if (in->in_flight || !in->dim2()) continue;
            if (busy2 >= cap2) break;
            Lane *L = free_lane();
            if (!L) break;
            std::vector<Inst *> one{in};
            int rc = issue_single(*L, in);
            if (rc) return rc;
            start(*L, one, true);
            busy2++;
            progress = true;
        }
        return PIT_OK;
    }

    bool any_busy() const
    {
        for (const auto &L : lanes_)
            if (L.busy) return true;
        return false;
    }

    // After a HIP failure: finish every active instance with PIT_EHIP once the
    // lanes are drained.
    void fail_all(int hip_code, std::vector<Inst *> &finished)
    {
        for (auto &L : lanes_) {  // drain everything issued, also a round cut short by the failure
            (void)hipStreamSynchronize(L.st);
            L.busy = false;
            L.members.clear();
        }
        for (Inst *in : active_) {
            in->status = PIT_EHIP;
            in->hip_error = hip_code;
            in->ph = PH_DONE;
            free_.push_back(in->slot);
            finished.push_back(in);
        }
        active_.clear();
    }

  private:
    int max_;
    bool bound_ = false;
    Inst1d *d_inst_ = nullptr;
    std::vector<Inst1d> h_inst_;
    std::vector<int> free_;
    std::vector<Inst *> active_;
    Lane lanes_[kLanes];
    uint64_t seq_ = 0;
    std::chrono::steady_clock::time_point t0_;
    FILE *trace_ = nullptr;

    double now() const
    {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0_).count();
    }

    void release()
    {
        for (auto &L : lanes_) {
            if (L.st) {
                (void)hipStreamSynchronize(L.st);
                (void)hipStreamDestroy(L.st);
            }
            if (L.ev) (void)hipEventDestroy(L.ev);
            if (L.blob.h) (void)hipHostFree(L.blob.h);
            if (L.h_red) (void)hipHostFree(L.h_red);
            L = Lane{};
        }
        bound_ = false;
    }

    // Instances per scheduling round before a group is split (PIT_BATCH_GROUP_MAX).
    static int group_cap()
    {
        // default 4: on the 64-instance batch, caps of 4 / 8 / 16 / none gave
        // makespans of 360 / 373 / 380 / 400 ms
        const char *e = std::getenv("PIT_BATCH_GROUP_MAX");
        const int v = e ? std::atoi(e) : 4;
        return v > 0 ? v : 1 << 30;
    }

    // Expected length of a 1D instance's next phase (microseconds, rough):
    // a fine apply is m chained line solves, a coarse sweep (N-1)c of them,
    // a line solve about (0.5 + M/8192) us; the other phases are short.
    static double phase_us(const Inst *in)
    {
        const pit_ctx *c = in->ctx;
        const double solve = 0.5 + c->npts / 8192.0;
        const double sweep = (double)(c->N - 1) * c->coarse.substeps * solve;
        switch (in->ph) {
        case PH_INIT: return 2.0 + sweep;
        case PH_A:
        case PH_B: return 2.0 + c->m * solve + sweep;
        default: return 2.0;
        }
    }

    Lane *free_lane()
    {
        for (auto &L : lanes_)
            if (!L.busy) return &L;
        return nullptr;
    }

    void start(Lane &L, const std::vector<Inst *> &members, bool kind2d)
    {
        L.members = members;
        L.busy = true;
        L.kind2d = kind2d;
        L.seq = ++seq_;
        const double t = trace_ ? now() : 0.0;
        for (Inst *in : members) {
            in->in_flight = true;
            in->t_issue = t;
            in->lane = (int)(&L - lanes_);
            in->group = (int)members.size();
        }
    }

    // -------------------------------------------------------------------
    // host side of Algorithm 1, per instance (mirrors pit_solve)
    // -------------------------------------------------------------------
    void to_final(Inst *in, int status)
    {
        in->status = status;
        in->ph = PH_FINAL;
    }

    // the stopping test and the loop guards, at the head of an iteration
    void test(Inst *in)
    {
        const pit_solve_opts &o = in->o;
        in->hist.push_back(in->nrm);
        if (!std::isfinite(in->nrm)) return to_final(in, PIT_EBREAKDOWN);
        if (!(in->nrm > o.tol * in->scale)) return to_final(in, PIT_OK);
        if (in->k >= o.max_iter) return to_final(in, PIT_ENOCONV);
        if (o.stall_window > 0) {
            if (in->nrm <= 0.5 * in->best) {
                in->best = in->nrm;
                in->best_at = in->k;
            } else if (in->k - in->best_at >= o.stall_window) {
                return to_final(in, PIT_ENOCONV);
            }
        }
        in->ph = PH_A;
        in->second_try = false;
    }

    void advance(Inst *in, const RedOut &h)
    {
        switch (in->ph) {
        case PH_INIT:
            in->rho = h.dot[0];
            in->nrm = h.nmax[1];
            in->scale = (in->o.norm_mode == PIT_REL && h.nmax[1] > 0.0) ? h.nmax[1] : 1.0;
            in->best = in->nrm;
            in->best_at = 0;
            in->k = 0;
            test(in);
            break;
        case PH_A: {
            const double dr = h.dot[0];
            if (dr == 0.0) {
                if (in->second_try) return to_final(in, PIT_EBREAKDOWN);
                in->pend_restart = true;  // restart with the current residual, redo D = G^{-1}F P
                in->ph = PH_A_RESTART;
                return;
            }
            in->alpha = in->rho / dr;
            in->ph = PH_B;
            break;
        }
        case PH_A_RESTART:
            in->rho = h.dot[0];
            in->restarts++;
            in->second_try = true;
            in->ph = PH_A;
            break;
        case PH_B: {
            const double ks = h.dot[0], kk = h.dot[1], snorm = h.nmax[2];
            if (kk == 0.0) {  // S = 0: the half step solved the system
                in->pend_xap = in->pend_rs = true;
                in->nrm = snorm;
                in->k++;
                return test(in);
            }
            in->omega = ks / kk;
            if (in->omega == 0.0) {
                in->pend_xap = in->pend_rs = in->pend_restart = true;
                in->ph = PH_W0;
                return;
            }
            in->ph = PH_C;
            break;
        }
        case PH_W0:
            in->rho = h.dot[0];
            in->nrm = h.nmax[0];
            in->restarts++;
            in->k++;
            test(in);
            break;
        case PH_C: {
            double rho_new = h.dot[0];
            in->nrm = h.nmax[1];
            in->beta = (in->alpha / in->omega) * (rho_new / in->rho);
            in->pend_p = true;                                         // new direction, issued with the next phase
            if (std::fabs(rho_new) <= in->o.restart_tol) {            // restart test with epsilon_0
                in->pend_restart = true;
                rho_new = h.dot[1];
                in->restarts++;
            }
            in->rho = rho_new;
            in->k++;
            test(in);
            break;
        }
        case PH_FINAL:
            in->ph = PH_DONE;
            break;
        default:
            break;
        }
    }

    void complete(Lane &L, std::vector<Inst *> &finished)
    {
        const double t = trace_ ? now() : 0.0;
        for (Inst *in : L.members) {
            in->in_flight = false;
            const RedOut h = in->red_pos >= 0 ? L.h_red[in->red_pos] : RedOut{};
            if (trace_)
                std::fprintf(trace_, "%d,%d,%d,%d,%d,%d,%d,%.4f,%.4f,%.4f\n", in->index, in->ctx->npts, in->ctx->N,
                             in->ctx->m, (int)in->ph, in->lane, in->group, in->t_ready, in->t_issue, t);
            in->t_ready = t;
            advance(in, h);
            if (in->ph == PH_DONE) {
                free_.push_back(in->slot);
                active_.erase(std::find(active_.begin(), active_.end(), in));
                finished.push_back(in);
            }
        }
        L.members.clear();
        L.busy = false;
    }

    // -------------------------------------------------------------------
    // issuing one round of phases
    // -------------------------------------------------------------------
    // Deferred single-vector operations (rare branches), in pit_solve's order.
    static hipError_t pre_ops(Inst *in, hipStream_t st)
    {
        hipError_t e = hipSuccess;
        const long n = in->n();
        if (in->pend_xap && e == hipSuccess) e = launch_axpby(in->v(VEC_X), in->v(VEC_X), 1.0, in->v(VEC_P), in->alpha, n, st);
        if (in->pend_rs && e == hipSuccess) e = launch_copy(in->v(VEC_R), in->v(VEC_S), n, st);
        if (in->pend_restart && e == hipSuccess) {
            e = launch_copy(in->v(VEC_RT), in->v(VEC_R), n, st);
            if (e == hipSuccess) e = launch_copy(in->v(VEC_P), in->v(VEC_R), n, st);
        }
        in->pend_xap = in->pend_rs = in->pend_restart = false;
        return e;
    }

    static void dot_pairs(Phase ph, int *q9)
    {
        // {nq, a[4], b[4]}
        std::fill(q9, q9 + kDotsAux, 0);
        auto set = [&](int nq, std::initializer_list<int> a, std::initializer_list<int> b) {
            q9[0] = nq;
            int i = 0;
            for (int x : a) q9[1 + i++] = x;
            i = 0;
            for (int x : b) q9[5 + i++] = x;
        };
        switch (ph) {
        case PH_INIT: set(2, {VEC_R, VEC_R}, {VEC_RT, VEC_R}); break;
        case PH_A: set(1, {VEC_D}, {VEC_RT}); break;
        case PH_B: set(3, {VEC_K, VEC_K, VEC_S}, {VEC_S, VEC_K, VEC_S}); break;
        case PH_C: set(2, {VEC_R, VEC_R}, {VEC_RT, VEC_R}); break;
        default: set(1, {VEC_R}, {VEC_R}); break;  // A_RESTART, W0
        }
    }

    // 2D instance: its own launches (single-instance kernels).
    int issue_single(Lane &L, Inst *in)
    {
        pit_ctx *c = in->ctx;
        hipStream_t st = L.st;
        const long n = in->n();
        const Phase ph = in->ph;
        in->red_pos = -1;
        if (ph == PH_INIT) {
            PIT_HIP(launch_fill0(in->v(VEC_S), n, st));
            PIT_HIP(launch_copy(in->v(VEC_S), in->u0, c->npts, st));
            PIT_HIP(fill_forced(c, in->v(VEC_S), st));
            PIT_HIP(launch_fill0(in->v(VEC_X), n, st));
        }
        if (ph == PH_A && in->pend_p) {
            PIT_HIP(launch_update_p(in->v(VEC_P), in->v(VEC_R), in->v(VEC_D), in->beta, in->omega, n, st));
            in->pend_p = false;
        }
        if (ph == PH_B) PIT_HIP(launch_axpby(in->v(VEC_S), in->v(VEC_R), 1.0, in->v(VEC_D), -in->alpha, n, st));
        if (ph == PH_C)
            PIT_HIP(launch_update_xr(in->v(VEC_X), in->v(VEC_R), in->v(VEC_P), in->v(VEC_S), in->v(VEC_K), in->alpha,
                                     in->omega, n, st));
        PIT_HIP(pre_ops(in, st));
        if (ph == PH_A || ph == PH_B) {
            PIT_HIP(op_apply(c, in->v(ph == PH_A ? VEC_P : VEC_S), in->v(VEC_TM), 0, 0, true, st));
            PIT_HIP(op_sweep(c, in->v(VEC_TM), in->v(ph == PH_A ? VEC_D : VEC_K), true, st));
            in->n_fine++;
            in->n_coarse++;
            in->matvecs++;
        }
        if (ph == PH_INIT) {
            PIT_HIP(op_sweep(c, in->v(VEC_S), in->v(VEC_R), true, st));
            in->n_coarse++;
            PIT_HIP(launch_copy(in->v(VEC_RT), in->v(VEC_R), n, st));
            PIT_HIP(launch_copy(in->v(VEC_P), in->v(VEC_R), n, st));
        }
        if (ph == PH_FINAL) {
            PIT_HIP(launch_copy(in->Xout, in->v(VEC_X), n, st));
        } else {
            int q9[kDotsAux];
            dot_pairs(ph, q9);
            DotPairs pr{};
            for (int q = 0; q < 4; ++q) {
                pr.a[q] = in->v(q9[1 + q]);
                pr.b[q] = in->v(q9[5 + q]);
            }
            PIT_HIP(launch_seg_dots(pr, q9[0], c->N, c->ld, c->bps, c->part(), c->w, c->red(), st));
            PIT_HIP(hipMemcpyAsync(&L.h_red[0], c->red(), sizeof(RedOut), hipMemcpyDeviceToHost, st));
            in->red_pos = 0;
        }
        PIT_HIP(hipEventRecord(L.ev, st));
        return PIT_OK;
    }

    // 1D instances: shared launches.
    int issue_batch(Lane &L, const std::vector<Inst *> &T)
    {
        hipStream_t st = L.st;
        Blob &B = L.blob;
        B.used = 0;
        std::vector<std::function<hipError_t()>> plan;
        bool overflow = false;
        auto group = [&](const std::vector<int> &list, const std::vector<int> &first, const std::vector<int> &aux,
                         const std::vector<double> &scal) {
            Group g{};
            g.inst = d_inst_;
            g.count = (int)list.size();
            g.list = B.put(list.data(), list.size());
            g.first = B.put(first.data(), first.size());
            g.aux = aux.empty() ? nullptr : B.put(aux.data(), aux.size());
            g.scal = scal.empty() ? nullptr : B.put(scal.data(), scal.size());
            g.red = L.d_red;
            if (!g.list || !g.first || (!aux.empty() && !g.aux) || (!scal.empty() && !g.scal)) overflow = true;
            return g;
        };
        // descriptors of newly admitted instances
        for (Inst *in : T) {
            in->red_pos = -1;
            if (in->ph != PH_INIT) continue;
            Inst1d *src = B.put(&h_inst_[in->slot], 1);
            if (!src) overflow = true;
            Inst1d *dst = d_inst_ + in->slot;
            pit_ctx *c = in->ctx;
            plan.push_back([=] { return hipMemcpyAsync(dst, src, sizeof(Inst1d), hipMemcpyDeviceToDevice, st); });
            plan.push_back([=] { return launch_fill0(in->v(VEC_S), in->n(), st); });
            plan.push_back([=] {
                return launch_to_chunked(in->u0, in->v(VEC_S), 1, c->npts, c->lf.sh.NT, c->lf.sh.C, st);
            });
            plan.push_back([=] { return fill_forced(c, in->v(VEC_S), st); });
            plan.push_back([=] { return launch_fill0(in->v(VEC_X), in->n(), st); });
        }
        // vector updates: deferred new direction (A), S = R - alpha D (B), X and R updates (C)
        {
            std::vector<int> list, first{0}, aux;
            std::vector<double> scal;
            for (Inst *in : T) {
                int op = -1;
                if (in->ph == PH_A && in->pend_p) op = VOP_UPDATE_P;
                if (in->ph == PH_B) op = VOP_S_AXPY;
                if (in->ph == PH_C) op = VOP_UPDATE_XR;
                if (op < 0) continue;
                in->pend_p = false;
                list.push_back(in->slot);
                first.push_back(first.back() + (int)((in->n() + kVecMultiSpan - 1) / kVecMultiSpan));
                aux.push_back(op);
                scal.insert(scal.end(), {in->alpha, in->omega, in->beta, 0.0});
            }
            if (!list.empty()) {
                const Group g = group(list, first, aux, scal);
                const int nb = first.back();
                plan.push_back([=] { return launch_vec_multi(g, nb, st); });
            }
        }
        // rare branches
        for (Inst *in : T)
            if (in->pend_xap || in->pend_rs || in->pend_restart) plan.push_back([=] { return pre_ops(in, st); });
        // fine applies (A: P, B: S) per line shape and fine form
        {
            std::map<ClassKey, std::vector<Inst *>> cls;
            for (Inst *in : T)
                if (in->ph == PH_A || in->ph == PH_B) {
                    const pit_ctx *c = in->ctx;
                    cls[{c->lf.sh.NT, c->lf.sh.C, c->fine32() ? 1 : 0, c->fine.scheme}].push_back(in);
                }
            for (auto &kv : cls) {
                std::vector<int> list, first{0}, aux;
                for (Inst *in : kv.second) {
                    list.push_back(in->slot);
                    first.push_back(first.back() + in->ctx->N);
                    aux.push_back(in->ph == PH_A ? VEC_P : VEC_S);
                    aux.push_back(VEC_TM);
                    in->n_fine++;
                    in->matvecs++;
                }
                const Group g = group(list, first, aux, {});
                const LineShape sh{kv.first.NT, kv.first.C};
                const int f32 = kv.first.a, sch = kv.first.b, nb = first.back();
                plan.push_back([=] { return launch_fine1d_multi(sh, f32, sch, g, nb, st); });
            }
        }
        // coarse sweeps (INIT: S -> R, A: Tm -> D, B: Tm -> K) per line shape and scheme
        {
            std::map<ClassKey, std::vector<Inst *>> cls;
            for (Inst *in : T)
                if (in->ph == PH_INIT || in->ph == PH_A || in->ph == PH_B) {
                    const pit_ctx *c = in->ctx;
                    cls[{c->lc.sh.NT, c->lc.sh.C, c->coarse.scheme, c->nu_t() ? 1 : 0}].push_back(in);
                }
            for (auto &kv : cls) {
                std::vector<int> list, first{0}, aux;
                // longest chains first, so they start first
                std::stable_sort(kv.second.begin(), kv.second.end(), [](const Inst *a, const Inst *b) {
                    return (long)a->ctx->N * a->ctx->coarse.substeps > (long)b->ctx->N * b->ctx->coarse.substeps;
                });
                for (Inst *in : kv.second) {
                    list.push_back(in->slot);
                    first.push_back(first.back() + 1);
                    aux.push_back(in->ph == PH_INIT ? VEC_S : VEC_TM);
                    aux.push_back(in->ph == PH_INIT ? VEC_R : (in->ph == PH_A ? VEC_D : VEC_K));
                    in->n_coarse++;
                }
                const Group g = group(list, first, aux, {});
                const LineShape sh{kv.first.NT, kv.first.C};
                const int sch = kv.first.a, per_slice = kv.first.b;
                plan.push_back([=] { return launch_sweep1d_multi(sh, sch, per_slice != 0, g, st); });
            }
        }
        for (Inst *in : T)
            if (in->ph == PH_INIT) {
                plan.push_back([=] { return launch_copy(in->v(VEC_RT), in->v(VEC_R), in->n(), st); });
                plan.push_back([=] { return launch_copy(in->v(VEC_P), in->v(VEC_R), in->n(), st); });
            }
        // inner products of every phase but FINAL
        int nred = 0;
        {
            std::vector<int> list, first{0}, aux;
            for (Inst *in : T) {
                if (in->ph == PH_FINAL) continue;
                int q9[kDotsAux];
                dot_pairs(in->ph, q9);
                list.push_back(in->slot);
                first.push_back(first.back() + in->ctx->bps * in->ctx->N);
                aux.insert(aux.end(), q9, q9 + kDotsAux);
                in->red_pos = nred++;
            }
            if (!list.empty()) {
                const Group g = group(list, first, aux, {});
                const int nb = first.back();
                plan.push_back([=] { return launch_dots_multi(g, nb, st); });
            }
        }
        for (Inst *in : T)
            if (in->ph == PH_FINAL) {
                pit_ctx *c = in->ctx;
                plan.push_back([=] {
                    return launch_from_chunked(in->v(VEC_X), in->Xout, c->N, c->npts, c->lf.sh.NT, c->lf.sh.C, st);
                });
            }
        if (overflow) return PIT_ENOMEM;
        if (B.used) PIT_HIP(hipMemcpyAsync(B.d, B.h, B.used, hipMemcpyHostToDevice, st));
        for (auto &f : plan) PIT_HIP(f());
        if (nred) PIT_HIP(hipMemcpyAsync(L.h_red, L.d_red, nred * sizeof(RedOut), hipMemcpyDeviceToHost, st));
        PIT_HIP(hipEventRecord(L.ev, st));
        return PIT_OK;
    }
};

}  // namespace pit

namespace {

double ms_since(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

int check_opts(pit_solve_opts &o, const pit_ctx *c)
{
    if (o.max_iter <= 0) o.max_iter = 2 * c->N;
    if (o.x0_mode != PIT_X0_ZERO || o.half_step_check != 0 || !(o.tol >= 0.0)) return PIT_EINVAL;
    return PIT_OK;
}

pit_solve_opts default_opts()
{
    pit_solve_opts o{};
    o.tol = 1e-10;
    o.restart_tol = 1e-30;
    o.norm_mode = PIT_ABS;
    o.x0_mode = PIT_X0_ZERO;
    return o;
}



void fill_info(const Inst *in, pit_solve_info *info)
{
    if (!info) return;
    info->status = in->status;
    info->iters = in->k;
    info->matvecs = in->matvecs;
    info->restarts = in->restarts;
    info->res_norm = in->nrm;
    int hl = 0;
    if (info->history)
        for (double v : in->hist)
            if (hl < info->history_cap) info->history[hl++] = v;
    info->history_len = hl;
    info->n_fine = in->n_fine;
    info->n_coarse = in->n_coarse;
    info->ms_fine = info->ms_coarse = 0.0f;
    info->n_fine_timed = info->n_coarse_timed = 0;
    info->ms_krylov = 0.0f;
    info->n_krylov_timed = 0;
    info->ms_total = (float)(in->t_done - in->t_admit);
}

}  // namespace

struct pit_batch {
    pit::Engine eng;
    int max_count;
    explicit pit_batch(int n) : eng(n), max_count(n) {}
};

struct pit_server {
    pit_server_cfg cfg{};
    pit::Engine eng;
    Arena arena;
    char *base = nullptr;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Inst *> queue;
    std::unordered_map<uint64_t, Inst *> live;
    std::unordered_map<uint64_t, pit_result> done;
    uint64_t next_ticket = 1;
    bool stop = false;
    int running = 0;
    std::thread worker;
    std::chrono::steady_clock::time_point t0;
    int start_rc = PIT_OK;
    explicit pit_server(int slots) : eng(slots) {}
    void run();
};

extern "C" {

int pit_batch_create(int32_t max_count, pit_batch **out)
{
    if (!out || max_count < 1 || max_count > 65536) return PIT_EINVAL;
    *out = new (std::nothrow) pit_batch(max_count);
    return *out ? PIT_OK : PIT_ENOMEM;
}

size_t pit_batch_workspace_bytes(const pit_batch *b) { return b ? pit::Engine::bytes(b->max_count) : 0; }

int pit_batch_bind_workspace(pit_batch *b, void *dev_ptr, size_t bytes)
{
    if (!b || !dev_ptr || (reinterpret_cast<uintptr_t>(dev_ptr) % kAlign) != 0) return PIT_EINVAL;
    return b->eng.bind(static_cast<char *>(dev_ptr), bytes);
}

int pit_batch_destroy(pit_batch *b)
{
    delete b;
    return PIT_OK;
}

int pit_batch_solve(pit_batch *b, pit_ctx *const *ctxs, int32_t count, const double *const *u0, double *const *X,
                    const pit_solve_opts *opts, pit_solve_info *infos, void *stream)
{
    if (!b || !b->eng.bound() || !ctxs || !u0 || !X || count < 0 || count > b->max_count) return PIT_EINVAL;
    std::vector<Inst> insts(count);
    for (int i = 0; i < count; ++i) {
        if (!ctxs[i] || !ctxs[i]->ws || !u0[i] || !X[i]) return PIT_EINVAL;
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == ctxs[i]) return PIT_EINVAL;
        Inst &in = insts[i];
        in.ctx = ctxs[i];
        in.o = opts ? opts[i] : default_opts();
        if (check_opts(in.o, in.ctx) != PIT_OK) return PIT_EINVAL;
        in.u0 = u0[i];
        in.Xout = X[i];
        in.index = i;
    }
    const auto t0 = std::chrono::steady_clock::now();
    int rc = b->eng.after(static_cast<hipStream_t>(stream));
    if (rc) return rc;
    for (auto &in : insts) {
        in.t_admit = 0.0;
        if ((rc = b->eng.admit(&in))) return rc;
    }
    std::vector<Inst *> finished;
    while (!b->eng.idle()) {
        bool progress = false;
        rc = b->eng.round(finished, progress);
        if (rc) {
            b->eng.fail_all(pit_last_hip_error(), finished);
            break;
        }
        for (Inst *in : finished) in->t_done = ms_since(t0);
        finished.clear();
        // nothing finished or started: look again shortly (every lane is
        // polled, so a short phase on one lane is not held up by a long one)
        if (!progress) std::this_thread::sleep_for(std::chrono::microseconds(10));
    }
    for (Inst *in : finished) in->t_done = ms_since(t0);
    int first_bad = PIT_OK;
    for (int i = 0; i < count; ++i) {
        if (infos) fill_info(&insts[i], &infos[i]);
        if (first_bad == PIT_OK && insts[i].status != PIT_OK) first_bad = insts[i].status;
    }
    return first_bad;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// server
// ---------------------------------------------------------------------------
void pit_server::run()
{
    if (hipSetDevice(cfg.device) != hipSuccess) {
        start_rc = PIT_EHIP;
        return;
    }
    std::vector<Inst *> finished;
    for (;;) {
        // admission: arrival order, while a slot is free and the workspace fits
        std::vector<Inst *> admitted;
        {
            std::unique_lock<std::mutex> lk(mu);
            while (!queue.empty() && eng.has_slot()) {
                Inst *in = queue.front();
                size_t off = 0;
                if (!arena.alloc(in->ws_bytes, off)) break;
                in->ws_off = off;
                queue.pop_front();
                admitted.push_back(in);
            }
            if (admitted.empty() && eng.idle()) {
                if (stop && queue.empty()) return;
                cv.wait_for(lk, std::chrono::milliseconds(50));
                continue;
            }
        }
        for (Inst *in : admitted) {
            int rc = pit_bind_workspace(in->ctx, base + in->ws_off, in->ws_bytes);
            in->t_admit = ms_since(t0);
            if (rc == PIT_OK) rc = eng.admit(in);
            if (rc != PIT_OK) {
                in->status = rc;
                in->hip_error = pit_last_hip_error();
                finished.push_back(in);
            } else {
                std::lock_guard<std::mutex> lk(mu);
                running++;
            }
        }
        bool progress = false;
        int rc = eng.round(finished, progress);
        if (rc == PIT_OK && !progress && eng.any_busy()) std::this_thread::sleep_for(std::chrono::microseconds(20));
        if (rc != PIT_OK) eng.fail_all(pit_last_hip_error(), finished);
        if (!finished.empty()) {
            std::lock_guard<std::mutex> lk(mu);
            for (Inst *in : finished) {
                in->t_done = ms_since(t0);
                pit_result r{};
                r.status = in->status;
                r.iters = in->k;
                r.matvecs = in->matvecs;
                r.restarts = in->restarts;
                r.res_norm = in->nrm;
                r.t_submit_ms = in->t_submit;
                r.t_admit_ms = in->t_admit;
                r.t_done_ms = in->t_done;
                r.workspace_bytes = in->ws_bytes;
                r.hip_error = in->hip_error;
                if (in->slot >= 0) running--;
                arena.release(in->ws_off, in->ws_bytes);
                done[in->ticket] = r;
                live.erase(in->ticket);
                pit_destroy(in->ctx);
                delete in;
            }
            finished.clear();
        }
    }
}

extern "C" {

int pit_server_create(const pit_server_cfg *cfg, pit_server **out)
{
    if (!cfg || !out || !cfg->arena || cfg->max_slots < 1 || cfg->max_slots > 65536 ||
        (reinterpret_cast<uintptr_t>(cfg->arena) % kAlign) != 0)
        return PIT_EINVAL;
    *out = nullptr;
    pit_server *s = new (std::nothrow) pit_server(cfg->max_slots);
    if (!s) return PIT_ENOMEM;
    s->cfg = *cfg;
    s->base = static_cast<char *>(cfg->arena);
    const size_t own = align_up(pit::Engine::bytes(cfg->max_slots));
    if (cfg->arena_bytes < own) {
        delete s;
        return PIT_ENOMEM;
    }
    int rc = PIT_OK;
    if (hipSetDevice(cfg->device) != hipSuccess) rc = PIT_EHIP;
    if (rc == PIT_OK) rc = s->eng.bind(s->base, own);
    if (rc != PIT_OK) {
        delete s;
        return rc;
    }
    s->arena.init(own, cfg->arena_bytes - own);
    s->t0 = std::chrono::steady_clock::now();
    s->worker = std::thread([s] { s->run(); });
    *out = s;
    return PIT_OK;
}

int pit_submit(pit_server *s, const pit_request *req, uint64_t *ticket)
{
    if (!s || !req || !ticket || !req->u0 || !req->X) return PIT_EINVAL;
    pit_ctx *c = nullptr;
    int rc = pit_create(&req->problem, req->N, req->m, req->fine, req->coarse, &c);
    if (rc != PIT_OK) return rc;
    Inst *in = new (std::nothrow) Inst();
    if (!in) {
        pit_destroy(c);
        return PIT_ENOMEM;
    }
    in->ctx = c;
    in->o = req->opts;
    if (check_opts(in->o, c) != PIT_OK) {
        pit_destroy(c);
        delete in;
        return PIT_EINVAL;
    }
    in->u0 = req->u0;
    in->Xout = req->X;
    in->ws_bytes = align_up(pit_workspace_bytes(c));
    std::lock_guard<std::mutex> lk(s->mu);
    in->ticket = s->next_ticket++;
    in->t_submit = ms_since(s->t0);
    *ticket = in->ticket;
    if (in->ws_bytes > s->cfg.arena_bytes - align_up(pit::Engine::bytes(s->cfg.max_slots))) {
        // larger than the whole arena: it can never be admitted
        pit_result r{};
        r.status = PIT_ENOMEM;
        r.t_submit_ms = r.t_admit_ms = r.t_done_ms = in->t_submit;
        r.workspace_bytes = in->ws_bytes;
        s->done[in->ticket] = r;
        pit_destroy(c);
        delete in;
        return PIT_OK;
    }
    s->live[in->ticket] = in;
    s->queue.push_back(in);
    s->cv.notify_one();
    return PIT_OK;
}

int pit_poll(pit_server *s, uint64_t ticket, pit_result *res)
{
    if (!s) return PIT_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->done.find(ticket);
    if (it != s->done.end()) {
        if (res) *res = it->second;
        s->done.erase(it);
        return PIT_OK;
    }
    return s->live.count(ticket) ? PIT_EAGAIN : PIT_EINVAL;
}

int pit_server_load(pit_server *s, int32_t *queued, int32_t *running, uint64_t *arena_used)
{
    if (!s) return PIT_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    if (queued) *queued = (int32_t)s->queue.size();
    if (running) *running = s->running;
    if (arena_used) *arena_used = s->arena.used;
    return PIT_OK;
}

int pit_server_destroy(pit_server *s)
{
    if (!s) return PIT_EINVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_one();
    if (s->worker.joinable()) s->worker.join();
    for (auto &kv : s->live) {  // only if the worker could not start
        pit_destroy(kv.second->ctx);
        delete kv.second;
    }
    delete s;
    return PIT_OK;
}

}  // extern "C"
