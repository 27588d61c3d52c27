// Shared launches: several independent systems -- each with its own
// hierarchy, right-hand sides and Krylov scalars -- solved together, one
// launch per kernel step for all of them (per operator type).  This is how
// the serving loop batches solves of uneven grid size: the active requests'
// flow solves (CG on the Discussion's many solves of one model) or
// travel-time pairs (Benchmarking Examples, Eq. 1) share every launch of
// their iterations instead of each paying its own.
//
// Each launch runs k_seg over a table of per-system argument records; a
// block plays the block of its system's own grid, so every system sees the
// rows, block partials and summation order of a launch of its own, and its
// iterates, stopping test and restarts are bit for bit those of a solve on
// its own (amg_solve_pcg, amg_solve_bicgstab_pair).  The tables of one batch
// are built on the host once, copied to the device in one transfer, and the
// iterations replay the recorded launches (or, with graph = 1, captured HIP
// graphs of whole blocks of iterations).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "gw_device.h"
#include "gw_internal.h"
#include "solve_kernels.h"

namespace gw {

namespace {

double ms_now() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ---------------------------------------------------------------- plan ---
// Argument tables of a batch (one host image, copied to the device once)
// and sequences of recorded launches over them.
struct Launch {
    void (*fn)(const void *table, int nseg, unsigned nblk, hipStream_t s);
    size_t off;
    int nseg;
    unsigned nblk;
    int kid;       // timing class, or -1
    double bytes;  // algorithmic bytes of all its records
};
using Seq = std::vector<Launch>;

// The table of a launch: its records, then the record index of every block.
template <class A>
void launch_seg(const void *table, int nseg, unsigned nblk, hipStream_t s) {
    const Seg<A> *t = static_cast<const Seg<A> *>(table);
    hipLaunchKernelGGL(k_seg<A>, dim3(nblk), dim3(kBlock), 0, s, t, reinterpret_cast<const uint16_t *>(t + nseg));
}

struct Plan {
    std::vector<unsigned char> host;
    DBuf<unsigned char> dev;

    template <class A>
    void add(Seq &q, const std::vector<std::pair<A, unsigned>> &recs, int kid, double bytes) {
        static_assert(std::is_trivially_copyable<Seg<A>>::value, "records are copied as bytes");
        if (recs.empty()) return;
        GW_REQUIRE(recs.size() <= 65535, "shared launch: too many systems");
        uint32_t total = 0;
        for (const auto &r : recs) total += r.second;
        const size_t off = (host.size() + 255) / 256 * 256;
        const size_t idx = off + recs.size() * sizeof(Seg<A>);
        host.resize(idx + total * sizeof(uint16_t));
        uint32_t blk = 0;
        for (size_t k = 0; k < recs.size(); ++k) {
            const Seg<A> sg{recs[k].first, blk, recs[k].second};
            std::memcpy(host.data() + off + k * sizeof(Seg<A>), &sg, sizeof(Seg<A>));
            const uint16_t id = (uint16_t)k;
            for (uint32_t b = 0; b < recs[k].second; ++b)
                std::memcpy(host.data() + idx + (blk + b) * sizeof(uint16_t), &id, sizeof(id));
            blk += recs[k].second;
        }
        q.push_back(Launch{&launch_seg<A>, off, (int)recs.size(), blk, kid, bytes});
    }
    // copy the tables to the device (after every sequence is recorded)
    void upload(hipStream_t s) {
        dev.alloc(std::max<size_t>(host.size(), 256));
        GW_HIP(hipMemcpyAsync(dev.p, host.data(), host.size(), hipMemcpyHostToDevice, s));
        GW_HIP(hipStreamSynchronize(s));  // the host image may change after this
    }
    void run(const Seq &q, hipStream_t s) const {
        for (const Launch &L : q) {
            if (L.kid >= 0) {
                ProfScope ps(L.kid, L.bytes, s);
                L.fn(dev.p + L.off, L.nseg, L.nblk, s);
            } else {
                L.fn(dev.p + L.off, L.nseg, L.nblk, s);
            }
        }
        GW_HIP(hipGetLastError());
    }
};

// Records of one step, grouped by argument type (one launch per operator
// type met among the systems).
struct Buckets {
    struct Base {
        virtual ~Base() = default;
        virtual void emit(Plan &P, Seq &q, int kid) = 0;
    };
    template <class A>
    struct Bk : Base {
        std::vector<std::pair<A, unsigned>> recs;
        double bytes = 0.0;
        void emit(Plan &P, Seq &q, int kid) override { P.add<A>(q, recs, kid, bytes); }
    };
    std::vector<std::pair<const void *, std::unique_ptr<Base>>> list;
    template <class A>
    void put(const A &a, unsigned nb, double bytes) {
        static const char tag = 0;  // one address per argument type
        Bk<A> *b = nullptr;
        for (auto &e : list)
            if (e.first == &tag) b = static_cast<Bk<A> *>(e.second.get());
        if (!b) {
            list.emplace_back(&tag, std::unique_ptr<Base>(new Bk<A>()));
            b = static_cast<Bk<A> *>(list.back().second.get());
        }
        b->recs.emplace_back(a, nb);
        b->bytes += bytes;
    }
    void emit(Plan &P, Seq &q, int kid) {
        for (auto &e : list) e.second->emit(P, q, kid);
        list.clear();
    }
};

// ------------------------------------------------------------- systems ---
struct Sys {
    amg_hierarchy *H;
    int64_t n;
    unsigned g1, gG;      // grids of element-wise and row-product kernels
    double *part;         // the hierarchy's block partials
    KScalars *ks;         // this system's scalar records (one, or three for a pair)
    const int32_t *done;  // the flag its V-cycle kernels read
    double abytes;
};

// Operators of the shared launches: the sliced copy, or CSR with its lane
// group as a run-time value, so that systems whose matrices pick different
// groups still share one launch (same row sums as the one-system kernels).
template <class V>
OpCsrDyn<V> dyn(const Csr &A, const V *val) {
    return OpCsrDyn<V>{A.rowptr.p, A.col.p, val, A.grp};
}

template <class F>
void with_l0(const Level &L0, F &&f) {
    if (L0.St.built()) f(sten_op<double>(L0.St, L0.St.c.p));
    else if (L0.As.built()) f(OpSell<double>{view(L0.As), L0.As.val.p});
    else f(dyn<double>(L0.A, L0.A.val.p));
}

template <class V, class F>
void with_level_dyn(const Level &Lv, F &&f) {
    if (Lv.St.built() && LevelOps<V>::stval(Lv)) f(sten_op<V>(Lv.St, LevelOps<V>::stval(Lv)));
    else if (Lv.As.built() && LevelOps<V>::asval(Lv)) f(OpSell<V>{view(Lv.As), LevelOps<V>::asval(Lv)});
    else f(dyn<V>(Lv.A, LevelOps<V>::aval(Lv)));
}

// ---------------------------------------------------- V-cycle recording ---
// The kernel steps of one V-cycle of every system in `act` from level l down,
// in the order vcycle_level launches them for one system: b[j] the system's
// right-hand side at this level (type Bt), out[j] where its result goes
// (type Zt; null: the level's own buffer); x1_ready: the restriction into
// this level also wrote the first sweep (x1 = M b) into the level's x buffer
// of every system not on its coarsest level.  Returns each system's result.
template <class V, class Bt, class Zt, int NR>
std::vector<void *> rec_vcycle(Plan &P, Seq &q, std::vector<Sys> &S, const std::vector<int> &act, int l,
                               const std::vector<const Bt *> &b, const std::vector<Zt *> &out,
                               bool x1_ready = false) {
    const int vb = (int)sizeof(V);
    const double nr = NR;
    std::vector<void *> res(act.size(), nullptr);
    std::vector<int> fine;     // positions in act of systems that are not on their coarsest level
    Buckets B;
    for (size_t a = 0; a < act.size(); ++a) {
        amg_hierarchy *H = S[act[a]].H;
        Level &Lv = H->L[l];
        const int64_t n = Lv.A.n;
        if (l == H->nlev - 1) {
            Zt *y = out[a] ? out[a] : reinterpret_cast<Zt *>(Lv.vx.p);
            B.put(CoarseGemvK<Bt, Zt, NR>{(int32_t)n, H->inv.p, b[a], y, S[act[a]].done},
                  blocks_for(n * dev::kWave), (double)n * n * 8 + nr * n * (double)(sizeof(Bt) + sizeof(Zt)));
            res[a] = y;
        } else {
            fine.push_back((int)a);
        }
    }
    B.emit(P, q, K_COARSE_SOLVE);
    if (fine.empty()) return res;

    std::vector<V *> x(act.size()), t(act.size());
    for (int a : fine) {
        Level &Lv = S[act[a]].H->L[l];
        x[a] = reinterpret_cast<V *>(Lv.vx.p);
        t[a] = reinterpret_cast<V *>(Lv.vt.p);
    }
    const int npre = S[act[fine[0]]].H->prm.npre, npost = S[act[fine[0]]].H->prm.npost;
    // pre-smoothing (npre >= 1: the batch requires it)
    const int swept = x1_ready ? 1 : (npre >= 2 ? 2 : 1);
    for (int a : fine) {
        if (x1_ready) break;
        Level &Lv = S[act[a]].H->L[l];
        const int64_t n = Lv.A.n;
        const double abytes = op_bytes(Lv, vb);
        with_level_dyn<V>(Lv, [&](auto op) {
            using OP = decltype(op);
            B.put(SmoothFirstK<OP, V, Bt, V, NR>{n, op, LevelOps<V>::mval(Lv), b[a], x[a], npre >= 2 ? 1 : 0,
                                                  S[act[a]].done},
                  grid_rows(n, op.lanes()), (npre >= 2 ? abytes : 0.0) + n * (double)vb + nr * n * (double)(sizeof(Bt) + vb));
        });
    }
    if (!x1_ready) B.emit(P, q, level_kid(K_SMOOTH_FIRST0, l));
    auto sweep = [&](auto yout_of) {
        for (int a : fine) {
            Level &Lv = S[act[a]].H->L[l];
            const int64_t n = Lv.A.n;
            const double abytes = op_bytes(Lv, vb);
            auto *yo = yout_of(a);
            using YT = std::remove_pointer_t<decltype(yo)>;
            with_level_dyn<V>(Lv, [&](auto op) {
                using OP = decltype(op);
                B.put(SmoothK<OP, V, Bt, V, YT, NR>{n, op, LevelOps<V>::mval(Lv), b[a], x[a], yo, S[act[a]].done},
                      grid_rows(n, op.lanes()), abytes + n * (double)vb + nr * n * (double)(sizeof(Bt) + vb + sizeof(YT)));
            });
        }
        B.emit(P, q, level_kid(K_SMOOTH0, l));
    };
    for (int k = swept; k < npre; ++k) {
        sweep([&](int a) { return t[a]; });
        for (int a : fine) std::swap(x[a], t[a]);
    }
    // residual, then restriction
    std::vector<V *> bnext(act.size(), nullptr);
    for (int a : fine) bnext[a] = reinterpret_cast<V *>(S[act[a]].H->L[l + 1].vb.p);
    for (int a : fine) {
        Level &Lv = S[act[a]].H->L[l];
        const int64_t n = Lv.A.n;
        const double abytes = op_bytes(Lv, vb);
        with_level_dyn<V>(Lv, [&](auto op) {
            using OP = decltype(op);
            B.put(ResidualK<OP, V, Bt, V, V, NR>{n, op, b[a], x[a], t[a], S[act[a]].done}, grid_rows(n, op.lanes()),
                  abytes + nr * n * (double)(sizeof(Bt) + 2 * vb));
        });
    }
    B.emit(P, q, level_kid(K_RESIDUAL0, l));
    for (int a : fine) {
        amg_hierarchy *H = S[act[a]].H;
        Level &Lv = H->L[l], &Nx = H->L[l + 1];
        const int64_t n = Lv.A.n, nc = Lv.nc;
        const OpCsrDyn<V> op = dyn<V>(Lv.R, LevelOps<V>::rval(Lv));
        const bool x1c = restrict_writes_x1(H, l);
        B.put(RestrictK<OpCsrDyn<V>, V, NR>{nc, op, t[a], bnext[a], x1c ? LevelOps<V>::mval(Nx) : (const V *)nullptr,
                                            x1c ? reinterpret_cast<V *>(Nx.vx.p) : (V *)nullptr, S[act[a]].done},
              grid_rows(nc, op.lanes()),
              csr_bytes(nc, Lv.R.nnz, vb) + nr * (double)(n + nc) * vb + (x1c ? (nr + 1) * nc * (double)vb : 0.0));
    }
    B.emit(P, q, level_kid(K_RESTRICT0, l));
    // the next level, for the systems that continue
    std::vector<int> act2;
    std::vector<const V *> b2;
    std::vector<V *> o2;
    for (int a : fine) {
        act2.push_back(act[a]);
        b2.push_back(bnext[a]);
        o2.push_back(nullptr);
    }
    // every system that continues past level l+1 has its first sweep there
    std::vector<void *> xc = rec_vcycle<V, V, V, NR>(P, q, S, act2, l + 1, b2, o2, true);
    for (size_t k = 0; k < fine.size(); ++k) {
        const int a = fine[k];
        Level &Lv = S[act[a]].H->L[l];
        const int64_t n = Lv.A.n, nc = Lv.nc;
        const OpCsrDyn<V> op = dyn<V>(Lv.P, LevelOps<V>::pval(Lv));
        B.put(ProlongK<OpCsrDyn<V>, V, V, NR>{n, op, static_cast<const V *>(xc[k]), x[a], S[act[a]].done},
              grid_rows(n, op.lanes()), csr_bytes(n, Lv.P.nnz, vb) + nr * (double)(2 * n + nc) * vb);
    }
    B.emit(P, q, level_kid(K_PROLONG0, l));
    // post-smoothing (npost >= 1); the last sweep writes the requested output
    for (int k = 0; k < npost; ++k) {
        const bool last = k == npost - 1;
        std::vector<int> to_out, to_t;
        for (int a : fine) (last && out[a] ? to_out : to_t).push_back(a);
        // a level's systems all have or all lack an output buffer (level 0:
        // all have one; deeper levels: none)
        if (!to_out.empty()) {
            sweep([&](int a) { return out[a]; });
            for (int a : fine) res[a] = out[a];
        } else {
            sweep([&](int a) { return t[a]; });
            for (int a : fine) {
                std::swap(x[a], t[a]);
                res[a] = x[a];
            }
        }
    }
    return res;
}

// One V-cycle of every system in `act`: z[j] = V(r[j]) (NR interleaved
// right-hand sides, FP64 at the boundary), in the hierarchy's precision.
template <int NR>
void rec_precond(Plan &P, Seq &q, std::vector<Sys> &S, const std::vector<int> &act,
                 const std::vector<const double *> &r, const std::vector<double *> &z, bool mixed) {
    if (mixed) rec_vcycle<float, double, double, NR>(P, q, S, act, 0, r, z);
    else rec_vcycle<double, double, double, NR>(P, q, S, act, 0, r, z);
}

// Finalize step of every system in `act` (one block each).
void rec_fin(Plan &P, Seq &q, std::vector<Sys> &S, const std::vector<int> &act, int op, bool pair,
             double rtol, const std::vector<unsigned> &nb, int mask = 3) {
    Buckets B;
    for (size_t a = 0; a < act.size(); ++a) {
        Sys &y = S[act[a]];
        if (pair) B.put(Fin2K{op, nb[a], y.part, rtol, y.ks, mask}, 1u, 0.0);
        else B.put(FinK{op, nb[a], y.part, rtol, y.ks}, 1u, 0.0);
    }
    B.emit(P, q, -1);
}

void check_member(const amg_hierarchy *H, const amg_hierarchy *first, const char *who) {
    GW_REQUIRE(H, std::string(who) + ": null hierarchy");
    GW_REQUIRE(H->nlev >= 1 && H->prm.smoother != GW_SMOOTHER_ILU0,
               std::string(who) + ": every system needs a diagonal-smoother AMG preconditioner");
    GW_REQUIRE(H->prm.npre >= 1 && H->prm.npost >= 1,
               std::string(who) + ": shared launches need at least one pre- and one post-sweep");
    GW_REQUIRE(H->prm.precision == first->prm.precision && H->prm.npre == first->prm.npre &&
                   H->prm.npost == first->prm.npost,
               std::string(who) + ": the systems must share precision and sweep counts");
}

}  // namespace

// ---------------------------------------------------------------- engine ---
// The shared-launch solver: an active set of systems of one kind (CG or the
// BiCGSTAB pair) with the same hierarchy precision and sweep counts and the
// same stopping parameters.  Each step admits the systems that joined since
// the last one (their start: r = b - A x0 with x0 = 0, and for CG the first
// preconditioner application), runs one block of iterations of every active
// system in shared launches, reads every system's scalars, and completes the
// systems whose flag says done (true residual, then final or a restart, as
// their own solve would).  Systems join and leave between blocks, so a system
// that converges early returns at once and one that arrives later starts at
// the next block.  A system's kernels and their order are those of its own
// solve (krylov_pcg / krylov_bicgstab2), so are its iterates, bit for bit.
struct BatchEngine::State {
    Plan plan;
    Seq iter[2];
};

struct BatchEngine::Member {
    void *tag = nullptr;
    amg_hierarchy *H = nullptr;
    const double *b0 = nullptr, *b1 = nullptr;
    double *x0 = nullptr, *x1 = nullptr;
    Sys sys{};
    int slot = -1;
    int par_off = 0;  // CG: block parity at the system's (re)start
    PollPlan plan[2] = {{1, false}, {1, false}};
    int restarts[2] = {0, 0}, status[2] = {GW_NOT_CONVERGED, GW_NOT_CONVERGED}, final[2] = {0, 0};
    KScalars kfinal[2] = {};
    double *v[10] = {};  // CG: r z pa pb q x; pair: b r rh p v s t ph sh x (interleaved)
    double t0 = 0.0;
};

namespace {

constexpr int kCgVecs = 6, kPairVecs = 20;

}  // namespace

BatchEngine::BatchEngine(int kind, const amg_solve_params &sp, int capacity, hipStream_t s)
    : kind_(kind), sp_(sp), cap_(capacity), s_(s) {
    nrec_ = kind == 0 ? 1 : 3;
    ks_.alloc((size_t)cap_ * nrec_);
    stage_.reset(new Pinned((size_t)cap_ * nrec_ * sizeof(KScalars)));
    for (int k = cap_ - 1; k >= 0; --k) free_.push_back(k);
    check_ = std::max(1, sp.check_every);
    cnt_ = check_;
}

BatchEngine::~BatchEngine() = default;

bool BatchEngine::accepts(const amg_hierarchy *H, const amg_solve_params &sp) const {
    if ((int)(members_.size() + joining_.size()) >= cap_) return false;
    if (sp.rtol != sp_.rtol || sp.maxiter != sp_.maxiter || sp.check_every != sp_.check_every ||
        sp.flexible != sp_.flexible)
        return false;
    const amg_hierarchy *ref = !members_.empty() ? members_[0]->H : (!joining_.empty() ? joining_[0]->H : nullptr);
    return !ref || (H->prm.precision == ref->prm.precision && H->prm.npre == ref->prm.npre &&
                    H->prm.npost == ref->prm.npost);
}

void BatchEngine::join(void *tag, amg_hierarchy *H, const double *b0, const double *b1, double *x0, double *x1) {
    const char *who = kind_ == 0 ? "amg_solve_pcg_batch" : "amg_solve_bicgstab_pair_batch";
    const amg_hierarchy *ref = !members_.empty() ? members_[0]->H : (!joining_.empty() ? joining_[0]->H : H);
    check_member(H, ref, who);
    for (auto &m : members_) GW_REQUIRE(m->H != H, std::string(who) + ": a hierarchy appears twice");
    for (auto &m : joining_) GW_REQUIRE(m->H != H, std::string(who) + ": a hierarchy appears twice");
    GW_REQUIRE(!free_.empty(), std::string(who) + ": too many systems");
    std::unique_ptr<Member> m(new Member());
    m->tag = tag;
    m->H = H;
    m->b0 = b0;
    m->b1 = b1;
    m->x0 = x0;
    m->x1 = x1;
    m->slot = free_.back();
    free_.pop_back();
    m->t0 = ms_now();
    ensure_krylov_workspace(H, kind_ == 0 ? kCgVecs : kPairVecs);
    if (kind_ == 1) ensure_level_vectors(H, 2);
    const Level &L0 = H->L[0];
    Sys &y = m->sys;
    y.H = H;
    y.n = L0.A.n;
    const int G = (L0.St.built() || L0.As.built()) ? 1 : L0.A.grp;
    y.g1 = kgrid(y.n, 1);
    y.gG = kgrid(y.n, G);
    y.part = H->partials.p;
    y.ks = ks_.p + (size_t)m->slot * nrec_;
    y.done = kind_ == 0 ? &y.ks->done : &y.ks[2].done;
    y.abytes = op_bytes(L0, 8);
    const int64_t len = kind_ == 0 ? y.n : 2 * y.n;
    for (int k = 0; k < (kind_ == 0 ? kCgVecs : 10); ++k) m->v[k] = H->kvec.p + k * len;
    m->plan[0] = m->plan[1] = PollPlan{check_, false};
    joining_.push_back(std::move(m));
}

bool BatchEngine::empty() const { return members_.empty() && joining_.empty(); }
int BatchEngine::size() const { return (int)(members_.size() + joining_.size()); }

namespace {

std::vector<Sys> sys_of(const std::vector<BatchEngine::Member *> &ms) {
    std::vector<Sys> S;
    for (auto *m : ms) S.push_back(m->sys);
    return S;
}

std::vector<int> iota_n(size_t n) {
    std::vector<int> a(n);
    for (size_t k = 0; k < n; ++k) a[k] = (int)k;
    return a;
}

}  // namespace

void BatchEngine::read_ks() {
    const size_t bytes = (size_t)cap_ * nrec_ * sizeof(KScalars);
    GW_HIP(hipMemcpyAsync(stage_->p, ks_.p, bytes, hipMemcpyDeviceToHost, s_));
    GW_HIP(hipStreamSynchronize(s_));
}

KScalars *BatchEngine::hks(const Member &m) {
    return static_cast<KScalars *>(stage_->p) + (size_t)m.slot * nrec_;
}

void BatchEngine::write_ks(const Member &m) {
    GW_HIP(hipMemcpyAsync(ks_.p + (size_t)m.slot * nrec_, hks(m), nrec_ * sizeof(KScalars), hipMemcpyHostToDevice,
                          s_));
    GW_HIP(hipStreamSynchronize(s_));
}

// Record and run one step for the systems `ms` (a plan of its own).
template <class Rec>
void BatchEngine::run_once(const std::vector<Member *> &ms, Rec &&rec) {
    if (ms.empty()) return;
    Plan P;
    Seq q;
    std::vector<Sys> S = sys_of(ms);
    rec(P, q, S);
    P.upload(s_);
    P.run(q, s_);
}

void BatchEngine::admit(std::vector<Member *> &done_now) {
    if (joining_.empty()) return;
    std::vector<Member *> J;
    for (auto &m : joining_) J.push_back(m.get());
    const double rtol = sp_.rtol;
    // scalars: zero, maxiter, flexible (CG), status
    for (Member *m : J) {
        KScalars *k = hks(*m);
        for (int r = 0; r < nrec_; ++r) k[r] = KScalars{};
        for (int r = 0; r < (kind_ == 0 ? 1 : 2); ++r) {
            k[r].maxiter = std::max(0, sp_.maxiter);
            k[r].status = GW_NOT_CONVERGED;
            if (kind_ == 0)
                k[r].flexible = sp_.flexible < 0 ? (m->H->mixed() ? 1 : 0) : (sp_.flexible ? 1 : 0);
        }
        write_ks(*m);
    }
    const std::vector<int> all = iota_n(J.size());
    if (kind_ == 0) {
        for (Member *m : J) fill_f64(m->v[5], 0.0, m->sys.n, s_);
        run_once(J, [&](Plan &P, Seq &q, std::vector<Sys> &S) {
            Buckets B;
            std::vector<unsigned> nb;
            for (size_t a = 0; a < J.size(); ++a) {
                Member *m = J[a];
                with_l0(m->H->L[0], [&](auto o) {
                    using OP = decltype(o);
                    B.put(KrInitK<OP>{m->sys.n, o, m->b0, m->v[5], m->v[0], nullptr, m->v[2], nullptr, m->sys.part},
                          m->sys.gG, m->sys.abytes + 4 * 8.0 * m->sys.n);
                });
                nb.push_back(m->sys.gG);
            }
            B.emit(P, q, K_KRYLOV_SPMV);
            rec_fin(P, q, S, all, FIN_INIT_FIRST, false, rtol, nb);
        });
    } else {
        for (Member *m : J) fill_f64(m->v[9], 0.0, 2 * m->sys.n, s_);
        run_once(J, [&](Plan &P, Seq &q, std::vector<Sys> &S) {
            Buckets B;
            std::vector<unsigned> nb;
            for (Member *m : J)
                B.put(InterleaveK{m->sys.n, m->b0, m->b1, m->v[0]}, m->sys.g1, 4 * 8.0 * m->sys.n);
            B.emit(P, q, -1);
            for (Member *m : J) {
                with_l0(m->H->L[0], [&](auto o) {
                    using OP = decltype(o);
                    B.put(KrInit2K<OP>{m->sys.n, o, m->v[0], m->v[9], m->v[1], m->v[2], m->v[3], m->v[4],
                                       m->sys.part, 3},
                          m->sys.gG, m->sys.abytes + 7 * 16.0 * m->sys.n);
                });
                nb.push_back(m->sys.gG);
            }
            B.emit(P, q, K_KRYLOV_SPMV);
            rec_fin(P, q, S, all, FIN_INIT_FIRST, true, rtol, nb);
        });
    }
    read_ks();
    std::vector<Member *> go;  // CG systems that take their first preconditioner application
    for (Member *m : J) {
        KScalars *k = hks(*m);
        if (kind_ == 0) {
            if (k->bnorm == 0.0) {
                // b = 0: x = 0, nothing to iterate
                m->final[0] = 1;
                m->status[0] = GW_OK;
                k->done = 1;
                k->iters = 0;
                k->rr = 0.0;
                k->rel_true = 0.0;
                m->kfinal[0] = *k;
                write_ks(*m);
                continue;
            }
            if (!k->done) go.push_back(m);
        } else {
            bool zero = false;
            for (int c = 0; c < 2; ++c) {
                if (k[c].bnorm != 0.0) continue;
                m->final[c] = 1;
                m->status[c] = GW_OK;
                k[c].done = 1;
                k[c].iters = 0;
                k[c].rr = 0.0;
                k[c].rel_true = 0.0;
                m->kfinal[c] = k[c];
                zero = true;
            }
            if (zero) {
                k[2].done = k[0].done && k[1].done;
                write_ks(*m);
            }
        }
    }
    if (kind_ == 0 && !go.empty()) first_z(go);
    for (auto &m : joining_) {
        m->par_off = parity_;
        Member *raw = m.get();
        members_.push_back(std::move(m));
        const bool all_final = raw->final[0] && (kind_ == 0 || raw->final[1]);
        if (all_final) done_now.push_back(raw);
    }
    joining_.clear();
    dirty_ = true;
}

// CG: z = V(r), then r.z and z.q and beta's first form, for the systems `ms`.
void BatchEngine::first_z(const std::vector<Member *> &ms) {
    const bool mixed = ms[0]->H->mixed();
    const double rtol = sp_.rtol;
    run_once(ms, [&](Plan &P, Seq &q, std::vector<Sys> &S) {
        const std::vector<int> all = iota_n(ms.size());
        std::vector<const double *> rin;
        std::vector<double *> zout;
        std::vector<unsigned> nb;
        for (Member *m : ms) rin.push_back(m->v[0]), zout.push_back(m->v[1]), nb.push_back(m->sys.g1);
        rec_precond<1>(P, q, S, all, rin, zout, mixed);
        Buckets B;
        for (Member *m : ms)
            B.put(CgDotK{m->sys.n, m->v[0], m->v[1], m->v[4], m->sys.part, m->sys.ks}, m->sys.g1, 3 * 8.0 * m->sys.n);
        B.emit(P, q, K_KRYLOV_DOT);
        rec_fin(P, q, S, all, FIN_CG_BETA_FIRST, false, rtol, nb);
    });
}

// The iteration plan of every active system (CG: two variants, by block
// parity; each system's p buffers follow its own parity).
void BatchEngine::record_iterations() {
    st_.reset(new State());
    std::vector<Member *> ms;
    for (auto &m : members_)
        if (!(m->final[0] && (kind_ == 0 || m->final[1]))) ms.push_back(m.get());
    if (ms.empty()) return;
    std::vector<Sys> S = sys_of(ms);
    const std::vector<int> all = iota_n(ms.size());
    const bool mixed = ms[0]->H->mixed();
    const double rtol = sp_.rtol;
    std::vector<unsigned> nb1, nbG;
    for (Member *m : ms) nb1.push_back(m->sys.g1), nbG.push_back(m->sys.gG);
    Plan &P = st_->plan;
    if (kind_ == 0) {
        for (int par = 0; par < 2; ++par) {
            Seq &q = st_->iter[par];
            Buckets B;
            for (Member *m : ms) {
                const int lp = par ^ m->par_off;
                double *po = lp ? m->v[3] : m->v[2], *pn = lp ? m->v[2] : m->v[3];
                with_l0(m->H->L[0], [&](auto o) {
                    using OP = decltype(o);
                    B.put(CgSpmvK<OP>{m->sys.n, o, m->v[1], po, pn, m->v[4], m->sys.part, m->sys.ks}, m->sys.gG,
                          m->sys.abytes + 4 * 8.0 * m->sys.n);
                });
            }
            B.emit(P, q, K_KRYLOV_SPMV);
            rec_fin(P, q, S, all, FIN_CG_ALPHA, false, rtol, nbG);
            for (Member *m : ms) {
                const int lp = par ^ m->par_off;
                double *pn = lp ? m->v[2] : m->v[3];
                B.put(CgUpdateK{m->sys.n, m->v[5], m->v[0], pn, m->v[4], m->sys.part, m->sys.ks}, m->sys.g1,
                      6 * 8.0 * m->sys.n);
            }
            B.emit(P, q, K_KRYLOV_UPDATE);
            rec_fin(P, q, S, all, FIN_CG_CONV, false, rtol, nb1);
            std::vector<const double *> rin;
            std::vector<double *> zout;
            for (Member *m : ms) rin.push_back(m->v[0]), zout.push_back(m->v[1]);
            rec_precond<1>(P, q, S, all, rin, zout, mixed);
            for (Member *m : ms)
                B.put(CgDotK{m->sys.n, m->v[0], m->v[1], m->v[4], m->sys.part, m->sys.ks}, m->sys.g1,
                      3 * 8.0 * m->sys.n);
            B.emit(P, q, K_KRYLOV_DOT);
            rec_fin(P, q, S, all, FIN_CG_BETA, false, rtol, nb1);
        }
    } else {
        Seq &q = st_->iter[0];
        Buckets B;
        for (Member *m : ms)
            B.put(BcgP2K{m->sys.n, m->v[1], m->v[3], m->v[4], m->sys.ks}, m->sys.g1, 4 * 16.0 * m->sys.n);
        B.emit(P, q, K_KRYLOV_UPDATE);
        {
            std::vector<const double *> in;
            std::vector<double *> out;
            for (Member *m : ms) in.push_back(m->v[3]), out.push_back(m->v[7]);
            rec_precond<2>(P, q, S, all, in, out, mixed);
        }
        for (Member *m : ms)
            with_l0(m->H->L[0], [&](auto o) {
                using OP = decltype(o);
                B.put(BcgV2K<OP>{m->sys.n, o, m->v[7], m->v[4], m->v[2], m->sys.part, m->sys.ks}, m->sys.gG,
                      m->sys.abytes + 3 * 16.0 * m->sys.n);
            });
        B.emit(P, q, K_KRYLOV_SPMV);
        rec_fin(P, q, S, all, FIN_BCG_ALPHA, true, rtol, nbG);
        for (Member *m : ms)
            B.put(BcgS2K{m->sys.n, m->v[1], m->v[4], m->v[5], m->sys.part, m->sys.ks}, m->sys.g1,
                  3 * 16.0 * m->sys.n);
        B.emit(P, q, K_KRYLOV_UPDATE);
        rec_fin(P, q, S, all, FIN_BCG_S, true, rtol, nb1);
        {
            std::vector<const double *> in;
            std::vector<double *> out;
            for (Member *m : ms) in.push_back(m->v[5]), out.push_back(m->v[8]);
            rec_precond<2>(P, q, S, all, in, out, mixed);
        }
        for (Member *m : ms)
            with_l0(m->H->L[0], [&](auto o) {
                using OP = decltype(o);
                B.put(BcgT2K<OP>{m->sys.n, o, m->v[8], m->v[6], m->v[5], m->sys.part, m->sys.ks}, m->sys.gG,
                      m->sys.abytes + 3 * 16.0 * m->sys.n);
            });
        B.emit(P, q, K_KRYLOV_SPMV);
        rec_fin(P, q, S, all, FIN_BCG_OMEGA, true, rtol, nbG);
        for (Member *m : ms)
            B.put(BcgXr2K{m->sys.n, m->v[9], m->v[1], m->v[7], m->v[8], m->v[5], m->v[6], m->v[2], m->sys.part,
                          m->sys.ks},
                  m->sys.g1, 8 * 16.0 * m->sys.n);
        B.emit(P, q, K_KRYLOV_UPDATE);
        rec_fin(P, q, S, all, FIN_BCG_XR, true, rtol, nb1);
    }
    P.upload(s_);
    dirty_ = false;
}

// A system whose flag says done: true residual, then final (its output
// written) or a restart from its iterate.  Returns whether it is final.
void BatchEngine::complete(const std::vector<Member *> &ms, std::vector<Member *> &done_now) {
    const double rtol = sp_.rtol;
    run_once(ms, [&](Plan &P, Seq &q, std::vector<Sys> &S) {
        Buckets B;
        std::vector<unsigned> nb;
        for (Member *m : ms) {
            with_l0(m->H->L[0], [&](auto o) {
                using OP = decltype(o);
                if (kind_ == 0)
                    B.put(TrueResK<OP>{m->sys.n, o, m->b0, m->v[5], m->sys.part}, m->sys.gG,
                          m->sys.abytes + 2 * 8.0 * m->sys.n);
                else
                    B.put(TrueRes2K<OP>{m->sys.n, o, m->v[0], m->v[9], m->sys.part}, m->sys.gG,
                          m->sys.abytes + 2 * 16.0 * m->sys.n);
            });
            nb.push_back(m->sys.gG);
        }
        B.emit(P, q, K_TRUE_RESIDUAL);
        rec_fin(P, q, S, iota_n(ms.size()), FIN_TRUE_RES, kind_ == 1, rtol, nb);
    });
    read_ks();
    std::vector<Member *> again;
    std::vector<int> masks;
    for (Member *m : ms) {
        KScalars *k = hks(*m);
        int mask = 0;
        for (int c = 0; c < (kind_ == 0 ? 1 : 2); ++c) {
            if (m->final[c]) continue;
            const KScalars &q1 = k[c];
            if (q1.status == GW_BREAKDOWN) m->status[c] = GW_BREAKDOWN, m->final[c] = 1;
            else if (q1.rel_true <= rtol) m->status[c] = GW_OK, m->final[c] = 1;
            else if (q1.iters >= q1.maxiter || m->restarts[c] >= 8) m->status[c] = GW_NOT_CONVERGED, m->final[c] = 1;
            else {
                ++m->restarts[c];
                mask |= 1 << c;
            }
            if (m->final[c]) m->kfinal[c] = q1;
        }
        if (mask) {
            again.push_back(m);
            masks.push_back(mask);
        } else {
            done_now.push_back(m);
        }
    }
    if (again.empty()) return;
    // restart from the iterate: r = b - A x (and the pair's r_hat, p, v)
    run_once(again, [&](Plan &P, Seq &q, std::vector<Sys> &S) {
        Buckets B;
        std::vector<unsigned> nb;
        for (size_t a = 0; a < again.size(); ++a) {
            Member *m = again[a];
            with_l0(m->H->L[0], [&](auto o) {
                using OP = decltype(o);
                if (kind_ == 0)
                    B.put(KrInitK<OP>{m->sys.n, o, m->b0, m->v[5], m->v[0], nullptr, m->v[2], nullptr, m->sys.part},
                          m->sys.gG, 0.0);
                else
                    B.put(KrInit2K<OP>{m->sys.n, o, m->v[0], m->v[9], m->v[1], m->v[2], m->v[3], m->v[4],
                                       m->sys.part, masks[a]},
                          m->sys.gG, 0.0);
            });
            nb.push_back(m->sys.gG);
        }
        B.emit(P, q, K_KRYLOV_SPMV);
        for (size_t a = 0; a < again.size(); ++a) {
            Member *m = again[a];
            if (kind_ == 0) B.put(FinK{FIN_INIT_RESTART, nb[a], m->sys.part, rtol, m->sys.ks}, 1u, 0.0);
            else B.put(Fin2K{FIN_INIT_RESTART, nb[a], m->sys.part, rtol, m->sys.ks, masks[a]}, 1u, 0.0);
        }
        B.emit(P, q, -1);
    });
    read_ks();
    if (kind_ == 0) {
        std::vector<Member *> go;
        for (Member *m : again) {
            m->par_off = parity_;  // its p buffers start over as at its first iteration
            m->plan[0] = PollPlan{check_, false};
            if (!hks(*m)->done) go.push_back(m);
        }
        if (!go.empty()) first_z(go);
    } else {
        for (Member *m : again) m->plan[0] = m->plan[1] = PollPlan{check_, false};
    }
    dirty_ = true;
}

std::vector<BatchEngine::Result> BatchEngine::step() {
    std::vector<Member *> done_now;
    admit(done_now);
    // systems still iterating
    auto running = [&](Member *m) {
        const KScalars *k = hks(*m);
        return kind_ == 0 ? (!m->final[0] && !k->done) : (!k[2].done);
    };
    bool any = false;
    for (auto &m : members_) any |= running(m.get());
    if (any) {
        if (dirty_) record_iterations();
        for (int c = 0; c < cnt_; ++c) {
            st_->plan.run(st_->iter[kind_ == 0 ? parity_ : 0], s_);
            if (kind_ == 0) parity_ ^= 1;
        }
        read_ks();
        int c2 = 1;
        for (auto &m : members_) {
            KScalars *k = hks(*m);
            for (int c = 0; c < (kind_ == 0 ? 1 : 2); ++c) {
                const int cq = m->plan[c].next(std::sqrt(k[c].rr), k[c].tol, k[c].iters);
                if (!k[c].done && !m->final[c]) c2 = std::max(c2, cq);
            }
        }
        cnt_ = c2;
    }
    // systems that stopped iterating and are not final yet
    std::vector<Member *> fin;
    for (auto &m : members_) {
        const bool final_all = m->final[0] && (kind_ == 0 || m->final[1]);
        if (final_all) continue;
        if (!running(m.get())) fin.push_back(m.get());
    }
    if (!fin.empty()) complete(fin, done_now);
    // outputs of the finished systems, then they leave
    std::vector<Result> out;
    if (done_now.empty()) return out;
    {
        std::vector<Member *> pairs;
        for (Member *m : done_now) {
            if (kind_ == 0) copy_bytes(m->x0, m->v[5], sizeof(double) * (size_t)m->sys.n, s_);
            else pairs.push_back(m);
        }
        if (!pairs.empty())
            run_once(pairs, [&](Plan &P, Seq &q, std::vector<Sys> &) {
                Buckets B;
                for (Member *m : pairs) B.put(SplitK{m->sys.n, m->v[9], m->x0, m->x1}, m->sys.g1, 4 * 8.0 * m->sys.n);
                B.emit(P, q, -1);
            });
        GW_HIP(hipStreamSynchronize(s_));
    }
    const double now = ms_now();
    for (Member *m : done_now) {
        Result r;
        r.tag = m->tag;
        for (int c = 0; c < (kind_ == 0 ? 1 : 2); ++c) {
            const KScalars &q1 = m->kfinal[c];
            amg_solve_info &i = r.info[c];
            i.iters = q1.iters;
            i.status = m->status[c];
            i.restarts = m->restarts[c];
            i.rel_res = q1.bnorm != 0.0 ? std::sqrt(q1.rr) / q1.bnorm : 0.0;
            i.rel_res_true = q1.bnorm != 0.0 ? q1.rel_true : 0.0;
            i.setup_ms = 0.0;
            i.solve_ms = now - m->t0;
        }
        if (kind_ == 0) {
            r.status = m->status[0];
        } else {
            const int s0 = m->status[0], s1 = m->status[1];
            r.status = (s0 == GW_BREAKDOWN || s1 == GW_BREAKDOWN) ? GW_BREAKDOWN
                       : (s0 != GW_OK || s1 != GW_OK)           ? GW_NOT_CONVERGED
                                                                : GW_OK;
        }
        out.push_back(r);
        free_.push_back(m->slot);
    }
    // remove them
    std::vector<std::unique_ptr<Member>> keep;
    for (auto &m : members_) {
        bool gone = false;
        for (Member *d : done_now) gone |= d == m.get();
        if (!gone) keep.push_back(std::move(m));
    }
    members_.swap(keep);
    dirty_ = true;
    return out;
}

// ------------------------------------------------------- one-shot batches ---
namespace {

int run_batch(int kind, amg_hierarchy *const *Hs, const double *const *b0, const double *const *b1,
              double *const *x0, double *const *x1, int32_t nsys, const amg_solve_params &sp, amg_solve_info *info,
              hipStream_t s) {
    const char *who = kind == 0 ? "amg_solve_pcg_batch" : "amg_solve_bicgstab_pair_batch";
    GW_REQUIRE(nsys >= 1 && nsys <= 256, std::string(who) + ": nsys must be in [1, 256]");
    GW_REQUIRE(Hs, std::string(who) + ": null hierarchy list");
    BatchEngine E(kind, sp, nsys, s);
    for (int j = 0; j < nsys; ++j)
        E.join(reinterpret_cast<void *>((intptr_t)j), Hs[j], b0[j], kind ? b1[j] : nullptr, x0[j],
               kind ? x1[j] : nullptr);
    int worst = GW_OK;
    while (!E.empty())
        for (const auto &r : E.step()) {
            const int j = (int)(intptr_t)r.tag;
            if (info) {
                if (kind == 0) info[j] = r.info[0];
                else info[2 * j] = r.info[0], info[2 * j + 1] = r.info[1];
            }
            if (r.status == GW_BREAKDOWN) worst = GW_BREAKDOWN;
            else if (r.status != GW_OK && worst == GW_OK) worst = GW_NOT_CONVERGED;
        }
    return worst;
}

}  // namespace

int krylov_pcg_batch(amg_hierarchy *const *Hs, const double *const *b, double *const *x_out, int32_t nsys,
                     const amg_solve_params &sp, amg_solve_info *info, hipStream_t s) {
    return run_batch(0, Hs, b, nullptr, x_out, nullptr, nsys, sp, info, s);
}

int krylov_bicgstab2_batch(amg_hierarchy *const *Hs, const double *const *b0, const double *const *b1,
                           double *const *x0, double *const *x1, int32_t nsys, const amg_solve_params &sp,
                           amg_solve_info *info, hipStream_t s) {
    return run_batch(1, Hs, b0, b1, x0, x1, nsys, sp, info, s);
}

}  // namespace gw
