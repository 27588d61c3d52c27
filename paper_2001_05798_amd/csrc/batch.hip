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

template <class A>
void launch_seg(const void *table, int nseg, unsigned nblk, hipStream_t s) {
    hipLaunchKernelGGL(k_seg<A>, dim3(nblk), dim3(kBlock), 0, s, static_cast<const Seg<A> *>(table), nseg);
}

struct Plan {
    std::vector<unsigned char> host;
    DBuf<unsigned char> dev;

    template <class A>
    void add(Seq &q, const std::vector<std::pair<A, unsigned>> &recs, int kid, double bytes) {
        static_assert(std::is_trivially_copyable<Seg<A>>::value, "records are copied as bytes");
        if (recs.empty()) return;
        const size_t off = (host.size() + 255) / 256 * 256;
        host.resize(off + recs.size() * sizeof(Seg<A>));
        uint32_t blk = 0;
        for (size_t k = 0; k < recs.size(); ++k) {
            const Seg<A> sg{recs[k].first, blk, recs[k].second};
            std::memcpy(host.data() + off + k * sizeof(Seg<A>), &sg, sizeof(Seg<A>));
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

template <class F>
void with_l0(const Level &L0, F &&f) {
    if (L0.As.built()) f(OpSell<double>{view(L0.As), L0.As.val.p});
    else with_csr<double>(L0.A, L0.A.val.p, f);
}

// ---------------------------------------------------- V-cycle recording ---
// The kernel steps of one V-cycle of every system in `act` from level l down,
// in the order vcycle_level launches them for one system: b[j] the system's
// right-hand side at this level (type Bt), out[j] where its result goes
// (type Zt; null: the level's own buffer).  Returns each system's result.
template <class V, class Bt, class Zt, int NR>
std::vector<void *> rec_vcycle(Plan &P, Seq &q, std::vector<Sys> &S, const std::vector<int> &act, int l,
                               const std::vector<const Bt *> &b, const std::vector<Zt *> &out) {
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
    for (int a : fine) {
        Level &Lv = S[act[a]].H->L[l];
        const int64_t n = Lv.A.n;
        const double abytes = op_bytes(Lv.A, Lv.As, vb);
        with_level_op<V>(Lv, [&](auto op) {
            using OP = decltype(op);
            B.put(SmoothFirstK<OP, V, Bt, V, NR>{n, op, LevelOps<V>::mval(Lv), b[a], x[a], npre >= 2 ? 1 : 0,
                                                  S[act[a]].done},
                  grid_rows(n, OP::G), (npre >= 2 ? abytes : 0.0) + n * (double)vb + nr * n * (double)(sizeof(Bt) + vb));
        });
    }
    B.emit(P, q, level_kid(K_SMOOTH_FIRST0, l));
    auto sweep = [&](auto yout_of) {
        for (int a : fine) {
            Level &Lv = S[act[a]].H->L[l];
            const int64_t n = Lv.A.n;
            const double abytes = op_bytes(Lv.A, Lv.As, vb);
            auto *yo = yout_of(a);
            using YT = std::remove_pointer_t<decltype(yo)>;
            with_level_op<V>(Lv, [&](auto op) {
                using OP = decltype(op);
                B.put(SmoothK<OP, V, Bt, V, YT, NR>{n, op, LevelOps<V>::mval(Lv), b[a], x[a], yo, S[act[a]].done},
                      grid_rows(n, OP::G), abytes + n * (double)vb + nr * n * (double)(sizeof(Bt) + vb + sizeof(YT)));
            });
        }
        B.emit(P, q, level_kid(K_SMOOTH0, l));
    };
    for (int k = 2; k < npre; ++k) {
        sweep([&](int a) { return t[a]; });
        for (int a : fine) std::swap(x[a], t[a]);
    }
    // residual, then restriction
    std::vector<V *> bnext(act.size(), nullptr);
    for (int a : fine) bnext[a] = reinterpret_cast<V *>(S[act[a]].H->L[l + 1].vb.p);
    for (int a : fine) {
        Level &Lv = S[act[a]].H->L[l];
        const int64_t n = Lv.A.n;
        const double abytes = op_bytes(Lv.A, Lv.As, vb);
        with_level_op<V>(Lv, [&](auto op) {
            using OP = decltype(op);
            B.put(ResidualK<OP, V, Bt, V, V, NR>{n, op, b[a], x[a], t[a], S[act[a]].done}, grid_rows(n, OP::G),
                  abytes + nr * n * (double)(sizeof(Bt) + 2 * vb));
        });
    }
    B.emit(P, q, level_kid(K_RESIDUAL0, l));
    for (int a : fine) {
        Level &Lv = S[act[a]].H->L[l];
        const int64_t n = Lv.A.n, nc = Lv.nc;
        with_csr<V>(Lv.R, LevelOps<V>::rval(Lv), [&](auto op) {
            using OP = decltype(op);
            B.put(SpmvK<OP, V, V, V, NR>{nc, op, t[a], bnext[a], S[act[a]].done},
                  grid_rows(nc, OP::G), csr_bytes(nc, Lv.R.nnz, vb) + nr * (double)(n + nc) * vb);
        });
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
    std::vector<void *> xc = rec_vcycle<V, V, V, NR>(P, q, S, act2, l + 1, b2, o2);
    for (size_t k = 0; k < fine.size(); ++k) {
        const int a = fine[k];
        Level &Lv = S[act[a]].H->L[l];
        const int64_t n = Lv.A.n, nc = Lv.nc;
        with_csr<V>(Lv.P, LevelOps<V>::pval(Lv), [&](auto op) {
            using OP = decltype(op);
            B.put(ProlongK<OP, V, V, NR>{n, op, static_cast<const V *>(xc[k]), x[a], S[act[a]].done},
                  grid_rows(n, OP::G), csr_bytes(n, Lv.P.nnz, vb) + nr * (double)(2 * n + nc) * vb);
        });
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

void check_batch(amg_hierarchy *const *Hs, int32_t nsys, const char *who) {
    GW_REQUIRE(nsys >= 1 && nsys <= 256, std::string(who) + ": nsys must be in [1, 256]");
    GW_REQUIRE(Hs, std::string(who) + ": null hierarchy list");
    const amg_params &p0 = Hs[0] ? Hs[0]->prm : amg_params{};
    for (int j = 0; j < nsys; ++j) {
        const amg_hierarchy *H = Hs[j];
        GW_REQUIRE(H, std::string(who) + ": null hierarchy");
        for (int k = 0; k < j; ++k) GW_REQUIRE(Hs[k] != H, std::string(who) + ": a hierarchy appears twice");
        GW_REQUIRE(H->nlev >= 1 && H->prm.smoother != GW_SMOOTHER_ILU0,
                   std::string(who) + ": every system needs a diagonal-smoother AMG preconditioner");
        GW_REQUIRE(H->prm.npre >= 1 && H->prm.npost >= 1,
                   std::string(who) + ": shared launches need at least one pre- and one post-sweep");
        GW_REQUIRE(H->prm.precision == p0.precision && H->prm.npre == p0.npre && H->prm.npost == p0.npost,
                   std::string(who) + ": the systems must share precision and sweep counts");
    }
}

void read_all(const DBuf<KScalars> &ks, Pinned &stage, std::vector<KScalars> &h, hipStream_t s) {
    const size_t bytes = h.size() * sizeof(KScalars);
    GW_HIP(hipMemcpyAsync(stage.p, ks.p, bytes, hipMemcpyDeviceToHost, s));
    GW_HIP(hipStreamSynchronize(s));
    std::memcpy(h.data(), stage.p, bytes);
}

void write_all(DBuf<KScalars> &ks, Pinned &stage, const std::vector<KScalars> &h, hipStream_t s) {
    const size_t bytes = h.size() * sizeof(KScalars);
    std::memcpy(stage.p, h.data(), bytes);
    GW_HIP(hipMemcpyAsync(ks.p, stage.p, bytes, hipMemcpyHostToDevice, s));
    GW_HIP(hipStreamSynchronize(s));
}

// Blocks of `cnt` iterations: the recorded launches one by one, or a HIP
// graph captured once per (parity, cnt) for this batch.
struct Runner {
    const Plan &P;
    bool graph;
    hipStream_t cap = nullptr;
    struct G {
        int parity, cnt;
        hipGraphExec_t ex;
    };
    std::vector<G> graphs;
    ~Runner() {
        for (auto &g : graphs) (void)hipGraphExecDestroy(g.ex);
        if (cap) (void)hipStreamDestroy(cap);
    }
    void block(const Seq (&iter)[2], int parity, int cnt, hipStream_t s) {
        auto emit = [&](hipStream_t cs) {
            int par = parity;
            for (int c = 0; c < cnt; ++c) {
                P.run(iter[par], cs);
                par ^= iter[1].empty() ? 0 : 1;
            }
        };
        if (!graph) {
            emit(s);
            return;
        }
        hipGraphExec_t ex = nullptr;
        for (auto &g : graphs)
            if (g.parity == parity && g.cnt == cnt) ex = g.ex;
        if (!ex) {
            if (!cap) GW_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
            GW_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
            hipGraph_t g = nullptr;
            try {
                emit(cap);
            } catch (...) {
                if (hipStreamEndCapture(cap, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
                throw;
            }
            GW_HIP(hipStreamEndCapture(cap, &g));
            const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            GW_HIP(e);
            graphs.push_back({parity, cnt, ex});
        }
        GW_HIP(hipGraphLaunch(ex, s));
    }
};

}  // namespace

// ------------------------------------------------------------- CG batch ---
int krylov_pcg_batch(amg_hierarchy *const *Hs, const double *const *b, double *const *x_out, int32_t nsys,
                     const amg_solve_params &sp, amg_solve_info *info, hipStream_t s) {
    check_batch(Hs, nsys, "amg_solve_pcg_batch");
    const double t0 = ms_now();
    const bool mixed = Hs[0]->mixed();
    const int flexible = sp.flexible < 0 ? (mixed ? 1 : 0) : (sp.flexible ? 1 : 0);
    std::vector<Sys> S(nsys);
    DBuf<KScalars> ks((size_t)nsys);
    Pinned stage((size_t)nsys * sizeof(KScalars));
    std::vector<double *> r(nsys), z(nsys), pa(nsys), pb(nsys), q(nsys), x(nsys);
    for (int j = 0; j < nsys; ++j) {
        amg_hierarchy *H = Hs[j];
        ensure_krylov_workspace(H, 6);
        const Level &L0 = H->L[0];
        Sys &y = S[j];
        y.H = H;
        y.n = L0.A.n;
        const int G = L0.As.built() ? 1 : L0.A.grp;
        y.g1 = kgrid(y.n, 1);
        y.gG = kgrid(y.n, G);
        y.part = H->partials.p;
        y.ks = ks.p + j;
        y.done = &ks.p[j].done;
        y.abytes = op_bytes(L0.A, L0.As, 8);
        r[j] = H->kvec.p;
        z[j] = r[j] + y.n;
        pa[j] = z[j] + y.n;
        pb[j] = pa[j] + y.n;
        q[j] = pb[j] + y.n;
        x[j] = q[j] + y.n;
    }
    std::vector<int> all(nsys);
    for (int j = 0; j < nsys; ++j) all[j] = j;
    std::vector<unsigned> nb1(nsys), nbG(nsys);
    for (int j = 0; j < nsys; ++j) nb1[j] = S[j].g1, nbG[j] = S[j].gG;

    // the recorded sequences
    Plan P;
    Seq init_first, first_z, iter[2], tres;
    {
        Buckets B;
        for (int j = 0; j < nsys; ++j)
            with_l0(S[j].H->L[0], [&](auto o) {
                using OP = decltype(o);
                B.put(KrInitK<OP>{S[j].n, o, b[j], x[j], r[j], nullptr, pa[j], nullptr, S[j].part}, S[j].gG,
                      S[j].abytes + 4 * 8.0 * S[j].n);
            });
        B.emit(P, init_first, K_KRYLOV_SPMV);
        rec_fin(P, init_first, S, all, FIN_INIT_FIRST, false, sp.rtol, nbG);
    }
    auto rec_z_dot_beta = [&](Seq &qq, int fin) {
        std::vector<const double *> rin(r.begin(), r.end());
        rec_precond<1>(P, qq, S, all, rin, z, mixed);
        Buckets B;
        for (int j = 0; j < nsys; ++j)
            B.put(CgDotK{S[j].n, r[j], z[j], q[j], S[j].part, S[j].ks}, S[j].g1, 3 * 8.0 * S[j].n);
        B.emit(P, qq, K_KRYLOV_DOT);
        rec_fin(P, qq, S, all, fin, false, sp.rtol, nb1);
    };
    rec_z_dot_beta(first_z, FIN_CG_BETA_FIRST);
    for (int par = 0; par < 2; ++par) {
        Seq &qq = iter[par];
        Buckets B;
        for (int j = 0; j < nsys; ++j) {
            double *po = par ? pb[j] : pa[j], *pn = par ? pa[j] : pb[j];
            with_l0(S[j].H->L[0], [&](auto o) {
                using OP = decltype(o);
                B.put(CgSpmvK<OP>{S[j].n, o, z[j], po, pn, q[j], S[j].part, S[j].ks}, S[j].gG,
                      S[j].abytes + 4 * 8.0 * S[j].n);
            });
        }
        B.emit(P, qq, K_KRYLOV_SPMV);
        rec_fin(P, qq, S, all, FIN_CG_ALPHA, false, sp.rtol, nbG);
        for (int j = 0; j < nsys; ++j) {
            double *pn = par ? pa[j] : pb[j];
            B.put(CgUpdateK{S[j].n, x[j], r[j], pn, q[j], S[j].part, S[j].ks}, S[j].g1, 6 * 8.0 * S[j].n);
        }
        B.emit(P, qq, K_KRYLOV_UPDATE);
        rec_fin(P, qq, S, all, FIN_CG_CONV, false, sp.rtol, nb1);
        rec_z_dot_beta(qq, FIN_CG_BETA);
    }
    {
        Buckets B;
        for (int j = 0; j < nsys; ++j)
            with_l0(S[j].H->L[0], [&](auto o) {
                using OP = decltype(o);
                B.put(TrueResK<OP>{S[j].n, o, b[j], x[j], S[j].part}, S[j].gG, S[j].abytes + 2 * 8.0 * S[j].n);
            });
        B.emit(P, tres, K_TRUE_RESIDUAL);
        rec_fin(P, tres, S, all, FIN_TRUE_RES, false, sp.rtol, nbG);
    }
    P.upload(s);

    std::vector<KScalars> k(nsys);
    for (int j = 0; j < nsys; ++j) {
        k[j] = KScalars{};
        k[j].maxiter = std::max(0, sp.maxiter);
        k[j].flexible = flexible;
        k[j].status = GW_NOT_CONVERGED;
    }
    write_all(ks, stage, k, s);
    for (int j = 0; j < nsys; ++j) fill_f64(x[j], 0.0, S[j].n, s);
    P.run(init_first, s);
    read_all(ks, stage, k, s);
    std::vector<int> final(nsys, 0), restarts(nsys, 0), status(nsys, GW_NOT_CONVERGED);
    bool any_zero = false;
    for (int j = 0; j < nsys; ++j)
        if (k[j].bnorm == 0.0) {
            // b = 0: x = 0, nothing to iterate
            final[j] = 1;
            status[j] = GW_OK;
            k[j].done = 1;
            k[j].iters = 0;
            k[j].rr = 0.0;
            k[j].rel_true = 0.0;
            any_zero = true;
        }
    if (any_zero) write_all(ks, stage, k, s);
    const int check = std::max(1, sp.check_every);
    Runner run{P, sp.graph > 0};
    int parity = 0;
    std::vector<KScalars> kfinal(k);
    Plan Prestart;  // tables of restarts (rare), built when needed
    for (;;) {
        bool any = false;
        for (int j = 0; j < nsys; ++j) any |= !final[j] && !k[j].done;
        if (any) {
            P.run(first_z, s);
            std::vector<PollPlan> plans(nsys, PollPlan{check, sp.graph > 0});
            int cnt = check;
            for (;;) {
                run.block(iter, parity, cnt, s);
                parity ^= cnt & 1;
                read_all(ks, stage, k, s);
                bool all_done = true;
                int c2 = 1;
                for (int j = 0; j < nsys; ++j) {
                    const int cj = plans[j].next(std::sqrt(k[j].rr), k[j].tol, k[j].iters);
                    if (!k[j].done) {
                        all_done = false;
                        c2 = std::max(c2, cj);
                    }
                }
                if (all_done) break;
                cnt = c2;
            }
        }
        P.run(tres, s);
        read_all(ks, stage, k, s);
        std::vector<int> again;
        for (int j = 0; j < nsys; ++j) {
            if (final[j]) continue;
            KScalars &kj = k[j];
            if (kj.status == GW_BREAKDOWN) status[j] = GW_BREAKDOWN, final[j] = 1;
            else if (kj.rel_true <= sp.rtol) status[j] = GW_OK, final[j] = 1;
            else if (kj.iters >= kj.maxiter || restarts[j] >= 8) status[j] = GW_NOT_CONVERGED, final[j] = 1;
            else again.push_back(j);
            if (final[j]) kfinal[j] = kj;
        }
        if (again.empty()) break;
        // restart the systems in `again` from their iterate: r = b - A x
        parity = 0;
        Prestart = Plan();
        Seq init_re;
        {
            Buckets B;
            std::vector<unsigned> nb;
            for (int j : again) {
                ++restarts[j];
                with_l0(S[j].H->L[0], [&](auto o) {
                    using OP = decltype(o);
                    B.put(KrInitK<OP>{S[j].n, o, b[j], x[j], r[j], nullptr, pa[j], nullptr, S[j].part}, S[j].gG, 0.0);
                });
                nb.push_back(S[j].gG);
            }
            B.emit(Prestart, init_re, K_KRYLOV_SPMV);
            rec_fin(Prestart, init_re, S, again, FIN_INIT_RESTART, false, sp.rtol, nb);
        }
        Prestart.upload(s);
        Prestart.run(init_re, s);
        read_all(ks, stage, k, s);
        // systems already final keep done = 1 and skip every launch
    }
    for (int j = 0; j < nsys; ++j) copy_bytes(x_out[j], x[j], sizeof(double) * (size_t)S[j].n, s);
    GW_HIP(hipStreamSynchronize(s));
    const double ms = ms_now() - t0;
    int worst = GW_OK;
    for (int j = 0; j < nsys; ++j) {
        const KScalars &q1 = kfinal[j];
        if (info) {
            info[j].iters = q1.iters;
            info[j].status = status[j];
            info[j].restarts = restarts[j];
            info[j].rel_res = q1.bnorm != 0.0 ? std::sqrt(q1.rr) / q1.bnorm : 0.0;
            info[j].rel_res_true = q1.bnorm != 0.0 ? q1.rel_true : 0.0;
            info[j].setup_ms = 0.0;
            info[j].solve_ms = ms;
        }
        if (status[j] == GW_BREAKDOWN) worst = GW_BREAKDOWN;
        else if (status[j] != GW_OK && worst == GW_OK) worst = GW_NOT_CONVERGED;
    }
    return worst;
}

// -------------------------------------------------- BiCGSTAB pair batch ---
int krylov_bicgstab2_batch(amg_hierarchy *const *Hs, const double *const *b0, const double *const *b1,
                           double *const *x0, double *const *x1, int32_t nsys, const amg_solve_params &sp,
                           amg_solve_info *info, hipStream_t s) {
    check_batch(Hs, nsys, "amg_solve_bicgstab_pair_batch");
    const double t0 = ms_now();
    const bool mixed = Hs[0]->mixed();
    std::vector<Sys> S(nsys);
    DBuf<KScalars> ks((size_t)nsys * 3);
    Pinned stage((size_t)nsys * 3 * sizeof(KScalars));
    struct V10 {
        double *b, *r, *rh, *p, *v, *sv, *t, *ph, *sh, *x;
    };
    std::vector<V10> w(nsys);
    for (int j = 0; j < nsys; ++j) {
        amg_hierarchy *H = Hs[j];
        ensure_krylov_workspace(H, 20);
        ensure_level_vectors(H, 2);
        const Level &L0 = H->L[0];
        Sys &y = S[j];
        y.H = H;
        y.n = L0.A.n;
        const int G = L0.As.built() ? 1 : L0.A.grp;
        y.g1 = kgrid(y.n, 1);
        y.gG = kgrid(y.n, G);
        y.part = H->partials.p;
        y.ks = ks.p + 3 * j;
        y.done = &ks.p[3 * j + 2].done;
        y.abytes = op_bytes(L0.A, L0.As, 8);
        const int64_t n2 = 2 * y.n;
        double *base = H->kvec.p;
        w[j] = V10{base, base + n2, base + 2 * n2, base + 3 * n2, base + 4 * n2, base + 5 * n2, base + 6 * n2,
                   base + 7 * n2, base + 8 * n2, base + 9 * n2};
    }
    std::vector<int> all(nsys);
    for (int j = 0; j < nsys; ++j) all[j] = j;
    std::vector<unsigned> nb1(nsys), nbG(nsys);
    for (int j = 0; j < nsys; ++j) nb1[j] = S[j].g1, nbG[j] = S[j].gG;

    Plan P;
    Seq init_first, iter[2], tres, split;
    {
        Buckets B;
        for (int j = 0; j < nsys; ++j)
            B.put(InterleaveK{S[j].n, b0[j], b1[j], w[j].b}, S[j].g1, 4 * 8.0 * S[j].n);
        B.emit(P, init_first, -1);
        for (int j = 0; j < nsys; ++j)
            with_l0(S[j].H->L[0], [&](auto o) {
                using OP = decltype(o);
                B.put(KrInit2K<OP>{S[j].n, o, w[j].b, w[j].x, w[j].r, w[j].rh, w[j].p, w[j].v, S[j].part, 3},
                      S[j].gG, S[j].abytes + 7 * 16.0 * S[j].n);
            });
        B.emit(P, init_first, K_KRYLOV_SPMV);
        rec_fin(P, init_first, S, all, FIN_INIT_FIRST, true, sp.rtol, nbG);
    }
    {
        Seq &qq = iter[0];
        Buckets B;
        for (int j = 0; j < nsys; ++j) B.put(BcgP2K{S[j].n, w[j].r, w[j].p, w[j].v, S[j].ks}, S[j].g1, 4 * 16.0 * S[j].n);
        B.emit(P, qq, K_KRYLOV_UPDATE);
        {
            std::vector<const double *> in(nsys);
            std::vector<double *> out(nsys);
            for (int j = 0; j < nsys; ++j) in[j] = w[j].p, out[j] = w[j].ph;
            rec_precond<2>(P, qq, S, all, in, out, mixed);
        }
        for (int j = 0; j < nsys; ++j)
            with_l0(S[j].H->L[0], [&](auto o) {
                using OP = decltype(o);
                B.put(BcgV2K<OP>{S[j].n, o, w[j].ph, w[j].v, w[j].rh, S[j].part, S[j].ks}, S[j].gG,
                      S[j].abytes + 3 * 16.0 * S[j].n);
            });
        B.emit(P, qq, K_KRYLOV_SPMV);
        rec_fin(P, qq, S, all, FIN_BCG_ALPHA, true, sp.rtol, nbG);
        for (int j = 0; j < nsys; ++j)
            B.put(BcgS2K{S[j].n, w[j].r, w[j].v, w[j].sv, S[j].part, S[j].ks}, S[j].g1, 3 * 16.0 * S[j].n);
        B.emit(P, qq, K_KRYLOV_UPDATE);
        rec_fin(P, qq, S, all, FIN_BCG_S, true, sp.rtol, nb1);
        {
            std::vector<const double *> in(nsys);
            std::vector<double *> out(nsys);
            for (int j = 0; j < nsys; ++j) in[j] = w[j].sv, out[j] = w[j].sh;
            rec_precond<2>(P, qq, S, all, in, out, mixed);
        }
        for (int j = 0; j < nsys; ++j)
            with_l0(S[j].H->L[0], [&](auto o) {
                using OP = decltype(o);
                B.put(BcgT2K<OP>{S[j].n, o, w[j].sh, w[j].t, w[j].sv, S[j].part, S[j].ks}, S[j].gG,
                      S[j].abytes + 3 * 16.0 * S[j].n);
            });
        B.emit(P, qq, K_KRYLOV_SPMV);
        rec_fin(P, qq, S, all, FIN_BCG_OMEGA, true, sp.rtol, nbG);
        for (int j = 0; j < nsys; ++j)
            B.put(BcgXr2K{S[j].n, w[j].x, w[j].r, w[j].ph, w[j].sh, w[j].sv, w[j].t, w[j].rh, S[j].part, S[j].ks},
                  S[j].g1, 8 * 16.0 * S[j].n);
        B.emit(P, qq, K_KRYLOV_UPDATE);
        rec_fin(P, qq, S, all, FIN_BCG_XR, true, sp.rtol, nb1);
    }
    {
        Buckets B;
        for (int j = 0; j < nsys; ++j)
            with_l0(S[j].H->L[0], [&](auto o) {
                using OP = decltype(o);
                B.put(TrueRes2K<OP>{S[j].n, o, w[j].b, w[j].x, S[j].part}, S[j].gG, S[j].abytes + 2 * 16.0 * S[j].n);
            });
        B.emit(P, tres, K_TRUE_RESIDUAL);
        rec_fin(P, tres, S, all, FIN_TRUE_RES, true, sp.rtol, nbG);
        for (int j = 0; j < nsys; ++j) B.put(SplitK{S[j].n, w[j].x, x0[j], x1[j]}, S[j].g1, 4 * 8.0 * S[j].n);
        B.emit(P, split, -1);
    }
    P.upload(s);

    std::vector<KScalars> k((size_t)nsys * 3);
    for (int j = 0; j < nsys; ++j)
        for (int c = 0; c < 3; ++c) {
            KScalars &q1 = k[3 * j + c];
            q1 = KScalars{};
            if (c < 2) {
                q1.maxiter = std::max(0, sp.maxiter);
                q1.status = GW_NOT_CONVERGED;
            }
        }
    write_all(ks, stage, k, s);
    for (int j = 0; j < nsys; ++j) fill_f64(w[j].x, 0.0, 2 * S[j].n, s);
    P.run(init_first, s);
    read_all(ks, stage, k, s);
    std::vector<int> final((size_t)nsys * 2, 0), restarts((size_t)nsys * 2, 0), status((size_t)nsys * 2, GW_NOT_CONVERGED);
    bool any_zero = false;
    for (int j = 0; j < nsys; ++j) {
        for (int c = 0; c < 2; ++c) {
            KScalars &q1 = k[3 * j + c];
            if (q1.bnorm != 0.0) continue;
            final[2 * j + c] = 1;
            status[2 * j + c] = GW_OK;
            q1.done = 1;
            q1.iters = 0;
            q1.rr = 0.0;
            q1.rel_true = 0.0;
            any_zero = true;
        }
        k[3 * j + 2].done = k[3 * j].done && k[3 * j + 1].done;
    }
    if (any_zero) write_all(ks, stage, k, s);
    const int check = std::max(1, sp.check_every);
    iter[1].clear();  // one sequence: no parity
    Runner run{P, sp.graph > 0};
    std::vector<KScalars> kfinal(k);
    Plan Prestart;
    for (;;) {
        std::vector<PollPlan> plans((size_t)nsys * 2, PollPlan{check, sp.graph > 0});
        int cnt = check;
        for (;;) {
            bool all_done = true;
            for (int j = 0; j < nsys; ++j) all_done &= k[3 * j + 2].done != 0;
            if (all_done) break;
            run.block(iter, 0, cnt, s);
            read_all(ks, stage, k, s);
            int c2 = 1;
            for (int j = 0; j < nsys; ++j)
                for (int c = 0; c < 2; ++c) {
                    const KScalars &q1 = k[3 * j + c];
                    const int cq = plans[2 * j + c].next(std::sqrt(q1.rr), q1.tol, q1.iters);
                    if (!q1.done) c2 = std::max(c2, cq);
                }
            cnt = c2;
        }
        P.run(tres, s);
        read_all(ks, stage, k, s);
        std::vector<int> again;
        std::vector<int> masks;
        for (int j = 0; j < nsys; ++j) {
            int mask = 0;
            for (int c = 0; c < 2; ++c) {
                const int e = 2 * j + c;
                if (final[e]) continue;
                const KScalars &q1 = k[3 * j + c];
                if (q1.status == GW_BREAKDOWN) status[e] = GW_BREAKDOWN, final[e] = 1;
                else if (q1.rel_true <= sp.rtol) status[e] = GW_OK, final[e] = 1;
                else if (q1.iters >= q1.maxiter || restarts[e] >= 8) status[e] = GW_NOT_CONVERGED, final[e] = 1;
                else {
                    ++restarts[e];
                    mask |= 1 << c;
                }
                if (final[e]) kfinal[3 * j + c] = q1;
            }
            if (mask) again.push_back(j), masks.push_back(mask);
        }
        if (again.empty()) break;
        Prestart = Plan();
        Seq init_re;
        {
            Buckets B;
            std::vector<unsigned> nb;
            for (size_t a = 0; a < again.size(); ++a) {
                const int j = again[a];
                with_l0(S[j].H->L[0], [&](auto o) {
                    using OP = decltype(o);
                    B.put(KrInit2K<OP>{S[j].n, o, w[j].b, w[j].x, w[j].r, w[j].rh, w[j].p, w[j].v, S[j].part,
                                       masks[a]},
                          S[j].gG, 0.0);
                });
                nb.push_back(S[j].gG);
            }
            B.emit(Prestart, init_re, K_KRYLOV_SPMV);
            // one finalize per system, each with its own mask
            for (size_t a = 0; a < again.size(); ++a) {
                const int j = again[a];
                B.put(Fin2K{FIN_INIT_RESTART, nb[a], S[j].part, sp.rtol, S[j].ks, masks[a]}, 1u, 0.0);
            }
            B.emit(Prestart, init_re, -1);
        }
        Prestart.upload(s);
        Prestart.run(init_re, s);
        read_all(ks, stage, k, s);
    }
    P.run(split, s);
    GW_HIP(hipStreamSynchronize(s));
    const double ms = ms_now() - t0;
    int worst = GW_OK;
    for (int j = 0; j < nsys; ++j)
        for (int c = 0; c < 2; ++c) {
            const int e = 2 * j + c;
            const KScalars &q1 = kfinal[3 * j + c];
            if (info) {
                info[e].iters = q1.iters;
                info[e].status = status[e];
                info[e].restarts = restarts[e];
                info[e].rel_res = q1.bnorm != 0.0 ? std::sqrt(q1.rr) / q1.bnorm : 0.0;
                info[e].rel_res_true = q1.bnorm != 0.0 ? q1.rel_true : 0.0;
                info[e].setup_ms = 0.0;
                info[e].solve_ms = ms;
            }
            if (status[e] == GW_BREAKDOWN) worst = GW_BREAKDOWN;
            else if (status[e] != GW_OK && worst == GW_OK) worst = GW_NOT_CONVERGED;
        }
    return worst;
}

}  // namespace gw
