// Batched solves of many structured problems (amgmpcg_setup_batched).
#include "host_common.hpp"
#include "grid_kernels.hpp"
#include "batched.hpp"
#include "batched_layout.hpp"
#include "batched_persistent.hpp"

namespace amg {

// ------------------------------------------------------------------ batched


template <typename T, int DIM>
class BatchedSolver : public BatchedBase {
   public:
    BatchedSolver(int cnt, const amgmpcg_grid* grids, const amgmpcg_options& o, hipStream_t stream)
        : opt_(o), stream_(stream) {
        count = cnt;
        mixed_ = std::is_same<T, float>::value;
        std::vector<int> ns(cnt), nls(cnt);
        for (int i = 0; i < cnt; ++i) {
            ns[i] = grids[i].n;
            nls[i] = grids[i].nlevels;
        }
        const host::BatchLayout lay = host::batch_layout(DIM, ns, nls, kBChunk, kBlock, kBPartRows);
        offs_ = lay.offs;
        nlev_ = nls;
        pos_ = lay.pos;
        total = (int64_t)offs_[cnt];
        x_.alloc(offs_[cnt]);
        r_.alloc(offs_[cnt]);
        b_.alloc(offs_[cnt]);
        P_.alloc(lay.nP);
        Q_.alloc(lay.nP);
        cL_.alloc(offs_[cnt]);
        coef_.alloc(std::max<size_t>(lay.ncoef, 1));
        g_.alloc(std::max<size_t>(lay.nvec, 1));
        c1_.alloc(std::max<size_t>(lay.nvec, 1));
        Y_.alloc(std::max<size_t>(lay.nY, 1));
        HIPCHK(hipMemset(P_.p, 0, P_.n * sizeof(T)));
        HIPCHK(hipMemset(Q_.p, 0, Q_.n * sizeof(T)));
        HIPCHK(hipMemset(Y_.p, 0, Y_.n * sizeof(T)));
        for (const host::BatchGroup& G : lay.groups) {
            groups_.push_back(Group{G.nlev, G.first, G.count, Range{G.fine.off, G.fine.cnt}});
        }
        ctl_.alloc(cnt);
        small_.alloc((size_t)cnt * kBSmall);
        HIPCHK(hipMemset(small_.p, 0, small_.n * sizeof(double)));
        part_.alloc(lay.npart);

        // per-problem hierarchy (host Galerkin) and device pointers
        hinst_.resize(cnt);
        std::vector<T> coef_host(lay.ncoef);
        for (int q = 0; q < cnt; ++q) {
            const host::BatchProblem& B = lay.inst[q];
            const int nl = B.nlev, n = B.n[nl - 1];
            BInst<T>& I = hinst_[q];
            std::memset(&I, 0, sizeof(I));
            I.nlev = nl;
            for (int l = 0; l < nl; ++l) {
                I.n[l] = B.n[l];
                I.N[l] = (int)B.N[l];
            }
            const int N = (int)B.N[nl - 1];
            const double h2inv = double(n + 1) * double(n + 1);
            I.op.n = n;
            I.op.N = N;
            I.op.s0 = T(h2inv);
            I.op.inv0 = T(1.0 / (2.0 * DIM * h2inv));
            I.op64.n = n;
            I.op64.N = N;
            I.op64.s0 = h2inv;
            I.op64.inv0 = 1.0 / (2.0 * DIM * h2inv);
            I.x = x_.p + B.fine_off;
            I.r = r_.p + B.fine_off;
            I.b = b_.p + B.fine_off;
            I.cL = cL_.p + B.fine_off;
            I.P = P_.p + B.P_off;
            I.Q = Q_.p + B.P_off;
            I.ctl = ctl_.p + q;
            I.small = small_.p + (size_t)q * kBSmall;
            I.part = part_.p + B.part_off;
            I.pcnt = B.pcnt;
            if (nl > 1) {
                host::FineFaces faces = host::fine_faces(DIM, n, nullptr);
                std::vector<host::StencilLevel> lev(nl);
                lev[nl - 1] = host::faces_to_stencil(DIM, n, faces);
                for (int l = nl - 2; l >= 0; --l) {
                    lev[l] = host::galerkin(lev[l + 1]);
                    const int ctr = lev[l].center();
                    for (int64_t k = 0; k < lev[l].N; ++k)
                        if (!(lev[l].coef[(size_t)ctr * lev[l].N + k] > 0.0))
                            throw ApiError(AMGMPCG_NOT_SPD, "non-positive diagonal on a coarse level");
                }
                for (int l = 0; l + 1 < nl; ++l) {
                    const size_t cnt_c = (size_t)(DIM == 2 ? 9 : 27) * (size_t)B.N[l];
                    for (size_t k = 0; k < cnt_c; ++k) coef_host[B.coef_off[l] + k] = T(lev[l].coef[k]);
                    I.coef[l] = coef_.p + B.coef_off[l];
                    I.g[l] = g_.p + B.vec_off[l];
                    I.c1[l] = c1_.p + B.vec_off[l];
                    I.Y[l] = Y_.p + B.Y_off[l];
                }
            }
        }
        if (lay.ncoef) HIPCHK(hipMemcpy(coef_.p, coef_host.data(), lay.ncoef * sizeof(T), hipMemcpyHostToDevice));
        inst_.alloc(cnt);
        HIPCHK(hipMemcpy(inst_.p, hinst_.data(), cnt * sizeof(BInst<T>), hipMemcpyHostToDevice));

        // block maps (the same four ints per block as the kernels' BBlk)
        static_assert(sizeof(BBlk) == sizeof(host::BatchBlock), "block map entry layout");
        all_ = Range{lay.all.off, lay.all.cnt};
        dmax_ = lay.dmax;
        for (int d = 0; d < kMaxLevels; ++d) {
            dep_[d] = Range{lay.dep[d].off, lay.dep[d].cnt};
            pro_[d] = Range{lay.pro[d].off, lay.pro[d].cnt};
        }
        std::vector<BBlk> maps(lay.maps.size());
        for (size_t k = 0; k < maps.size(); ++k)
            maps[k] = BBlk{lay.maps[k].inst, lay.maps[k].blk, lay.maps[k].start, lay.maps[k].end};
        maps_.alloc(maps.size());
        HIPCHK(hipMemcpy(maps_.p, maps.data(), maps.size() * sizeof(BBlk), hipMemcpyHostToDevice));

        // persistent launch: the problems largest first (then in table order)
        std::vector<int> ord(cnt);
        for (int q = 0; q < cnt; ++q) ord[q] = q;
        std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
            return lay.inst[a].N[lay.inst[a].nlev - 1] > lay.inst[b].N[lay.inst[b].nlev - 1];
        });
        porder_.alloc(cnt);
        HIPCHK(hipMemcpy(porder_.p, ord.data(), cnt * sizeof(int), hipMemcpyHostToDevice));
        queue_.alloc(1);
        HIPCHK(hipMemset(queue_.p, 0, sizeof(int)));
        int dev = 0, cus = 0, per_cu = 0;
        HIPCHK(hipGetDevice(&dev));
        HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_b_persistent<DIM, T>, kPB, 0));
        pgrid_ = std::max(1, std::min(cnt, cus * std::max(1, per_cu)));
        HIPCHK(hipHostMalloc((void**)&hctl_, (size_t)cnt * sizeof(Ctl), hipHostMallocDefault));
        HIPCHK(hipEventCreate(&ev0_));
        HIPCHK(hipEventCreate(&ev1_));
        kpoll_ = opt_.k_poll;
    }

    ~BatchedSolver() override {
        if (exec_) (void)hipGraphExecDestroy(exec_);
        if (graph_) (void)hipGraphDestroy(graph_);
        if (pexec_) (void)hipGraphExecDestroy(pexec_);
        if (pgraph_) (void)hipGraphDestroy(pgraph_);
        if (cap_stream_) (void)hipStreamDestroy(cap_stream_);
        if (hctl_) (void)hipHostFree(hctl_);
        if (ev0_) (void)hipEventDestroy(ev0_);
        if (ev1_) (void)hipEventDestroy(ev1_);
    }

    int solve(const double* b_dev, double* x_dev, double tol, int maxit, amgmpcg_info* infos,
              double* batch_ms) override {
        if (maxit <= 0) maxit = opt_.maxit;
        const double unit = mixed_ ? std::ldexp(1.0, -24) : std::ldexp(1.0, -53);
        for (int i = 0; i < count; ++i) {
            Ctl& c = hctl_[pos_[i]];
            std::memset(&c, 0, sizeof(Ctl));
            c.maxit = maxit;
            c.drop2 = opt_.refresh_drop * opt_.refresh_drop;
            c.tau = opt_.pinv_tau > 0 ? opt_.pinv_tau : 64.0 * nlev_[i] * unit;
            c.tol = tol;
        }
        const size_t nbytes = (size_t)offs_[count] * sizeof(double);
        if (opt_.persistent) return solve_persistent(b_dev, x_dev, nbytes, infos, batch_ms);
        HIPCHK(hipEventRecord(ev0_, stream_));
        HIPCHK(hipMemcpyAsync(ctl_.p, hctl_, (size_t)count * sizeof(Ctl), hipMemcpyHostToDevice, stream_));
        HIPCHK(hipMemcpyAsync(b_.p, b_dev, nbytes, hipMemcpyDeviceToDevice, stream_));
        HIPCHK(hipMemcpyAsync(x_.p, x_dev, nbytes, hipMemcpyDeviceToDevice, stream_));
        enqueue_init(stream_, tol);
        HIPCHK(hipGetLastError());
        if (!exec_) capture();
        const int launches_max = maxit / kpoll_ + 3;
        for (int launch = 0; launch < launches_max; ++launch) {
            HIPCHK(hipMemcpyAsync(hctl_, ctl_.p, (size_t)count * sizeof(Ctl), hipMemcpyDeviceToHost, stream_));
            HIPCHK(hipStreamSynchronize(stream_));
            bool all = true;
            for (int q = 0; q < count && all; ++q) all = hctl_[q].state == 2;
            if (all) break;
            HIPCHK(hipGraphLaunch(exec_, stream_));
        }
        HIPCHK(hipMemcpyAsync(x_dev, x_.p, nbytes, hipMemcpyDeviceToDevice, stream_));
        HIPCHK(hipEventRecord(ev1_, stream_));
        HIPCHK(hipMemcpyAsync(hctl_, ctl_.p, (size_t)count * sizeof(Ctl), hipMemcpyDeviceToHost, stream_));
        HIPCHK(hipStreamSynchronize(stream_));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, ev0_, ev1_));
        return finish(infos, batch_ms, ms);
    }

   private:
    // One persistent launch (with the reset of its queue) for the whole
    // solve: captured once into a graph and launched once per solve.
    int solve_persistent(const double* b_dev, double* x_dev, size_t nbytes, amgmpcg_info* infos, double* batch_ms) {
        if (!pexec_) {
            if (!cap_stream_) HIPCHK(hipStreamCreateWithFlags(&cap_stream_, hipStreamNonBlocking));
            HIPCHK(hipStreamBeginCapture(cap_stream_, hipStreamCaptureModeThreadLocal));
            k_b_reset_queue<<<1, 64, 0, cap_stream_>>>(queue_.p);
            k_b_persistent<DIM, T><<<pgrid_, kPB, 0, cap_stream_>>>(inst_.p, porder_.p, count, queue_.p,
                                                                     T(opt_.omega), opt_.nu >= 2 ? 1 : 0,
                                                                     mixed_ ? 1 : 0);
            hipError_t launch_err = hipGetLastError();
            HIPCHK(hipStreamEndCapture(cap_stream_, &pgraph_));
            HIPCHK(launch_err);
            HIPCHK(hipGraphInstantiate(&pexec_, pgraph_, nullptr, nullptr, 0));
        }
        HIPCHK(hipEventRecord(ev0_, stream_));
        HIPCHK(hipMemcpyAsync(ctl_.p, hctl_, (size_t)count * sizeof(Ctl), hipMemcpyHostToDevice, stream_));
        HIPCHK(hipMemcpyAsync(b_.p, b_dev, nbytes, hipMemcpyDeviceToDevice, stream_));
        HIPCHK(hipMemcpyAsync(x_.p, x_dev, nbytes, hipMemcpyDeviceToDevice, stream_));
        HIPCHK(hipGraphLaunch(pexec_, stream_));
        HIPCHK(hipMemcpyAsync(x_dev, x_.p, nbytes, hipMemcpyDeviceToDevice, stream_));
        HIPCHK(hipEventRecord(ev1_, stream_));
        HIPCHK(hipMemcpyAsync(hctl_, ctl_.p, (size_t)count * sizeof(Ctl), hipMemcpyDeviceToHost, stream_));
        HIPCHK(hipStreamSynchronize(stream_));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, ev0_, ev1_));
        return finish(infos, batch_ms, ms);
    }

    // Per-problem results from the control words (hctl_, instance order).
    int finish(amgmpcg_info* infos, double* batch_ms, float ms) {
        if (batch_ms) *batch_ms = ms;
        int worst = AMGMPCG_OK;
        for (int i = 0; i < count; ++i) {
            const Ctl& h = hctl_[pos_[i]];
            const int status = h.state == 2 ? h.status : AMGMPCG_MAXIT;
            if (infos) {
                infos[i].status = status;
                infos[i].iterations = h.it;
                infos[i].bnorm = std::sqrt(h.bnorm2);
                infos[i].relres = h.bnorm2 > 0 ? std::sqrt(h.rho / h.bnorm2) : 0.0;
                infos[i].refreshes = h.refreshes;
                infos[i].nb = nlev_[i];
                infos[i].solve_ms = ms;
            }
            if (status != AMGMPCG_OK && worst == AMGMPCG_OK) worst = status;
        }
        return worst;
    }

    struct Range {
        int off = 0, cnt = 0;   // entries of maps_
    };
    struct Group {
        int nlev, first, count;   // problems first .. first+count-1 of the instance array
        Range fine;
    };

    const BBlk* map(const Range& r) const { return maps_.p + r.off; }
    Range dep_[kMaxLevels], pro_[kMaxLevels];   // per depth below the finest level, all groups
    int dmax_ = 0;

    template <int V>
    struct IC {
        static constexpr int value = V;
    };
    template <typename F>
    static void dispatch(int nb, F&& f) {
        switch (nb) {
            case 1: f(IC<1>{}); break;
            case 2: f(IC<2>{}); break;
            case 3: f(IC<3>{}); break;
            case 4: f(IC<4>{}); break;
            case 5: f(IC<5>{}); break;
            case 6: f(IC<6>{}); break;
            default: throw ApiError(AMGMPCG_INVALID_ARG, "batched problems support up to 6 levels");
        }
    }

    // Z = MG(r) of every problem of group G: finest smoother, restriction
    // chain, coarse smoothing, prolongation of the block carry.
    // The multigrid chain of every problem in the same launches, a level
    // named by its depth below the finest one: the finest smoother beside
    // the restriction to depth 1, the smoother of each depth beside the
    // restriction to the next, the deepest alone, then the block carry from
    // the deepest depth up (2 dmax launches, whatever the groups).
    void enqueue_mg_all(hipStream_t s) {
        const T omega = T(opt_.omega);
        const int two = opt_.nu >= 2 ? 1 : 0;
        if (dmax_ == 0) {
            k_b_fine_smooth<DIM, T><<<all_.cnt, kBlock, 0, s>>>(inst_.p, map(all_), omega, two);
            return;
        }
        k_b_dep_restrict_fine_smooth<DIM, T><<<dep_[1].cnt + all_.cnt, kBlock, 0, s>>>(
            inst_.p, map(dep_[1]), dep_[1].cnt, map(all_), omega, two);
        for (int d = 2; d <= dmax_; ++d)
            k_b_dep_restrict_coarse_smooth<DIM, T><<<dep_[d].cnt + dep_[d - 1].cnt, kBlock, 0, s>>>(
                inst_.p, map(dep_[d]), dep_[d].cnt, d, map(dep_[d - 1]), d - 1, omega, two);
        k_b_dep_restrict_coarse_smooth<DIM, T><<<dep_[dmax_].cnt, kBlock, 0, s>>>(
            inst_.p, nullptr, 0, 0, map(dep_[dmax_]), dmax_, omega, two);
        for (int d = dmax_ - 1; d >= 1; --d)
            if (pro_[d].cnt > 0) k_b_dep_prolong<DIM, T><<<pro_[d].cnt, kBlock, 0, s>>>(inst_.p, map(pro_[d]), d);
    }

    void enqueue_init(hipStream_t s, double tol) {
        k_b_init_residual<DIM, T><<<all_.cnt, kBlock, 0, s>>>(inst_.p, map(all_));
        k_b_reduce_init<T><<<count, kRedBlock, 0, s>>>(inst_.p, tol);
        k_b_zero_if<T><<<all_.cnt, kBlock, 0, s>>>(inst_.p, map(all_));
        enqueue_mg_all(s);
        for (const Group& G : groups_) {
            dispatch(G.nlev, [&](auto nbc) {
                constexpr int NB = decltype(nbc)::value;
                k_b_update_xP<DIM, T, NB><<<G.fine.cnt, kBlock, 0, s>>>(inst_.p, map(G.fine), 1);
                k_b_spmm_gram<DIM, T, NB><<<G.fine.cnt, kBlock, 0, s>>>(inst_.p, map(G.fine));
                k_b_reduce_alpha<T, NB><<<G.count, kRedBlock, 0, s>>>(inst_.p, G.first);
            });
        }
    }

    void enqueue_iteration(hipStream_t s) {
        for (const Group& G : groups_) {
            dispatch(G.nlev, [&](auto nbc) {
                constexpr int NB = decltype(nbc)::value;
                k_b_update_r<T, NB><<<G.fine.cnt, kBlock, 0, s>>>(inst_.p, map(G.fine));
            });
        }
        enqueue_mg_all(s);
        for (const Group& G : groups_) {
            dispatch(G.nlev, [&](auto nbc) {
                constexpr int NB = decltype(nbc)::value;
                k_b_fine_W<DIM, T, NB><<<G.fine.cnt, kBlock, 0, s>>>(inst_.p, map(G.fine));
                k_b_reduce_beta<T, NB><<<G.count, kRedBlock, 0, s>>>(inst_.p, G.first, mixed_ ? 1 : 0);
                k_b_update_xP<DIM, T, NB><<<G.fine.cnt, kBlock, 0, s>>>(inst_.p, map(G.fine), 0);
                if (mixed_) {
                    k_b_refresh<DIM, T><<<G.fine.cnt, kBlock, 0, s>>>(inst_.p, map(G.fine));
                    k_b_refresh_reduce<T><<<G.count, kRedBlock, 0, s>>>(inst_.p, G.first);
                }
                k_b_spmm_gram<DIM, T, NB><<<G.fine.cnt, kBlock, 0, s>>>(inst_.p, map(G.fine));
                k_b_reduce_alpha<T, NB><<<G.count, kRedBlock, 0, s>>>(inst_.p, G.first);
            });
        }
    }

    void capture() {
        if (!cap_stream_) HIPCHK(hipStreamCreateWithFlags(&cap_stream_, hipStreamNonBlocking));
        HIPCHK(hipStreamBeginCapture(cap_stream_, hipStreamCaptureModeThreadLocal));
        for (int k = 0; k < kpoll_; ++k) enqueue_iteration(cap_stream_);
        hipError_t launch_err = hipGetLastError();
        HIPCHK(hipStreamEndCapture(cap_stream_, &graph_));
        HIPCHK(launch_err);
        HIPCHK(hipGraphInstantiate(&exec_, graph_, nullptr, nullptr, 0));
    }

    amgmpcg_options opt_;
    hipStream_t stream_;
    hipStream_t cap_stream_ = nullptr;
    hipGraph_t graph_ = nullptr;
    hipGraphExec_t exec_ = nullptr;
    bool mixed_ = false;
    int kpoll_ = 8;
    std::vector<size_t> offs_;        // problem i's fine nodes start at offs_[i] (problem order)
    std::vector<int> nlev_, pos_;     // levels of problem i; its index in the instance array
    std::vector<Group> groups_;
    Range all_;
    std::vector<BInst<T>> hinst_;
    DevBuf<double> x_, r_, b_, small_, part_;
    DevBuf<T> P_, Q_, cL_, coef_, g_, c1_, Y_;
    DevBuf<Ctl> ctl_;
    DevBuf<BInst<T>> inst_;
    DevBuf<BBlk> maps_;
    DevBuf<int> porder_, queue_;      // persistent launch: problem order and queue counter
    int pgrid_ = 1;                   // its workgroups
    hipGraph_t pgraph_ = nullptr;
    hipGraphExec_t pexec_ = nullptr;
    Ctl* hctl_ = nullptr;
    hipEvent_t ev0_ = nullptr, ev1_ = nullptr;
};


BatchedBase* new_batched_solver(int precision, int dim, int count, const amgmpcg_grid* grids,
                                const amgmpcg_options& o, hipStream_t stream) {
    if (precision == 0) {
        if (dim == 2) return new BatchedSolver<double, 2>(count, grids, o, stream);
        return new BatchedSolver<double, 3>(count, grids, o, stream);
    }
    if (dim == 2) return new BatchedSolver<float, 2>(count, grids, o, stream);
    return new BatchedSolver<float, 3>(count, grids, o, stream);
}

}  // namespace amg
