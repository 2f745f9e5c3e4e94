// Batched solves of many structured problems (amgmpcg_setup_batched).
#include "host_common.hpp"
#include "grid_kernels.hpp"
#include "batched.hpp"

namespace amg {

// ------------------------------------------------------------------ batched


template <typename T, int DIM>
class BatchedSolver : public BatchedBase {
   public:
    BatchedSolver(int cnt, const amgmpcg_grid* grids, const amgmpcg_options& o, hipStream_t stream)
        : opt_(o), stream_(stream) {
        count = cnt;
        mixed_ = std::is_same<T, float>::value;
        offs_.assign(cnt + 1, 0);
        nlev_.resize(cnt);
        std::vector<std::vector<int>> sizes(cnt);
        size_t nP = 0, ncoef = 0, nvec = 0, nY = 0;
        for (int i = 0; i < cnt; ++i) {
            const int nl = grids[i].nlevels;
            nlev_[i] = nl;
            sizes[i].resize(nl);
            sizes[i][nl - 1] = grids[i].n;
            for (int l = nl - 2; l >= 0; --l) sizes[i][l] = sizes[i][l + 1] / 2;
            const size_t N = (size_t)host::ipow(grids[i].n, DIM);
            offs_[i + 1] = offs_[i] + N;
            nP += (size_t)even_up(nl) * N;
            for (int l = 0; l + 1 < nl; ++l) {
                const size_t Nl = (size_t)host::ipow(sizes[i][l], DIM);
                ncoef += (size_t)(DIM == 2 ? 9 : 27) * Nl;
                nvec += Nl;
                nY += (size_t)even_up(l + 1) * Nl;
            }
        }
        total = (int64_t)offs_[cnt];
        x_.alloc(offs_[cnt]);
        r_.alloc(offs_[cnt]);
        b_.alloc(offs_[cnt]);
        P_.alloc(nP);
        Q_.alloc(nP);
        cL_.alloc(offs_[cnt]);
        coef_.alloc(std::max<size_t>(ncoef, 1));
        g_.alloc(std::max<size_t>(nvec, 1));
        c1_.alloc(std::max<size_t>(nvec, 1));
        Y_.alloc(std::max<size_t>(nY, 1));
        HIPCHK(hipMemset(P_.p, 0, P_.n * sizeof(T)));
        HIPCHK(hipMemset(Q_.p, 0, Q_.n * sizeof(T)));
        HIPCHK(hipMemset(Y_.p, 0, Y_.n * sizeof(T)));

        // instance array ordered by number of levels: the groups
        std::vector<int> order(cnt);
        for (int i = 0; i < cnt; ++i) order[i] = i;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return nlev_[a] < nlev_[b]; });
        pos_.resize(cnt);
        for (int q = 0; q < cnt; ++q) pos_[order[q]] = q;
        for (int q = 0; q < cnt; ++q) {
            const int nl = nlev_[order[q]];
            if (groups_.empty() || groups_.back().nlev != nl) groups_.push_back(Group{nl, q, 0});
            ++groups_.back().count;
        }

        ctl_.alloc(cnt);
        small_.alloc((size_t)cnt * kBSmall);
        HIPCHK(hipMemset(small_.p, 0, small_.n * sizeof(double)));
        size_t npart = 0;
        std::vector<int> pcnt(cnt);
        for (int i = 0; i < cnt; ++i) {
            const size_t N = offs_[i + 1] - offs_[i];
            pcnt[i] = (int)((N + kBChunk - 1) / kBChunk);
            npart += (size_t)pcnt[i] * kBPartRows;
        }
        part_.alloc(npart);

        // per-problem hierarchy (host Galerkin) and device pointers
        hinst_.resize(cnt);
        size_t oP = 0, oc = 0, ov = 0, oY = 0, opart = 0;
        std::vector<T> coef_host(ncoef);
        for (int i = 0; i < cnt; ++i) {
            const int nl = nlev_[i], n = grids[i].n;
            BInst<T>& I = hinst_[pos_[i]];
            std::memset(&I, 0, sizeof(I));
            I.nlev = nl;
            for (int l = 0; l < nl; ++l) {
                I.n[l] = sizes[i][l];
                I.N[l] = (int)host::ipow(sizes[i][l], DIM);
            }
            const size_t N = offs_[i + 1] - offs_[i];
            const double h2inv = double(n + 1) * double(n + 1);
            I.op.n = n;
            I.op.N = (int)N;
            I.op.s0 = T(h2inv);
            I.op.inv0 = T(1.0 / (2.0 * DIM * h2inv));
            I.op64.n = n;
            I.op64.N = (int)N;
            I.op64.s0 = h2inv;
            I.op64.inv0 = 1.0 / (2.0 * DIM * h2inv);
            I.x = x_.p + offs_[i];
            I.r = r_.p + offs_[i];
            I.b = b_.p + offs_[i];
            I.cL = cL_.p + offs_[i];
            I.P = P_.p + oP;
            I.Q = Q_.p + oP;
            oP += (size_t)even_up(nl) * N;
            I.ctl = ctl_.p + pos_[i];
            I.small = small_.p + (size_t)pos_[i] * kBSmall;
            I.part = part_.p + opart;
            I.pcnt = pcnt[i];
            opart += (size_t)pcnt[i] * kBPartRows;
            if (nl > 1) {
                host::FineFaces faces = host::fine_faces(DIM, n, nullptr);
                std::vector<host::StencilLevel> lev(nl);
                lev[nl - 1] = host::faces_to_stencil(DIM, n, faces);
                for (int l = nl - 2; l >= 0; --l) {
                    lev[l] = host::galerkin(lev[l + 1]);
                    const int ctr = lev[l].center();
                    for (int64_t q = 0; q < lev[l].N; ++q)
                        if (!(lev[l].coef[(size_t)ctr * lev[l].N + q] > 0.0))
                            throw ApiError(AMGMPCG_NOT_SPD, "non-positive diagonal on a coarse level");
                }
                for (int l = 0; l + 1 < nl; ++l) {
                    const size_t Nl = (size_t)I.N[l];
                    const size_t cnt_c = (size_t)(DIM == 2 ? 9 : 27) * Nl;
                    for (size_t q = 0; q < cnt_c; ++q) coef_host[oc + q] = T(lev[l].coef[q]);
                    I.coef[l] = coef_.p + oc;
                    oc += cnt_c;
                    I.g[l] = g_.p + ov;
                    I.c1[l] = c1_.p + ov;
                    ov += Nl;
                    I.Y[l] = Y_.p + oY;
                    oY += (size_t)even_up(l + 1) * Nl;
                }
            }
        }
        if (ncoef) HIPCHK(hipMemcpy(coef_.p, coef_host.data(), ncoef * sizeof(T), hipMemcpyHostToDevice));
        inst_.alloc(cnt);
        HIPCHK(hipMemcpy(inst_.p, hinst_.data(), cnt * sizeof(BInst<T>), hipMemcpyHostToDevice));

        // block maps: all problems' fine nodes, per group its fine nodes
        std::vector<BBlk> maps;
        auto fine_blocks = [&](int q0, int q1) {
            for (int q = q0; q < q1; ++q) {
                const BInst<T>& I = hinst_[q];
                const int N = I.N[I.nlev - 1];
                for (int j = 0; j < I.pcnt; ++j)
                    maps.push_back(BBlk{q, j, j * kBChunk, std::min(N, (j + 1) * kBChunk)});
            }
        };
        all_.off = (int)maps.size();
        fine_blocks(0, cnt);
        all_.cnt = (int)maps.size() - all_.off;
        for (Group& G : groups_) {
            G.fine.off = (int)maps.size();
            fine_blocks(G.first, G.first + G.count);
            G.fine.cnt = (int)maps.size() - G.fine.off;
        }
        // per depth below the finest level, over all groups: that coarse
        // level's nodes (restriction and smoothing), and the same for the
        // problems where it is not the coarsest level (carry into it)
        dmax_ = 0;
        for (const Group& G : groups_) dmax_ = std::max(dmax_, G.nlev - 1);
        for (int d = 1; d <= dmax_; ++d) {
            for (int pass = 0; pass < 2; ++pass) {
                Range& R = pass == 0 ? dep_[d] : pro_[d];
                R.off = (int)maps.size();
                for (const Group& G : groups_) {
                    const int l = G.nlev - 1 - d;
                    if (l < 0 || (pass == 1 && l == 0)) continue;
                    for (int q = G.first; q < G.first + G.count; ++q) {
                        const int Nl = hinst_[q].N[l];
                        for (int j = 0, s0 = 0; s0 < Nl; ++j, s0 += kBlock)
                            maps.push_back(BBlk{q, j, s0, std::min(Nl, s0 + kBlock)});
                    }
                }
                R.cnt = (int)maps.size() - R.off;
            }
        }
        maps_.alloc(maps.size());
        HIPCHK(hipMemcpy(maps_.p, maps.data(), maps.size() * sizeof(BBlk), hipMemcpyHostToDevice));
        HIPCHK(hipHostMalloc((void**)&hctl_, (size_t)cnt * sizeof(Ctl), hipHostMallocDefault));
        HIPCHK(hipEventCreate(&ev0_));
        HIPCHK(hipEventCreate(&ev1_));
        kpoll_ = opt_.k_poll;
    }

    ~BatchedSolver() override {
        if (exec_) (void)hipGraphExecDestroy(exec_);
        if (graph_) (void)hipGraphDestroy(graph_);
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
        }
        const size_t nbytes = (size_t)offs_[count] * sizeof(double);
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

   private:
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
        HIPCHK(hipStreamCreateWithFlags(&cap_stream_, hipStreamNonBlocking));
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
