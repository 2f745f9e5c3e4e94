// The general (CSR) hierarchy solver (amgmpcg_setup_csr).
#include "host_common.hpp"
#include "grid_kernels.hpp"
#include "csr_kernels.hpp"

namespace amg {

// ------------------------------------------------------------------ CSR
// Algorithm 1 on a general hierarchy given as sparse matrices (the
// amgmpcg_setup_csr entry point): the same iteration, control word, graph
// capture and reductions as the structured solver, with the CSR kernels of
// csr_kernels.hpp for the operators and transfers.

template <typename T>
class CsrSolver : public SolverBase {
   public:
    CsrSolver(const host::Csr& A, const std::vector<host::Csr>& Ps, double rscale, const amgmpcg_options& o,
              hipStream_t stream)
        : opt_(o), stream_(stream) {
        dim = 0;
        nlev = (int)Ps.size() + 1;
        nb = nlev;
        L_ = nlev - 1;
        mixed_ = std::is_same<T, float>::value;
        // host hierarchy: Galerkin products from the finest level down
        std::vector<host::Csr> lev(nlev);
        lev[L_] = A;
        for (int l = L_ - 1; l >= 0; --l) lev[l] = host::csr_galerkin(lev[l + 1], Ps[l], rscale);
        n_axis.resize(nlev);
        N_.resize(nlev);
        for (int l = 0; l < nlev; ++l) {
            N_[l] = lev[l].n;
            n_axis[l] = lev[l].n;
            const std::vector<double> d = host::csr_diagonal(lev[l]);
            for (double v : d) {
                if (!std::isfinite(v)) throw ApiError(AMGMPCG_NONFINITE, "non-finite level operator");
                if (!(v > 0.0)) throw ApiError(AMGMPCG_NOT_SPD, "non-positive diagonal in a level operator");
            }
        }
        const int N = N_[L_];
        FB_ = fine_blocks(N);
        A_.resize(nlev);
        D_.resize(nlev);
        for (int l = 0; l < nlev; ++l) {
            A_[l].upload(lev[l]);
            D_[l].alloc(N_[l]);
            upload_conv(D_[l].p, host::csr_diagonal(lev[l]));
        }
        A64_.upload(lev[L_]);
        P_l_.resize(nlev);
        R_l_.resize(nlev);
        for (int l = 0; l < L_; ++l) {
            P_l_[l].upload(Ps[l]);
            R_l_[l].upload(host::csr_transpose(Ps[l], rscale));
        }
        g_.resize(nlev);
        c_.resize(nlev);
        c2_.resize(nlev);
        Y_.resize(nlev);
        for (int l = 0; l < L_; ++l) {
            g_[l].alloc(N_[l]);
            if (opt_.nu > 2) {
                c_[l].alloc(N_[l]);
                c2_[l].alloc(N_[l]);
            }
            Y_[l].alloc((size_t)even_up(l + 1) * N_[l]);
            HIPCHK(hipMemset(Y_[l].p, 0, Y_[l].n * sizeof(T)));
        }
        x_.alloc(N);
        r_.alloc(N);
        b_.alloc(N);
        cL_.alloc(N);
        if (opt_.nu > 2) {
            cL2_.alloc(N);
            cL3_.alloc(N);
        }
        m_ = opt_.m;
        kpoll_ = (opt_.k_poll + m_ - 1) / m_ * m_;
        pstride_ = slot_elems(nb, N);
        P_.alloc((size_t)m_ * pstride_ + kBlockSlack);
        Q_.alloc((size_t)m_ * pstride_ + kBlockSlack);
        HIPCHK(hipMemset(P_.p, 0, P_.n * sizeof(T)));
        HIPCHK(hipMemset(Q_.p, 0, Q_.n * sizeof(T)));
        part_.alloc((size_t)FB_ * kPartRow);
        partG_.alloc((size_t)kGramRow * FB_);
        partWin_.alloc((size_t)kMaxWin * kMaxNB * kMaxNB * FB_);
        small_.alloc(kMaxNB + 2 * kMaxWin * kMaxNB * kMaxNB);
        HIPCHK(hipMemset(small_.p, 0, small_.n * sizeof(double)));
        hist_cap_ = opt_.record_history ? std::max(opt_.maxit, 1) : 0;
        if (hist_cap_ > 0) {
            ahist_.alloc((size_t)hist_cap_ * nb);
            rhist_.alloc((size_t)hist_cap_ + 1);
        }
        HIPCHK(hipMalloc((void**)&ctl_, sizeof(Ctl)));
        HIPCHK(hipMalloc((void**)&ctl_free_, sizeof(Ctl)));
        HIPCHK(hipHostMalloc((void**)&hctl_, sizeof(Ctl), hipHostMallocDefault));
        HIPCHK(hipHostMalloc((void**)&hctl_in_, sizeof(Ctl), hipHostMallocDefault));
        Ctl zero{};
        HIPCHK(hipMemcpy(ctl_free_, &zero, sizeof(Ctl), hipMemcpyHostToDevice));
        HIPCHK(hipEventCreate(&ev0_));
        HIPCHK(hipEventCreate(&ev1_));
        tau_ = opt_.pinv_tau > 0 ? opt_.pinv_tau : 64.0 * nb * (mixed_ ? std::ldexp(1.0, -24) : std::ldexp(1.0, -53));
    }

    ~CsrSolver() override {
        if (exec_) (void)hipGraphExecDestroy(exec_);
        if (graph_) (void)hipGraphDestroy(graph_);
        if (cap_stream_) (void)hipStreamDestroy(cap_stream_);
        if (ctl_) (void)hipFree(ctl_);
        if (ctl_free_) (void)hipFree(ctl_free_);
        if (hctl_) (void)hipHostFree(hctl_);
        if (hctl_in_) (void)hipHostFree(hctl_in_);
        if (ev0_) (void)hipEventDestroy(ev0_);
        if (ev1_) (void)hipEventDestroy(ev1_);
    }

    int solve(const double* b_dev, double* x_dev, double tol, int maxit, amgmpcg_info* info) override {
        const int N = N_[L_];
        if (maxit <= 0) maxit = opt_.maxit;
        if (!exec_) capture_graph();
        Ctl& c = *hctl_in_;
        std::memset(&c, 0, sizeof(Ctl));
        c.maxit = maxit;
        c.hist_cap = std::min(hist_cap_, maxit);
        c.drop2 = opt_.refresh_drop * opt_.refresh_drop;
        c.tau = tau_;
        HIPCHK(hipEventRecord(ev0_, stream_));
        HIPCHK(hipMemcpyAsync(ctl_, hctl_in_, sizeof(Ctl), hipMemcpyHostToDevice, stream_));
        HIPCHK(hipMemcpyAsync(b_.p, b_dev, (size_t)N * sizeof(double), hipMemcpyDeviceToDevice, stream_));
        HIPCHK(hipMemcpyAsync(x_.p, x_dev, (size_t)N * sizeof(double), hipMemcpyDeviceToDevice, stream_));
        if (m_ > 1) {
            HIPCHK(hipMemsetAsync(P_.p + pstride_, 0, (size_t)(m_ - 1) * pstride_ * sizeof(T), stream_));
            HIPCHK(hipMemsetAsync(Q_.p + pstride_, 0, (size_t)(m_ - 1) * pstride_ * sizeof(T), stream_));
            HIPCHK(hipMemsetAsync(d_beta(0), 0, (size_t)2 * kMaxWin * kMaxNB * kMaxNB * sizeof(double), stream_));
        }
        enqueue_init(tol);
        HIPCHK(hipGetLastError());
        const int launches_max = maxit / kpoll_ + 3;
        // the first graph follows the set-up without a host check (its
        // kernels are predicated on the device state: a solve that the
        // set-up already ended runs them as no-ops); later ones after one
        HIPCHK(hipGraphLaunch(exec_, stream_));
        for (int launch = 1; launch < launches_max; ++launch) {
            HIPCHK(hipMemcpyAsync(hctl_, ctl_, sizeof(Ctl), hipMemcpyDeviceToHost, stream_));
            HIPCHK(hipStreamSynchronize(stream_));
            if (hctl_->state == 2) break;
            HIPCHK(hipGraphLaunch(exec_, stream_));
        }
        if (opt_.true_residual) {
            // ||b - A x|| / ||b|| of the returned x with the FP64 operator
            k_csr_init_residual<<<FB_, kBlock, 0, stream_>>>(A64_.op(), b_.p, x_.p, r_.p, part_init());
            k_true_relres<<<1, kRedBlock, 0, stream_>>>(ctl_, part_init(), FB_);
        }
        HIPCHK(hipMemcpyAsync(x_dev, x_.p, (size_t)N * sizeof(double), hipMemcpyDeviceToDevice, stream_));
        HIPCHK(hipEventRecord(ev1_, stream_));
        HIPCHK(hipMemcpyAsync(hctl_, ctl_, sizeof(Ctl), hipMemcpyDeviceToHost, stream_));
        HIPCHK(hipStreamSynchronize(stream_));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, ev0_, ev1_));
        const Ctl& h = *hctl_;
        last_iters_ = h.it;
        const int status = h.state == 2 ? h.status : AMGMPCG_MAXIT;
        if (info) {
            info->status = status;
            info->iterations = h.it;
            info->bnorm = std::sqrt(h.bnorm2);
            info->relres = h.bnorm2 > 0 ? std::sqrt(h.rho / h.bnorm2) : 0.0;
            info->refreshes = h.refreshes;
            info->nb = nb;
            info->solve_ms = ms;
            info->relres_true = opt_.true_residual ? h.relres_true : -1.0;
        }
        return status;
    }

    hipStream_t stream() const override { return stream_; }

    void buffers(std::vector<BufRef>& v) override {
        auto csr = [&](DevCsr<T>& M) {
            v.push_back(buf_ref(M.soff));
            v.push_back(buf_ref(M.swid));
            v.push_back(buf_ref(M.col));
            v.push_back(buf_ref(M.val));
        };
        for (std::vector<DevCsr<T>>* vm : {&A_, &P_l_, &R_l_})
            for (DevCsr<T>& M : *vm) csr(M);
        v.push_back(buf_ref(A64_.soff));
        v.push_back(buf_ref(A64_.swid));
        v.push_back(buf_ref(A64_.col));
        v.push_back(buf_ref(A64_.val));
        for (std::vector<DevBuf<T>>* vb : {&D_, &g_, &c_, &c2_, &Y_})
            for (DevBuf<T>& b : *vb) v.push_back(buf_ref(b));
        for (DevBuf<double>* b : {&x_, &r_, &b_, &part_, &partG_, &partWin_, &small_, &ahist_, &rhist_})
            v.push_back(buf_ref(*b));
        for (DevBuf<T>* b : {&P_, &Q_, &cL_, &cL2_, &cL3_}) v.push_back(buf_ref(*b));
    }

    void rebound() override {
        if (exec_) (void)hipGraphExecDestroy(exec_);
        if (graph_) (void)hipGraphDestroy(graph_);
        exec_ = nullptr;
        graph_ = nullptr;
    }

    void mg_block(const double* r_dev, double* Z_dev) override {
        enqueue_mg(ctl_free_, r_dev);
        dispatch([&](auto nbc) {
            constexpr int NB = decltype(nbc)::value;
            k_csr_write_Z<T, NB><<<FB_, kBlock, 0, stream_>>>(N_[L_], fineP(), fine_Y(), cL_final_, Z_dev);
        });
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(stream_));
    }

    void history(int cap, double* alpha, double* res, int* count) override {
        const int k = std::min(std::min(last_iters_, hist_cap_), cap);
        if (count) *count = hist_cap_ ? k : 0;
        if (hist_cap_ == 0) return;
        if (alpha && k > 0)
            HIPCHK(hipMemcpyAsync(alpha, ahist_.p, (size_t)k * nb * sizeof(double), hipMemcpyDeviceToHost, stream_));
        if (res) HIPCHK(hipMemcpyAsync(res, rhist_.p, (size_t)(k + 1) * sizeof(double), hipMemcpyDeviceToHost, stream_));
        HIPCHK(hipStreamSynchronize(stream_));
    }

    void residual(const double* b_dev, const double* x_dev, double* r_dev) override {
        k_csr_init_residual<<<FB_, kBlock, 0, stream_>>>(A64_.op(), b_dev, x_dev, r_dev, part_.p);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(stream_));
    }

    void apply_fine(const double* x_dev, double* y_dev, hipStream_t s) override {
        k_csr_apply<<<FB_, kBlock, 0, s>>>(A64_.op(), x_dev, y_dev);
        HIPCHK(hipGetLastError());
    }

    void level_stencil(int, double*) override { unsupported("level_stencil"); }
    int time_kernels(int, double*, int) override { unsupported("time_kernels"); return 0; }
    int profile_solve(const double*, double*, double, int, amgmpcg_info*, double*, int, int*) override {
        unsupported("profile_solve");
        return 0;
    }
    void attach(cnn::Net* net) override {
        if (net) unsupported("attach_cnn");
    }
    void make_pairs(const double*, const double*, const int*, int, double*, double*) override {
        unsupported("make_pairs");
    }
    void log_kappa(unsigned short*) override { unsupported("log_kappa"); }
    void project_prepare(const double*, double*, hipStream_t) override { unsupported("the learned direction"); }
    void project_direction(const double*, const double*, double*, hipStream_t) override {
        unsupported("the learned direction");
    }

   private:
    template <typename V>
    struct DevCsr {
        int n = 0;
        int maxw = 0;   // widest slice (entries per row, padded)
        DevBuf<int> soff, swid, col;
        DevBuf<V> val;
        // the sliced layout of CsrOp (host::csr_sliced)
        void upload(const host::Csr& M) {
            n = M.n;
            host::Sliced S;
            if (!host::csr_sliced(M, S)) throw ApiError(AMGMPCG_INVALID_ARG, "sparse matrix too large");
            maxw = 0;
            for (int w : S.wid) maxw = std::max(maxw, w);
            std::vector<V> v(S.val.begin(), S.val.end());
            soff.alloc(S.off.size());
            swid.alloc(S.wid.size());
            col.alloc(S.col.size());
            val.alloc(v.size());
            if (!S.off.empty()) {
                HIPCHK(hipMemcpy(soff.p, S.off.data(), S.off.size() * sizeof(int), hipMemcpyHostToDevice));
                HIPCHK(hipMemcpy(swid.p, S.wid.data(), S.wid.size() * sizeof(int), hipMemcpyHostToDevice));
            }
            HIPCHK(hipMemcpy(col.p, S.col.data(), S.col.size() * sizeof(int), hipMemcpyHostToDevice));
            HIPCHK(hipMemcpy(val.p, v.data(), v.size() * sizeof(V), hipMemcpyHostToDevice));
        }
        CsrOp<V> op() const { return CsrOp<V>{n, soff.p, swid.p, col.p, val.p}; }
    };

    static void upload_conv(T* dst, const std::vector<double>& src) {
        std::vector<T> tmp(src.begin(), src.end());
        HIPCHK(hipMemcpy(dst, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice));
    }

    [[noreturn]] static void unsupported(const char* what) {
        throw ApiError(AMGMPCG_INVALID_ARG, std::string(what) + " is not available for a CSR handle");
    }

    template <int V>
    struct IC {
        static constexpr int value = V;
    };
    template <typename F>
    void dispatch(F&& f) {
        switch (nb) {
            case 1: f(IC<1>{}); break;
            case 2: f(IC<2>{}); break;
            case 3: f(IC<3>{}); break;
            case 4: f(IC<4>{}); break;
            case 5: f(IC<5>{}); break;
            case 6: f(IC<6>{}); break;
            case 7: f(IC<7>{}); break;
            case 8: f(IC<8>{}); break;
            default: throw ApiError(AMGMPCG_INVALID_ARG, "unsupported number of levels");
        }
    }
    template <typename F>
    static void dispatch_nc(int nc, F&& f) {
        switch (nc) {
            case 1: f(IC<1>{}); break;
            case 2: f(IC<2>{}); break;
            case 3: f(IC<3>{}); break;
            case 4: f(IC<4>{}); break;
            case 5: f(IC<5>{}); break;
            case 6: f(IC<6>{}); break;
            default: f(IC<7>{}); break;
        }
    }

    CsrOp<T> fineP() const {
        return L_ > 0 ? P_l_[L_ - 1].op() : CsrOp<T>{N_[L_], nullptr, nullptr, nullptr, nullptr};
    }
    const T* fine_Y() const { return L_ > 0 ? Y_[L_ - 1].p : nullptr; }
    T* Pslot(int j) { return P_.p + (size_t)j * pstride_; }
    T* Qslot(int j) { return Q_.p + (size_t)j * pstride_; }
    double* part_init() { return part_.p; }
    double* part_rho() { return part_.p + (size_t)FB_ * 2; }
    double* part_ref() { return part_.p + (size_t)FB_ * (kPartRow - 1); }
    double* part_G() { return partG_.p; }
    double* part_Wslot(int j) { return partWin_.p + (size_t)j * kMaxNB * kMaxNB * FB_; }
    double* d_alpha() { return small_.p; }
    double* d_beta(int j = 0) { return small_.p + kMaxNB + (size_t)j * kMaxNB * kMaxNB; }
    double* d_Gplus(int j = 0) { return small_.p + kMaxNB + (size_t)(kMaxWin + j) * kMaxNB * kMaxNB; }
    PWin<T> window() {
        PWin<T> w{};
        for (int j = 0; j < m_; ++j) w.p[j] = Pslot(j);
        return w;
    }
    static int blocks(int n) {
        const int b = (n + kBlock - 1) / kBlock;
        return std::max(1, std::min(b, kMaxFineBlocks));
    }

    // nu damped-Jacobi sweeps from zero on level l (g in type G), result to
    // out[i * stride]; for nu > 2 the intermediate sweeps ping-pong through
    // a and b (both distinct from out).
    template <typename G>
    void smooth(const Ctl* ctl, int l, const G* g, T* out, int stride, T* a, T* b) {
        const T omega = T(opt_.omega);
        const int nu = opt_.nu;
        const CsrOp<T> A = A_[l].op();
        const int nbk = blocks(N_[l]);
        if (nu <= 2) {
            k_csr_smooth<T, G><<<nbk, kBlock, 0, stream_>>>(ctl, A, D_[l].p, g, out, stride, omega, nu >= 2 ? 1 : 0);
            return;
        }
        k_csr_smooth<T, G><<<nbk, kBlock, 0, stream_>>>(ctl, A, D_[l].p, g, a, 1, omega, 1);
        T* cur = a;
        for (int s = 0; s < nu - 2; ++s) {
            const bool last = s == nu - 3;
            T* nxt = last ? out : (cur == a ? b : a);
            k_csr_sweep<T, G><<<nbk, kBlock, 0, stream_>>>(ctl, A, D_[l].p, g, cur, 1, nxt, last ? stride : 1, omega);
            cur = nxt;
        }
    }

    // Z = MG(r): the finest smoother output cL, the restriction chain, the
    // smoother on every coarse level (into the last column of its block
    // carry) and the prolongation of the block carry up to level L-1.
    void enqueue_mg(const Ctl* ctl, const double* r) {
        if (opt_.nu <= 2 && L_ > 0) {
            enqueue_mg_fused(ctl, r);
            return;
        }
        smooth<double>(ctl, L_, r, cL_.p, 1, cL2_.p, cL3_.p);
        cL_final_ = cL_.p;
        if (L_ == 0) return;
        k_csr_restrict<T, double><<<blocks(N_[L_ - 1]), kBlock, 0, stream_>>>(ctl, R_l_[L_ - 1].op(), r, g_[L_ - 1].p);
        for (int l = L_ - 2; l >= 0; --l)
            k_csr_restrict<T, T><<<blocks(N_[l]), kBlock, 0, stream_>>>(ctl, R_l_[l].op(), g_[l + 1].p, g_[l].p);
        for (int l = 0; l < L_; ++l) smooth<T>(ctl, l, g_[l].p, Y_[l].p + l, even_up(l + 1), c_[l].p, c2_[l].p);
        enqueue_prolong(ctl);
    }

    // nu <= 2: each smoother runs beside a restriction (the finest beside
    // the first, both reading r; each restricted level beside the
    // restriction from it), level 0's alone: L + 1 launches for the chain's
    // restriction and smoothing instead of 2L + 1, with the same arithmetic.
    void enqueue_mg_fused(const Ctl* ctl, const double* r) {
        const T omega = T(opt_.omega);
        const int two = opt_.nu >= 2 ? 1 : 0;
        {
            const int l = L_ - 1;
            launch_rs<double, double>(ctl, &R_l_[l], r, g_[l].p, A_[L_], D_[L_].p, r, cL_.p, 1, omega, two);
            cL_final_ = cL_.p;
        }
        for (int l = L_ - 2; l >= 0; --l)
            launch_rs<T, T>(ctl, &R_l_[l], g_[l + 1].p, g_[l].p, A_[l + 1], D_[l + 1].p, g_[l + 1].p,
                            Y_[l + 1].p + (l + 1), even_up(l + 2), omega, two);
        launch_rs<T, T>(ctl, nullptr, static_cast<const T*>(nullptr), nullptr, A_[0], D_[0].p, g_[0].p, Y_[0].p,
                        even_up(1), omega, two);
        enqueue_prolong(ctl);
    }

    // One restriction + smoother launch; the rows of a half with at most
    // kCsrWaveRows rows of at least kCsrWaveWidth entries (padded slice
    // width) are taken one per wavefront (small coarse levels: their
    // ~27-entry rows would otherwise be walked by few threads in dependent
    // groups), the others one per thread.
    static constexpr int kCsrWaveRows = 1 << 12;
    static constexpr int kCsrWaveWidth = 16;
    static bool wave_rows(const DevCsr<T>& M) { return M.n <= kCsrWaveRows && M.maxw >= kCsrWaveWidth; }
    template <typename TI, typename G>
    void launch_rs(const Ctl* ctl, const DevCsr<T>* Rm, const TI* gf, T* gc, const DevCsr<T>& Am, const T* D,
                   const G* g, T* out, int stride, T omega, int two) {
        const CsrOp<T> R = Rm ? Rm->op() : CsrOp<T>{0, nullptr, nullptr, nullptr, nullptr};
        const CsrOp<T> A = Am.op();
        const bool wr = Rm && R.n > 0 && wave_rows(*Rm), ws = wave_rows(Am);
        const int nr = R.n > 0 ? (wr ? (R.n + kWaves - 1) / kWaves : blocks(R.n)) : 0;
        const int ns = ws ? (A.n + kWaves - 1) / kWaves : blocks(A.n);
        auto go = [&](auto k) { k<<<nr + ns, kBlock, 0, stream_>>>(ctl, R, gf, gc, nr, A, D, g, out, stride, omega, two); };
        if (wr && ws) go(k_csr_restrict_smooth_w<T, TI, G, 1, 1>);
        else if (wr) go(k_csr_restrict_smooth_w<T, TI, G, 1, 0>);
        else if (ws) go(k_csr_restrict_smooth_w<T, TI, G, 0, 1>);
        else go(k_csr_restrict_smooth<T, TI, G>);
    }

    void enqueue_prolong(const Ctl* ctl) {
        for (int l = 0; l + 1 < L_; ++l) {
            dispatch_nc(l + 1, [&](auto ncc) {
                constexpr int NC = decltype(ncc)::value;
                k_csr_prolong<T, NC><<<blocks(N_[l + 1]), kBlock, 0, stream_>>>(ctl, P_l_[l].op(), Y_[l].p,
                                                                                Y_[l + 1].p);
            });
        }
    }


    void enqueue_init(double tol) {
        const int N = N_[L_];
        k_csr_init_residual<<<FB_, kBlock, 0, stream_>>>(A64_.op(), b_.p, x_.p, r_.p, part_init());
        k_reduce_init<<<1, kRedBlock, 0, stream_>>>(ctl_, part_init(), FB_, tol, hist_cap_ ? rhist_.p : nullptr);
        k_zero_if<<<FB_, kBlock, 0, stream_>>>(ctl_, x_.p, N);
        enqueue_mg(ctl_, r_.p);
        dispatch([&](auto nbc) {
            constexpr int NB = decltype(nbc)::value;
            k_csr_update_xP<T, NB><<<FB_, kBlock, 0, stream_>>>(ctl_, N, fineP(), fine_Y(), cL_final_, window(),
                                                                m_, 0, 0, x_.p, d_alpha(), d_beta(), 1);
            k_csr_spmm_gram<T, NB><<<FB_, kBlock, 0, stream_>>>(ctl_, A_[L_].op(), Pslot(0), Qslot(0), r_.p,
                                                                part_G());
            k_reduce_alpha<NB><<<1, kRedBlock, 0, stream_>>>(ctl_, part_G(), FB_, d_Gplus(0), d_alpha(),
                                                          hist_cap_ ? ahist_.p : nullptr);
        });
    }

    void enqueue_iteration(hipStream_t s, int j) {
        const int N = N_[L_];
        const int cur = j % m_, nxt = (j + 1) % m_;
        hipStream_t saved = stream_;
        stream_ = s;
        dispatch([&](auto nbc) {
            constexpr int NB = decltype(nbc)::value;
            k_update_r<T, NB><<<FB_, kBlock, 0, s>>>(ctl_, N, Qslot(cur), d_alpha(), r_.p, part_rho());
            enqueue_mg(ctl_, r_.p);
            for (int q = 0; q < m_; ++q)
                k_csr_fine_W<T, NB><<<FB_, kBlock, 0, s>>>(ctl_, N, fineP(), fine_Y(), cL_final_, Qslot(q),
                                                           part_Wslot(q));
            k_reduce_beta<NB><<<1, kRedBlock, 0, s>>>(ctl_, part_rho(), FB_, part_Wslot(0), FB_, m_, cur, d_Gplus(0),
                                                   d_beta(0), hist_cap_ ? rhist_.p : nullptr, mixed_ ? 1 : 0);
            k_csr_update_xP<T, NB><<<FB_, kBlock, 0, s>>>(ctl_, N, fineP(), fine_Y(), cL_final_, window(), m_, cur,
                                                          nxt, x_.p, d_alpha(), d_beta(0), 0);
            if (mixed_) {
                k_csr_refresh<<<FB_, kBlock, 0, s>>>(ctl_, A64_.op(), b_.p, x_.p, r_.p, part_ref());
                k_refresh_reduce<<<1, kRedBlock, 0, s>>>(ctl_, part_ref(), FB_, hist_cap_ ? rhist_.p : nullptr);
            }
            k_csr_spmm_gram<T, NB><<<FB_, kBlock, 0, s>>>(ctl_, A_[L_].op(), Pslot(nxt), Qslot(nxt), r_.p,
                                                          part_G());
            k_reduce_alpha<NB><<<1, kRedBlock, 0, s>>>(ctl_, part_G(), FB_, d_Gplus(nxt), d_alpha(),
                                                    hist_cap_ ? ahist_.p : nullptr);
        });
        stream_ = saved;
    }

    void capture_graph() {
        if (!cap_stream_) HIPCHK(hipStreamCreateWithFlags(&cap_stream_, hipStreamNonBlocking));
        HIPCHK(hipStreamBeginCapture(cap_stream_, hipStreamCaptureModeThreadLocal));
        for (int k = 0; k < kpoll_; ++k) enqueue_iteration(cap_stream_, k);
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
    int L_ = 0, FB_ = 1, hist_cap_ = 0, last_iters_ = 0, m_ = 1, kpoll_ = 8;
    size_t pstride_ = 0;
    double tau_ = 0.0;
    std::vector<int> N_;
    std::vector<DevCsr<T>> A_, P_l_, R_l_;
    DevCsr<double> A64_;
    std::vector<DevBuf<T>> D_, g_, c_, c2_, Y_;
    DevBuf<double> x_, r_, b_, part_, partG_, partWin_, small_, ahist_, rhist_;
    DevBuf<T> P_, Q_, cL_, cL2_, cL3_;
    T* cL_final_ = nullptr;
    Ctl *ctl_ = nullptr, *ctl_free_ = nullptr, *hctl_ = nullptr, *hctl_in_ = nullptr;
    hipEvent_t ev0_ = nullptr, ev1_ = nullptr;
};


SolverBase* new_csr_solver(int precision, const host::Csr& A, const std::vector<host::Csr>& Ps, double rscale,
                           const amgmpcg_options& o, hipStream_t stream) {
    if (precision == 0) return new CsrSolver<double>(A, Ps, rscale, o, stream);
    return new CsrSolver<float>(A, Ps, rscale, o, stream);
}

}  // namespace amg
