// The structured-grid solver (amgmpcg_setup_grid / amgmpcg_setup_stencil):
// hierarchy setup, device workspace, the per-iteration launch sequence
// captured once into a HIP graph (k_poll iterations per graph), the
// device-side stop flag polled by the host between graph launches.
#pragma once
#include "host_common.hpp"
#include "grid_kernels.hpp"
#include "pcg_kernels.hpp"
#include "cnn_host.hpp"

namespace amg {

template <typename T, int DIM>
class Solver : public SolverBase {
   public:
    // st9: NULL, or (2D, kappa NULL) the constant 9-point finest stencil
    Solver(const amgmpcg_grid& g, const amgmpcg_options& o, hipStream_t stream, const double* st9 = nullptr)
        : opt_(o), stream_(stream) {
        dim = DIM;
        nlev = g.nlevels;
        method_ = o.method;
        nb = method_ == AMGMPCG_METHOD_MPCG ? nlev : 1;
        vnu_ = o.nu_pre > 0 ? o.nu_pre : std::max(1, o.nu / 2);
        L_ = nlev - 1;
        mixed_ = std::is_same<T, float>::value;
        n_axis.resize(nlev);
        n_axis[L_] = g.n;
        for (int l = L_ - 1; l >= 0; --l) n_axis[l] = n_axis[l + 1] / 2;
        N_.resize(nlev);
        for (int l = 0; l < nlev; ++l) N_[l] = (int)host::ipow(n_axis[l], DIM);
        const int N = N_[L_];
        rows_.n = g.n;
        rows_.nxp = (g.n + 63) / 64 * 64;
        rows_.total = (int)host::ipow(g.n, DIM - 1) * rows_.nxp;
        FB_ = fine_blocks(rows_.total);
        FBG_ = fine_blocks(rows_.total, kGramBlocks);
        XPB_ = fine_blocks(rows_.total, xp_blocks_per_cu<1>() * kNumCU);
        if (DIM == 3) {
            // z chunks so that the units fill the resident blocks (2 or 3 per
            // CU) about once
            zntx_ = (g.n + kZTileX - 1) / kZTileX;
            const int tiles = zntx_ * ((g.n + kZTY - 1) / kZTY);
            for (int v = 0; v < 2; ++v) {
                const int chunks = std::max(1, (v + 2) * kNumCU / tiles);
                zkz_[v] = kZKZ > 0 ? std::min(kZKZ, g.n) : (g.n + chunks - 1) / chunks;
                znkz_[v] = (g.n + zkz_[v] - 1) / zkz_[v];
                SB_[v] = tiles * znkz_[v];
            }
        }

        // ---- host hierarchy (FP64) -------------------------------------
        const bool var = g.kappa != nullptr;
        host::FineFaces faces = host::fine_faces(DIM, g.n, g.kappa);
        for (int64_t i = 0; i < (int64_t)N; ++i) {
            if (!std::isfinite(faces.D[i])) throw ApiError(AMGMPCG_NONFINITE, "non-finite kappa");
            if (!(faces.D[i] > 0.0)) throw ApiError(AMGMPCG_NOT_SPD, "non-positive diagonal on the finest level");
        }
        std::vector<host::StencilLevel> lev(nlev);
        if (L_ > 0) {
            lev[L_] = st9 ? host::constant_stencil9(g.n, st9) : host::faces_to_stencil(DIM, g.n, faces);
            for (int l = L_ - 1; l >= 0; --l) {
                lev[l] = host::galerkin(lev[l + 1]);
                const int ctr = lev[l].center();
                for (int64_t i = 0; i < lev[l].N; ++i) {
                    const double d = lev[l].coef[(size_t)ctr * lev[l].N + i];
                    if (!std::isfinite(d)) throw ApiError(AMGMPCG_NONFINITE, "non-finite coarse operator");
                    if (!(d > 0.0)) throw ApiError(AMGMPCG_NOT_SPD, "non-positive diagonal on a coarse level");
                }
            }
        }

        // ---- device memory ---------------------------------------------
        const double h2inv = double(g.n + 1) * double(g.n + 1);
        fop_.n = g.n;
        fop_.N = N;
        fop_.s0 = T(h2inv);
        fop_.D = fop_.ex = fop_.ey = fop_.ez = nullptr;
        fop_.inv0 = T(1.0 / (2.0 * DIM * h2inv));
        fop_.iD = nullptr;
        f64_.n = g.n;
        f64_.N = N;
        f64_.s0 = h2inv;
        f64_.D = f64_.ex = f64_.ey = f64_.ez = nullptr;
        f64_.inv0 = 1.0 / (2.0 * DIM * h2inv);
        f64_.iD = nullptr;
        if (DIM == 2 && st9) {
            fop_.k9 = f64_.k9 = 1;
            for (int q = 0; q < 9; ++q) {
                fop_.w9[q] = T(st9[q]);
                f64_.w9[q] = st9[q];
            }
            fop_.inv0 = T(1.0 / st9[4]);
            f64_.inv0 = 1.0 / st9[4];
        }
        if (var) {
            upload_faces(faces);
        }
        coef_.resize(nlev);
        g_.resize(nlev);
        c1_.resize(nlev);
        c_.resize(nlev);
        c2_.resize(nlev);
        Y_.resize(nlev);
        cst_.assign(nlev, 0);
        for (int l = 0; l < L_; ++l) {
            const int S = lev[l].S();
            // a level whose stencil is the same at every node (truncated at
            // the boundary; constant coefficient, odd grid sizes) keeps only
            // those S values
            cst_[l] = host::constant_with_truncation(lev[l]) ? 1 : 0;
            if (cst_[l]) {
                const int c = n_axis[l] / 2;
                const int64_t ref = c + (int64_t)n_axis[l] * (c + (DIM == 3 ? (int64_t)n_axis[l] * c : 0));
                std::vector<double> w(S);
                for (int q = 0; q < S; ++q) w[q] = lev[l].coef[(size_t)q * N_[l] + ref];
                coef_[l].alloc((size_t)S);
                upload_conv(coef_[l].p, w);
            } else {
                coef_[l].alloc((size_t)S * N_[l]);
                upload_conv(coef_[l].p, lev[l].coef);
            }
            g_[l].alloc(N_[l]);
            c1_[l].alloc(N_[l]);
            if (opt_.nu > 2) {
                c_[l].alloc(N_[l]);
                c2_[l].alloc(N_[l]);
            }
            // node-major block carry [P Y_{l-1} | c_l], l+1 columns, even stride
            Y_[l].alloc((size_t)even_up(l + 1) * N_[l]);
            HIPCHK(hipMemset(Y_[l].p, 0, Y_[l].n * sizeof(T)));
        }
        x_.alloc(N);
        r_.alloc(N);
        b_.alloc(N);
        m_ = opt_.m;
        kpoll_ = (opt_.k_poll + m_ - 1) / m_ * m_;
        pstride_ = slot_elems(nb, N);
        P_.alloc((size_t)m_ * pstride_ + kBlockSlack);
        Q_.alloc((size_t)m_ * pstride_ + kBlockSlack);
        HIPCHK(hipMemset(P_.p, 0, P_.n * sizeof(T)));
        HIPCHK(hipMemset(Q_.p, 0, Q_.n * sizeof(T)));
        cL_.alloc(N);
        if (opt_.nu > 2) cL2_.alloc(N);
        if (method_ != AMGMPCG_METHOD_MPCG) zv_.alloc(N);
        if (method_ == AMGMPCG_METHOD_VCYCLE_PCG) {
            vcL_.alloc(N);
            vtL_.alloc(N);
            vrL_.alloc(N);
            vg_.resize(nlev);
            vc_.resize(nlev);
            vt_.resize(nlev);
            vr_.resize(nlev);
            for (int l = 0; l < L_; ++l) {
                vg_[l].alloc(N_[l]);
                vc_[l].alloc(N_[l]);
                vt_[l].alloc(N_[l]);
                vr_[l].alloc(N_[l]);
            }
        }
        part_.alloc((size_t)FB_ * kPartRow);
        partG_.alloc((size_t)kGramRow * std::max(std::max(SB_[0], SB_[1]), FBG_));
        small_.alloc(kMaxNB + 2 * kMaxWin * kMaxNB * kMaxNB);
        partWin_.alloc((size_t)kMaxWin * kMaxNB * kMaxNB * FBG_);
        hist_cap_ = opt_.record_history ? std::max(opt_.maxit, 1) : 0;
        if (hist_cap_ > 0) {
            ahist_.alloc((size_t)hist_cap_ * nb);
            rhist_.alloc((size_t)hist_cap_ + 1);
        }
        HIPCHK(hipMalloc((void**)&ctl_, sizeof(Ctl)));
        HIPCHK(hipMalloc((void**)&ctl_free_, sizeof(Ctl)));
        HIPCHK(hipMalloc((void**)&ctl_proj_, sizeof(Ctl)));
        HIPCHK(hipHostMalloc((void**)&hctl_proj_, sizeof(Ctl), hipHostMallocDefault));
        HIPCHK(hipHostMalloc((void**)&hctl_, sizeof(Ctl), hipHostMallocDefault));
        HIPCHK(hipHostMalloc((void**)&hctl_in_, sizeof(Ctl), hipHostMallocDefault));
        std::memset(hctl_in_, 0, sizeof(Ctl));
        HIPCHK(hipMemcpyAsync(ctl_free_, hctl_in_, sizeof(Ctl), hipMemcpyHostToDevice, stream_));
        HIPCHK(hipMemsetAsync(small_.p, 0, small_.n * sizeof(double), stream_));
        HIPCHK(hipEventCreate(&ev0_));
        HIPCHK(hipEventCreate(&ev1_));
        HIPCHK(hipStreamCreateWithFlags(&side_, hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&ev_fork_, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&ev_join_, hipEventDisableTiming));
        HIPCHK(hipStreamSynchronize(stream_));
        set_tau();
        if (DIM == 3 && var) {
            // network input channel: log kappa at the n^3 nodes, normalised
            // to zero mean and unit standard deviation, rounded to bfloat16
            const int n = g.n, m = n + 2;
            std::vector<double> lk((size_t)N);
            double mean = 0.0;
            for (int z = 0; z < n; ++z)
                for (int y = 0; y < n; ++y)
                    for (int x = 0; x < n; ++x) {
                        const double v = std::log(g.kappa[((size_t)(z + 1) * m + (y + 1)) * m + (x + 1)]);
                        lk[((size_t)z * n + y) * n + x] = v;
                        mean += v;
                    }
            mean /= N;
            double var2 = 0.0;
            for (double v : lk) var2 += (v - mean) * (v - mean);
            const double sd = std::sqrt(var2 / N);
            std::vector<unsigned short> h((size_t)N);
            for (size_t i = 0; i < h.size(); ++i) {
                const float f = (float)((lk[i] - mean) / (sd > 0.0 ? sd : 1.0));
                uint32_t u;
                std::memcpy(&u, &f, 4);
                u += 0x7fffu + ((u >> 16) & 1u);
                h[i] = (unsigned short)(u >> 16);
            }
            lk_.alloc(N);
            HIPCHK(hipMemcpy(lk_.p, h.data(), h.size() * sizeof(unsigned short), hipMemcpyHostToDevice));
        }
    }

    // m > 1: the slots a solve has not written yet must hold zero blocks and a
    // zero G^+ (so that their beta and P_j beta vanish, also after a solve
    // that left non-finite values); slot 0 is written by the start.
    void clear_window() {
        if (m_ == 1) return;
        HIPCHK(hipMemsetAsync(Pslot(1), 0, (size_t)(m_ - 1) * pstride_ * sizeof(T), stream_));
        HIPCHK(hipMemsetAsync(Qslot(1), 0, (size_t)(m_ - 1) * pstride_ * sizeof(T), stream_));
        HIPCHK(hipMemsetAsync(d_beta(0), 0, (size_t)2 * kMaxWin * kMaxNB * kMaxNB * sizeof(double), stream_));
    }

    void set_tau() {
        tau_ = opt_.pinv_tau > 0 ? opt_.pinv_tau : 64.0 * nb * (mixed_ ? std::ldexp(1.0, -24) : std::ldexp(1.0, -53));
    }

    // Append (net != null) or remove the learned direction.  The column count
    // becomes L + 2; P, Q and the history grow, the captured graph is redone.
    void attach(cnn::Net* net) override {
        const int N = N_[L_];
        if (net) {
            if (method_ != AMGMPCG_METHOD_MPCG)
                throw ApiError(AMGMPCG_INVALID_ARG, "the learned direction needs the MPCG method");
            if (DIM != 3) throw ApiError(AMGMPCG_INVALID_ARG, "the learned direction needs a 3D problem");
            if (net->n != n_axis[L_]) throw ApiError(AMGMPCG_DIM_MISMATCH, "network grid differs from the problem grid");
            if (nlev + 1 > kMaxNB) throw ApiError(AMGMPCG_INVALID_ARG, "too many levels for an extra direction");
        }
        // the wider blocks would be allocated anew: do it before the buffers move
        if (bound()) throw ApiError(AMGMPCG_INVALID_ARG, "attach or detach the network before binding the workspace");
        net_ = net;
        nb = nlev + (net ? 1 : 0);
        pstride_ = slot_elems(nb, N);
        const size_t need = (size_t)m_ * pstride_ + kBlockSlack;
        if (P_.n < need) {
            P_.alloc(need);
            Q_.alloc(need);
            HIPCHK(hipMemset(P_.p, 0, P_.n * sizeof(T)));
            HIPCHK(hipMemset(Q_.p, 0, Q_.n * sizeof(T)));
        }
        if (net && !dl_.p) dl_.alloc(N);
        if (hist_cap_ > 0) ahist_.alloc((size_t)hist_cap_ * nb);
        set_tau();
        drop_graph();
    }

    void residual(const double* b_dev, const double* x_dev, double* r_dev) override {
        k_init_residual<DIM><<<FB_, kBlock, 0, stream_>>>(rows_, f64_, b_dev, x_dev, r_dev, part_init());
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(stream_));
    }

    // Training pairs from this handle's own iterates: for each k in ks, x_k =
    // k iterations from x0 = 0 (x_0 = 0), r_k = b - A x_k, e_k = xs - x_k.
    void make_pairs(const double* b_dev, const double* xs_dev, const int* ks, int nk, double* R_dev,
                    double* E_dev) override {
        const int N = N_[L_];
        if (!xt_.p) xt_.alloc(N);
        for (int i = 0; i < nk; ++i) {
            HIPCHK(hipMemsetAsync(xt_.p, 0, (size_t)N * sizeof(double), stream_));
            if (ks[i] > 0) solve(b_dev, xt_.p, 0.0, ks[i], nullptr);
            k_pair<DIM><<<(rows_.total + kBlock - 1) / kBlock, kBlock, 0, stream_>>>(
                rows_, f64_, b_dev, xs_dev, xt_.p, R_dev + (size_t)i * N, E_dev + (size_t)i * N);
            HIPCHK(hipGetLastError());
        }
        HIPCHK(hipStreamSynchronize(stream_));
    }

    void log_kappa(unsigned short* lk_dev) override {
        const int N = N_[L_];
        if (lk_.p)
            HIPCHK(hipMemcpyAsync(lk_dev, lk_.p, (size_t)N * sizeof(unsigned short), hipMemcpyDeviceToDevice, stream_));
        else
            HIPCHK(hipMemsetAsync(lk_dev, 0, (size_t)N * sizeof(unsigned short), stream_));
        HIPCHK(hipStreamSynchronize(stream_));
    }

    // y = A x (finest operator, FP64) on stream s, not synchronised.
    void apply_fine(const double* x_dev, double* y_dev, hipStream_t s) override {
        k_apply<DIM><<<(rows_.total + kBlock - 1) / kBlock, kBlock, 0, s>>>(rows_, f64_, x_dev, y_dev);
    }

    // A-orthogonal projection onto the level-correction block of r (the
    // first MPCG step from residual r): P = Z = MG(r), Q = A P, G^+, alpha =
    // G^+ P^T r and rhat = r - Q alpha.  Uses the handle's work vectors; P, Q
    // and G^+ stay for project_direction.  Needs FP64 and no attached network.
    void project_prepare(const double* r_dev, double* rhat_dev, hipStream_t s) override {
        if (mixed_ || net_) throw ApiError(AMGMPCG_INVALID_ARG, "projection needs an FP64 handle without a network");
        const int N = N_[L_];
        hipStream_t saved = stream_;
        stream_ = s;
        Ctl& c = *hctl_proj_;
        std::memset(&c, 0, sizeof(Ctl));
        c.maxit = 1;
        c.tau = tau_;
        HIPCHK(hipMemcpyAsync(ctl_proj_, hctl_proj_, sizeof(Ctl), hipMemcpyHostToDevice, s));
        enqueue_fine(ctl_proj_, r_dev);
        enqueue_coarse(ctl_proj_, r_dev);
        dispatch_plain([&](auto nbc) {
            constexpr int NB = decltype(nbc)::value;
            const int nc = L_ > 0 ? n_axis[L_ - 1] : 1;
            k_update_xP<DIM, T, NB, 0><<<xp_grid<NB>(), kBlock, 0, s>>>(ctl_proj_, rows_, fine_Y(), nc, cL_final_, nullptr,
                                                               nullptr, single(), 1, 0, 0, x_.p, d_alpha(), d_beta(),
                                                               1);
            launch_spmm<NB>(ctl_proj_, P_.p, Q_.p, r_dev, s);
            k_reduce_alpha<NB><<<1, kRedBlock, 0, s>>>(ctl_proj_, part_G(), spmm_blocks<NB>(), d_Gplus(), d_alpha(), nullptr);
            HIPCHK(hipMemcpyAsync(rhat_dev, r_dev, (size_t)N * sizeof(double), hipMemcpyDeviceToDevice, s));
            k_update_r<T, NB><<<FB_, kBlock, 0, s>>>(ctl_proj_, N, Q_.p, d_alpha(), rhat_dev, part_rho());
        });
        stream_ = saved;
    }

    // qhat = q - Q G^+ Q^T d for the block of the last project_prepare.
    void project_direction(const double* d_dev, const double* q_dev, double* qhat_dev, hipStream_t s) override {
        const int N = N_[L_];
        dispatch_plain([&](auto nbc) {
            constexpr int NB = decltype(nbc)::value;
            k_cols_dot<T, NB><<<FB_, kBlock, 0, s>>>(Q_.p, d_dev, N, part_W());
            k_proj_coef<NB><<<1, kRedBlock, 0, s>>>(part_W(), FB_, d_Gplus(), d_beta());
            k_sub_cols<T, NB><<<FB_, kBlock, 0, s>>>(q_dev, Q_.p, d_beta(), qhat_dev, N);
        });
    }

    const T* dl() const { return net_ ? dl_.p : nullptr; }
    const int* dflag() const { return net_ ? net_->flag.p : nullptr; }

    // The learned direction d = N(r) into dl_ (bulk type); flag on non-finite.
    void enqueue_learned(const Ctl* ctl, const double* r) {
        const int n = n_axis[L_];
        cnn::net_forward(*net_, ctl, r, lk_.p, stream_);
        cnn::k_clear_flag<<<1, 64, 0, stream_>>>(ctl, net_->flag.p);
        cnn::k_unpack_output<T><<<(N_[L_] + cnn::kCB - 1) / cnn::kCB, cnn::kCB, 0, stream_>>>(
            ctl, net_->out.p, dl_.p, n, net_->S, net_->flag.p);
    }

    ~Solver() override {
        if (exec_) (void)hipGraphExecDestroy(exec_);
        if (graph_) (void)hipGraphDestroy(graph_);
        if (cap_stream_) (void)hipStreamDestroy(cap_stream_);
        if (ctl_) (void)hipFree(ctl_);
        if (ctl_free_) (void)hipFree(ctl_free_);
        if (ctl_proj_) (void)hipFree(ctl_proj_);
        if (hctl_proj_) (void)hipHostFree(hctl_proj_);
        if (hctl_) (void)hipHostFree(hctl_);
        if (hctl_in_) (void)hipHostFree(hctl_in_);
        if (ev0_) (void)hipEventDestroy(ev0_);
        if (ev1_) (void)hipEventDestroy(ev1_);
        for (hipEvent_t e : prof_ev_) (void)hipEventDestroy(e);
        for (hipEvent_t e : xp_ev_)
            if (e) (void)hipEventDestroy(e);
        if (ev_fork_) (void)hipEventDestroy(ev_fork_);
        if (ev_join_) (void)hipEventDestroy(ev_join_);
        if (side_) (void)hipStreamDestroy(side_);
    }

    int solve(const double* b_dev, double* x_dev, double tol, int maxit, amgmpcg_info* info) override {
        const int N = N_[L_];
        if (maxit <= 0) maxit = opt_.maxit;
        if (!graph_ready_) capture_graph();
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
        clear_window();
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
            k_init_residual<DIM><<<FB_, kBlock, 0, stream_>>>(rows_, f64_, b_.p, x_.p, r_.p, part_init());
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
        int status = h.state == 2 ? h.status : AMGMPCG_MAXIT;
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
        for (DevBuf<T>* b : {&fD_, &fex_, &fey_, &fez_, &fiD_, &P_, &Q_, &cL_, &cL2_, &dl_, &zv_, &vcL_, &vtL_, &vrL_})
            v.push_back(buf_ref(*b));
        for (DevBuf<double>* b : {&gD_, &gex_, &gey_, &gez_, &giD_, &x_, &r_, &b_, &part_, &small_, &ahist_, &rhist_,
                                  &partWin_, &partG_, &xt_})
            v.push_back(buf_ref(*b));
        for (std::vector<DevBuf<T>>* vb : {&coef_, &g_, &c1_, &c_, &c2_, &Y_, &vg_, &vc_, &vt_, &vr_})
            for (DevBuf<T>& b : *vb) v.push_back(buf_ref(b));
        v.push_back(buf_ref(lk_));
    }

    void rebound() override {
        fop_.D = fD_.p;
        fop_.ex = fex_.p;
        fop_.ey = fey_.p;
        fop_.ez = DIM == 3 ? fez_.p : nullptr;
        fop_.iD = fiD_.p;
        if (std::is_same<T, double>::value) {
            f64_.D = (const double*)fD_.p;
            f64_.ex = (const double*)fex_.p;
            f64_.ey = (const double*)fey_.p;
            f64_.ez = DIM == 3 ? (const double*)fez_.p : nullptr;
            f64_.iD = (const double*)fiD_.p;
        } else {
            f64_.D = gD_.p;
            f64_.ex = gex_.p;
            f64_.ey = gey_.p;
            f64_.ez = DIM == 3 ? gez_.p : nullptr;
            f64_.iD = giD_.p;
        }
        drop_graph();
    }

    void drop_graph() {
        if (exec_) (void)hipGraphExecDestroy(exec_);
        if (graph_) (void)hipGraphDestroy(graph_);
        exec_ = nullptr;
        graph_ = nullptr;
        graph_ready_ = false;
    }

    void mg_block(const double* r_dev, double* Z_dev) override {
        if (method_ != AMGMPCG_METHOD_MPCG)
            throw ApiError(AMGMPCG_INVALID_ARG, "mg_block is defined for the MPCG method");
        enqueue_mg(ctl_free_, r_dev);
        const int N = N_[L_];
        dispatch_nb([&](auto nbc) {
            constexpr int NB = decltype(nbc)::value, NE = decltype(nbc)::ne;
            k_write_Z<DIM, T, NB, NE><<<(rows_.total + kBlock - 1) / kBlock, kBlock, 0, stream_>>>(
                rows_, N, fine_Y(), L_ > 0 ? n_axis[L_ - 1] : 1, cL_final_, dl(), dflag(), Z_dev);
        });
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(stream_));
    }

    void level_stencil(int level, double* out) override {
        if (level < 0 || level >= L_) throw ApiError(AMGMPCG_INVALID_ARG, "level must be a coarse level");
        const int S = DIM == 2 ? 9 : 27;
        const size_t cnt = (size_t)S * N_[level];
        if (!cst_[level]) {
            std::vector<T> tmp(cnt);
            HIPCHK(hipMemcpyAsync(tmp.data(), coef_[level].p, cnt * sizeof(T), hipMemcpyDeviceToHost, stream_));
            HIPCHK(hipStreamSynchronize(stream_));
            for (size_t i = 0; i < cnt; ++i) out[i] = double(tmp[i]);
            return;
        }
        // constant stencil: expanded with the couplings outside the grid dropped
        std::vector<T> w(S);
        HIPCHK(hipMemcpyAsync(w.data(), coef_[level].p, S * sizeof(T), hipMemcpyDeviceToHost, stream_));
        HIPCHK(hipStreamSynchronize(stream_));
        const int n = n_axis[level];
        for (int64_t idx = 0; idx < N_[level]; ++idx) {
            const int i = (int)(idx % n), j = (int)((idx / n) % n), k = DIM == 3 ? (int)(idx / ((int64_t)n * n)) : 0;
            int q = 0;
            for (int dz = (DIM == 3 ? -1 : 0); dz <= (DIM == 3 ? 1 : 0); ++dz)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx, ++q) {
                        const bool in = i + dx >= 0 && i + dx < n && j + dy >= 0 && j + dy < n &&
                                        (DIM == 2 || (k + dz >= 0 && k + dz < n));
                        out[(size_t)q * N_[level] + idx] = in ? double(w[q]) : 0.0;
                    }
        }
    }

    void history(int cap, double* alpha, double* res, int* count) override {
        const int k = std::min(std::min(last_iters_, hist_cap_), cap);
        if (count) *count = k;
        if (hist_cap_ == 0) {
            if (count) *count = 0;
            return;
        }
        if (alpha && k > 0)
            HIPCHK(hipMemcpyAsync(alpha, ahist_.p, (size_t)k * nb * sizeof(double), hipMemcpyDeviceToHost, stream_));
        if (res) HIPCHK(hipMemcpyAsync(res, rhist_.p, (size_t)(k + 1) * sizeof(double), hipMemcpyDeviceToHost, stream_));
        HIPCHK(hipStreamSynchronize(stream_));
    }

    // Average duration (ms) of each hot kernel, launched reps times back to
    // back between two HIP events on the handle's stream, on the state left
    // by the last solve.  Order: update_r, fine_smooth, restrict_fine,
    // coarse_smooth, prolong_top, fine_W, update_xP, spmm_gram, residual.
    int time_kernels(int reps, double* ms, int cap) override {
        const int N = N_[L_];
        const Ctl* cf = ctl_free_;
        const T omega = T(opt_.omega);
        int count = 0;
        auto timed = [&](auto&& launch) {
            HIPCHK(hipEventRecord(ev0_, stream_));
            for (int i = 0; i < reps; ++i) launch();
            HIPCHK(hipEventRecord(ev1_, stream_));
            HIPCHK(hipEventSynchronize(ev1_));
            HIPCHK(hipGetLastError());
            float t = 0.f;
            HIPCHK(hipEventElapsedTime(&t, ev0_, ev1_));
            if (count < cap) ms[count] = double(t) / reps;
            ++count;
        };
        enqueue_mg(cf, r_.p);   // sets the final smoother buffers
        dispatch_nb([&](auto nbc) {
            constexpr int NB = decltype(nbc)::value;
            [[maybe_unused]] constexpr int NE = decltype(nbc)::ne;
            const int nc = L_ > 0 ? n_axis[L_ - 1] : 1;
            timed([&] { k_update_r<T, NB><<<FB_, kBlock, 0, stream_>>>(cf, N, Q_.p, d_alpha(), r_.p, part_rho()); });
            timed([&] {
                k_fine_smooth<DIM, T, double><<<FB_, kBlock, 0, stream_>>>(cf, rows_, fop_, r_.p, cL_.p, omega,
                                                                            opt_.nu >= 2 ? 1 : 0);
            });
            if (L_ > 0) {
                const int l = L_ - 1;
                timed([&] {
                    k_restrict<DIM, double, T><<<(N_[l] + kBlock - 1) / kBlock, kBlock, 0, stream_>>>(
                        cf, r_.p, n_axis[L_], g_[l].p, n_axis[l], N_[l], diag(l), c1_[l].p, omega, cst_[l]);
                });
                CoarseLevels<T> cl = coarse_arg(0);
                const int off = cl.blk_off[L_];
                timed([&] { k_coarse_smooth<DIM, T><<<off, kBlock, 0, stream_>>>(cf, cl, omega, 0, opt_.nu >= 2 ? 1 : 0); });
                if (L_ >= 2) {
                    timed([&] { launch_prolong(cf, L_ - 2); });
                } else {
                    timed([&] {});
                }
            } else {
                timed([&] {});
                timed([&] {});
                timed([&] {});
            }
            enqueue_mg(cf, r_.p);
            timed([&] {
                k_fine_W<DIM, T, NB, NE><<<fw_grid<NB, NE>(), kBlock, 0, stream_>>>(
                    cf, rows_, fine_Y(), nc, cL_final_, dl(), dflag(), Q_.p, 0, part_W(), 0, fw_grid<NB, NE>());
            });
            timed([&] {
                k_update_xP<DIM, T, NB, NE><<<xp_grid<NB>(), kBlock, 0, stream_>>>(cf, rows_, fine_Y(), nc, cL_final_, dl(),
                                                                         dflag(), single(), 1, 0, 0, x_.p,
                                                                         d_alpha(), d_beta(), 0);
            });
            timed([&] { launch_spmm<NB>(cf, P_.p, Q_.p, r_.p, stream_); });
            timed([&] { k_init_residual<DIM><<<FB_, kBlock, 0, stream_>>>(rows_, f64_, b_.p, x_.p, r_.p, part_init()); });
        });
        return count;
    }

   private:
    template <int V, int E = 0>
    struct IC {
        static constexpr int value = V;
        static constexpr int ne = E;   // 1: the last column is the learned direction
    };

    // The plain level block (nlev columns), whatever is attached.
    template <typename F>
    void dispatch_plain(F&& f) {
        switch (nlev) {
            case 1: f(IC<1>{}); break;
            case 2: f(IC<2>{}); break;
            case 3: f(IC<3>{}); break;
            case 4: f(IC<4>{}); break;
            case 5: f(IC<5>{}); break;
            case 6: f(IC<6>{}); break;
            case 7: f(IC<7>{}); break;
            case 8: f(IC<8>{}); break;
            default: throw ApiError(AMGMPCG_INVALID_ARG, "unsupported number of directions");
        }
    }

    template <typename F>
    void dispatch_nb(F&& f) {
        if constexpr (DIM == 3) {
            if (net_) {
                switch (nb) {
                    case 2: f(IC<2, 1>{}); break;
                    case 3: f(IC<3, 1>{}); break;
                    case 4: f(IC<4, 1>{}); break;
                    case 5: f(IC<5, 1>{}); break;
                    case 6: f(IC<6, 1>{}); break;
                    case 7: f(IC<7, 1>{}); break;
                    case 8: f(IC<8, 1>{}); break;
                    default: throw ApiError(AMGMPCG_INVALID_ARG, "unsupported number of directions");
                }
                return;
            }
        }
        switch (nb) {
            case 1: f(IC<1>{}); break;
            case 2: f(IC<2>{}); break;
            case 3: f(IC<3>{}); break;
            case 4: f(IC<4>{}); break;
            case 5: f(IC<5>{}); break;
            case 6: f(IC<6>{}); break;
            case 7: f(IC<7>{}); break;
            case 8: f(IC<8>{}); break;
            default: throw ApiError(AMGMPCG_INVALID_ARG, "unsupported number of directions");
        }
    }

    void upload_faces(const host::FineFaces& f) {
        const int N = N_[L_];
        auto up = [&](DevBuf<T>& d, const std::vector<double>& v) {
            d.alloc(v.size());
            upload_conv(d.p, v);
        };
        up(fD_, f.D);
        {
            std::vector<double> inv(f.D.size());
            for (size_t i = 0; i < inv.size(); ++i) inv[i] = 1.0 / f.D[i];
            up(fiD_, inv);
            fop_.iD = fiD_.p;
            if (std::is_same<T, double>::value) {
                f64_.iD = (const double*)fiD_.p;
            } else {
                giD_.alloc(inv.size());
                HIPCHK(hipMemcpy(giD_.p, inv.data(), inv.size() * sizeof(double), hipMemcpyHostToDevice));
                f64_.iD = giD_.p;
            }
        }
        up(fex_, f.ex);
        up(fey_, f.ey);
        if (DIM == 3) up(fez_, f.ez);
        fop_.D = fD_.p;
        fop_.ex = fex_.p;
        fop_.ey = fey_.p;
        fop_.ez = DIM == 3 ? fez_.p : nullptr;
        if (std::is_same<T, double>::value) {
            f64_.D = (const double*)fD_.p;
            f64_.ex = (const double*)fex_.p;
            f64_.ey = (const double*)fey_.p;
            f64_.ez = DIM == 3 ? (const double*)fez_.p : nullptr;
        } else {
            auto up64 = [&](DevBuf<double>& d, const std::vector<double>& v) {
                d.alloc(v.size());
                HIPCHK(hipMemcpy(d.p, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice));
            };
            up64(gD_, f.D);
            up64(gex_, f.ex);
            up64(gey_, f.ey);
            if (DIM == 3) up64(gez_, f.ez);
            f64_.D = gD_.p;
            f64_.ex = gex_.p;
            f64_.ey = gey_.p;
            f64_.ez = DIM == 3 ? gez_.p : nullptr;
        }
        (void)N;
    }

    void upload_conv(T* dst, const std::vector<double>& src) {
        std::vector<T> tmp(src.begin(), src.end());
        HIPCHK(hipMemcpy(dst, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice));
    }

    // Diagonal (stencil centre) of coarse level l.
    const T* diag(int l) const {
        return coef_[l].p + (size_t)(DIM == 2 ? 4 : 13) * (cst_[l] ? 1 : N_[l]);
    }

    // The node-major level-(L-1) block from which the fine corrections are formed.
    const T* fine_Y() const { return L_ > 0 ? Y_[L_ - 1].p : nullptr; }

    // Arguments of the level-fused coarse smoother.  final_out: write into the
    // last column of each level's block carry (else into the c_ buffer).
    CoarseLevels<T> coarse_arg(int final_out) const {
        CoarseLevels<T> cl{};
        cl.nlev = L_;
        int off = 0;
        for (int l = 0; l < L_; ++l) {
            cl.blk_off[l] = off;
            off += (N_[l] + kBlock - 1) / kBlock;
            cl.n[l] = n_axis[l];
            cl.N[l] = N_[l];
            cl.coef[l] = coef_[l].p;
            cl.cst[l] = cst_[l];
            cl.g[l] = g_[l].p;
            cl.c1[l] = c1_[l].p;
            if (final_out || !c_[l].p) {
                cl.cout[l] = Y_[l].p + l;
                cl.cstride[l] = even_up(l + 1);
            } else {
                cl.cout[l] = c_[l].p;
                cl.cstride[l] = 1;
            }
            cl.cin[l] = nullptr;
        }
        cl.blk_off[L_] = off;
        return cl;
    }

    // Y_{l+2}[:, 0..l+1] from Y_l and c_{l+1} in one launch (k_prolong2).
    void launch_prolong2(const Ctl* ctl, int l) {
        const int grid = (N_[l + 2] + kBlock - 1) / kBlock;
        const T* Yc = Y_[l].p;
        const T* Ym = Y_[l + 1].p;
        T* Yf = Y_[l + 2].p;
        const int nc = n_axis[l], nm = n_axis[l + 1], nf = n_axis[l + 2], Nf = N_[l + 2];
        switch (l + 1) {
            case 1: k_prolong2<DIM, T, 1><<<grid, kBlock, 0, stream_>>>(ctl, Yc, nc, Ym, nm, Yf, nf, Nf); break;
            case 2: k_prolong2<DIM, T, 2><<<grid, kBlock, 0, stream_>>>(ctl, Yc, nc, Ym, nm, Yf, nf, Nf); break;
            case 3: k_prolong2<DIM, T, 3><<<grid, kBlock, 0, stream_>>>(ctl, Yc, nc, Ym, nm, Yf, nf, Nf); break;
            case 4: k_prolong2<DIM, T, 4><<<grid, kBlock, 0, stream_>>>(ctl, Yc, nc, Ym, nm, Yf, nf, Nf); break;
            case 5: k_prolong2<DIM, T, 5><<<grid, kBlock, 0, stream_>>>(ctl, Yc, nc, Ym, nm, Yf, nf, Nf); break;
            default: k_prolong2<DIM, T, 6><<<grid, kBlock, 0, stream_>>>(ctl, Yc, nc, Ym, nm, Yf, nf, Nf); break;
        }
    }

    // Y_{l+1}[:, 0..l] = P Y_l (l+1 columns).
    void launch_prolong(const Ctl* ctl, int l) {
        const int grid = (N_[l + 1] + kBlock - 1) / kBlock;
        const T* Yc = Y_[l].p;
        T* Yf = Y_[l + 1].p;
        const int nc = n_axis[l], nf = n_axis[l + 1], Nf = N_[l + 1];
        switch (l + 1) {
            case 1: k_prolong<DIM, T, 1><<<grid, kBlock, 0, stream_>>>(ctl, Yc, nc, Yf, nf, Nf); break;
            case 2: k_prolong<DIM, T, 2><<<grid, kBlock, 0, stream_>>>(ctl, Yc, nc, Yf, nf, Nf); break;
            case 3: k_prolong<DIM, T, 3><<<grid, kBlock, 0, stream_>>>(ctl, Yc, nc, Yf, nf, Nf); break;
            case 4: k_prolong<DIM, T, 4><<<grid, kBlock, 0, stream_>>>(ctl, Yc, nc, Yf, nf, Nf); break;
            case 5: k_prolong<DIM, T, 5><<<grid, kBlock, 0, stream_>>>(ctl, Yc, nc, Yf, nf, Nf); break;
            case 6: k_prolong<DIM, T, 6><<<grid, kBlock, 0, stream_>>>(ctl, Yc, nc, Yf, nf, Nf); break;
            default: k_prolong<DIM, T, 7><<<grid, kBlock, 0, stream_>>>(ctl, Yc, nc, Yf, nf, Nf); break;
        }
    }

    // Z = MG(r): every level correction and, when attached, the learned one.
    // With a network attached, the network and the fine smoother (they
    // depend only on r, like the coarse chain of restriction, coarse
    // smoothing and prolongation) run on a second stream, forked from and
    // joined back into the current one (inside graph capture this gives
    // parallel branches), so the coarse chain hides under the inference.
    // Without a network the fork costs more than it overlaps (measured), and
    // while profiling every kernel is timed alone: serial.
    void enqueue_mg(const Ctl* ctl, const double* r) {
        if (fused_mg()) {
            enqueue_mg_fused(ctl, r);
            return;
        }
        if (L_ > 0 && !net_) {
            enqueue_mg_paired(ctl, r);
            return;
        }
        if (prof_on_ || !side_ || !net_) {
            enqueue_fine(ctl, r);
            enqueue_coarse(ctl, r);
            if (net_) {
                mark(kSecLearned);
                enqueue_learned(ctl, r);
            }
            return;
        }
        HIPCHK(hipEventRecord(ev_fork_, stream_));
        HIPCHK(hipStreamWaitEvent(side_, ev_fork_, 0));
        hipStream_t main = stream_;
        stream_ = side_;
        enqueue_fine(ctl, r);
        if (net_) enqueue_learned(ctl, r);
        stream_ = main;
        HIPCHK(hipEventRecord(ev_join_, side_));
        enqueue_coarse(ctl, r);
        HIPCHK(hipStreamWaitEvent(stream_, ev_join_, 0));
    }

    // With nu <= 2 and no network the chain runs in fused launches: the
    // finest smoother beside the first restriction, the smoother of each
    // restricted level beside the next restriction, the smallest levels'
    // restrictions, smoothers and prolongations in the tail launch (the
    // kernels' arithmetic is that of the separate launches, so the results
    // are the same).
    bool fused_mg() const { return L_ > 0 && opt_.nu <= 2 && !net_; }

    SmoothLevel<T> smooth_level(int l) const {
        SmoothLevel<T> sm;
        sm.op = CoarseOp<T>{n_axis[l], N_[l], coef_[l].p, cst_[l]};
        sm.g = g_[l].p;
        sm.c1 = c1_[l].p;
        sm.out = Y_[l].p + l;
        sm.stride = even_up(l + 1);
        return sm;
    }

    void enqueue_mg_fused(const Ctl* ctl, const double* r) {
        const int L = L_;
        const T omega = T(opt_.omega);
        const int two = opt_.nu >= 2 ? 1 : 0;
        mark(kSecRestrict);
        {
            const int l = L - 1;
            const RestrictStep<double, T> rs{r, n_axis[L], g_[l].p, n_axis[l], N_[l], diag(l), c1_[l].p, cst_[l]};
            bool tiled = false;
            if constexpr (DIM == 3) {
                // constant coefficients, two sweeps, level L-1 of size (n - 1) / 2
                if (two && !fop_.D && !fop_.iD && n_axis[l] == (n_axis[L] - 1) / 2) {
                    const int n = n_axis[L];
                    const int ntx = (n + kRTX - 1) / kRTX, nty = (n + kRTY - 1) / kRTY, ntz = (n + kRTZ - 1) / kRTZ;
                    k_restrict_fine_smooth_tile<T><<<ntx * nty * ntz, kBlock, 0, stream_>>>(ctl, rs, fop_, r, cL_.p,
                                                                                           omega, ntx, nty, ntz);
                    tiled = true;
                }
            }
            if (!tiled) {
                const int nbr = ((N_[l] + kBlock - 1) / kBlock + kNumXcd - 1) / kNumXcd * kNumXcd;
                k_restrict_fine_smooth<DIM, T><<<nbr + FB_, kBlock, 0, stream_>>>(ctl, rs, nbr, rows_, fop_, r,
                                                                                cL_.p, omega, two);
            }
            cL_final_ = cL_.p;
        }
        int m = L - 2;
        for (; m >= 0 && N_[m] > kRestrictTailMax; --m) {
            const RestrictStep<T, T> rs{g_[m + 1].p, n_axis[m + 1], g_[m].p, n_axis[m], N_[m], diag(m), c1_[m].p,
                                        cst_[m]};
            bool tiled = false;
            if constexpr (DIM == 3) {
                // constant stencil on level m+1, two sweeps, level m of size
                // (n - 1) / 2, and boxes enough to fill the chip (63^3: 1024;
                // at 31^3 the 128 boxes ran slower than the per-node form)
                const int n = n_axis[m + 1];
                const int ntx = (n + kCBX - 1) / kCBX, nty = (n + kCBY - 1) / kCBY, ntz = (n + kCBZ - 1) / kCBZ;
                if (two && cst_[m + 1] && n_axis[m] == (n - 1) / 2 && ntx * nty * ntz >= 512) {
                    k_restrict_coarse_smooth_tile<T><<<ntx * nty * ntz, kBlock, 0, stream_>>>(
                        ctl, rs, smooth_level(m + 1), omega, ntx, nty, ntz);
                    tiled = true;
                }
            }
            if (!tiled) {
                const int nbr = (N_[m] + kBlock - 1) / kBlock;
                const int nbs = (N_[m + 1] + kBlock - 1) / kBlock;
                k_restrict_coarse_smooth<DIM, T><<<nbr + nbs, kBlock, 0, stream_>>>(ctl, rs, nbr, smooth_level(m + 1),
                                                                                  omega, two);
            }
        }
        // level m+1 is restricted but not yet smoothed; levels m..0 are small
        if (m >= 0) {
            RestrictChain<T> ch{};
            SmoothChain<T> sc{};
            for (int q = m; q >= 0; --q) {
                const int c = ch.count++;
                ch.nf[c] = n_axis[q + 1];
                ch.nc[c] = n_axis[q];
                ch.Nc[c] = N_[q];
                ch.gf[c] = g_[q + 1].p;
                ch.gc[c] = g_[q].p;
                ch.D[c] = diag(q);
                ch.dconst[c] = cst_[q];
                ch.c1[c] = c1_[q].p;
                sc.lev[sc.count++] = smooth_level(q);
            }
            // block 0 also carries the block up through the small levels
            ProlongChain<T> up{};
            up.l0 = 0;
            for (int l = 0; l < m; ++l) {
                const int q = up.count++;
                up.nc[q] = n_axis[l];
                up.nf[q] = n_axis[l + 1];
                up.Nf[q] = N_[l + 1];
                up.Yc[q] = Y_[l].p;
                up.Yf[q] = Y_[l + 1].p;
            }
            const int nbt = (N_[m + 1] + kTailBlock - 1) / kTailBlock;
            k_tail_smooth<DIM, T><<<1 + nbt, kTailBlock, 0, stream_>>>(ctl, ch, sc, smooth_level(m + 1), up, omega,
                                                                      two);
            mark(kSecProlong);
            for (int l = m; l + 1 < L;) {
                // two small carry steps in one launch where the level two up is small
                if (l + 2 < L && N_[l + 2] <= kProlong2Max) {
                    launch_prolong2(ctl, l);
                    l += 2;
                } else {
                    launch_prolong(ctl, l);
                    l += 1;
                }
            }
        } else {
            const int nbs = (N_[0] + kBlock - 1) / kBlock;
            k_restrict_coarse_smooth<DIM, T><<<nbs, kBlock, 0, stream_>>>(ctl, RestrictStep<T, T>{}, 0,
                                                                        smooth_level(0), omega, two);
            mark(kSecProlong);
            enqueue_prolong(ctl);
        }
    }

    // nu > 2 and no network: the restriction chain, then each sweep index
    // of every level (finest and all coarse) in one launch, then the
    // prolongation chain; the buffers alternate as in the separate launches.
    void enqueue_mg_paired(const Ctl* ctl, const double* r) {
        const int L = L_;
        const T omega = T(opt_.omega);
        const int extra = opt_.nu - 2;
        mark(kSecRestrict);
        enqueue_restrict_chain(ctl, r);
        mark(kSecCoarseSmooth);
        CoarseLevels<T> cl = coarse_arg(0);     // first sweeps into c_
        const int nbc = (cl.blk_off[L] + kNumXcd - 1) / kNumXcd * kNumXcd;
        T* first = (extra % 2 == 0) ? cL_.p : cL2_.p;
        T* other = (extra % 2 == 0) ? cL2_.p : cL_.p;
        k_sweep_levels<DIM, T><<<nbc + FB_, kBlock, 0, stream_>>>(ctl, cl, nbc, omega, 0, 1, rows_, fop_, r, nullptr,
                                                                  first);
        T* cur = first;
        for (int s2 = 0; s2 < extra; ++s2) {
            const bool last = s2 == extra - 1;
            const bool from_c = (s2 % 2) == 0;
            for (int l = 0; l < L; ++l) {
                cl.cin[l] = from_c ? c_[l].p : c2_[l].p;
                if (last) {
                    cl.cout[l] = Y_[l].p + l;
                    cl.cstride[l] = even_up(l + 1);
                } else {
                    cl.cout[l] = from_c ? c2_[l].p : c_[l].p;
                    cl.cstride[l] = 1;
                }
            }
            T* nxt = (cur == first) ? other : first;
            k_sweep_levels<DIM, T><<<nbc + FB_, kBlock, 0, stream_>>>(ctl, cl, nbc, omega, 1, 1, rows_, fop_, r, cur,
                                                                      nxt);
            cur = nxt;
        }
        cL_final_ = cur;
        mark(kSecProlong);
        enqueue_prolong(ctl);
    }

    // the finest level's smoother output cL_final_ (nu sweeps from zero)
    void enqueue_fine(const Ctl* ctl, const double* r) {
        const T omega = T(opt_.omega);
        const int nu = opt_.nu;
        const int two = nu >= 2 ? 1 : 0;
        const int extra = nu > 2 ? nu - 2 : 0;
        mark(kSecFineSmooth);
        {
            T* first = (extra % 2 == 0) ? cL_.p : cL2_.p;
            T* other = (extra % 2 == 0) ? cL2_.p : cL_.p;
            k_fine_smooth<DIM, T, double><<<FB_, kBlock, 0, stream_>>>(ctl, rows_, fop_, r, first, omega, two);
            T* cur = first;
            for (int s = 0; s < extra; ++s) {
                T* nxt = (cur == first) ? other : first;
                k_fine_sweep<DIM, T, double><<<FB_, kBlock, 0, stream_>>>(ctl, rows_, fop_, r, cur, nxt, omega);
                cur = nxt;
            }
            cL_final_ = cur;
        }
    }

    // restriction chain: big levels one launch each, the small ones in one block
    void enqueue_restrict_chain(const Ctl* ctl, const double* r) {
        const int L = L_;
        const T omega = T(opt_.omega);
        const int l = L - 1;
        k_restrict<DIM, double, T><<<(N_[l] + kBlock - 1) / kBlock, kBlock, 0, stream_>>>(
            ctl, r, n_axis[L], g_[l].p, n_axis[l], N_[l], diag(l), c1_[l].p, omega, cst_[l]);
        int m = L - 2;
        for (; m >= 0 && N_[m] > kRestrictTailMax; --m)
            k_restrict<DIM, T, T><<<(N_[m] + kBlock - 1) / kBlock, kBlock, 0, stream_>>>(
                ctl, g_[m + 1].p, n_axis[m + 1], g_[m].p, n_axis[m], N_[m], diag(m), c1_[m].p, omega, cst_[m]);
        if (m >= 0) {
            RestrictChain<T> ch{};
            for (; m >= 0; --m) {
                const int q = ch.count++;
                ch.nf[q] = n_axis[m + 1];
                ch.nc[q] = n_axis[m];
                ch.Nc[q] = N_[m];
                ch.gf[q] = g_[m + 1].p;
                ch.gc[q] = g_[m].p;
                ch.D[q] = diag(m);
                ch.dconst[q] = cst_[m];
                ch.c1[q] = c1_[m].p;
            }
            k_restrict_tail<DIM, T><<<1, kTailBlock, 0, stream_>>>(ctl, ch, omega);
        }
    }

    // the coarse levels: restriction chain, smoothing, prolongation chain
    void enqueue_coarse(const Ctl* ctl, const double* r) {
        const int L = L_;
        const T omega = T(opt_.omega);
        const int nu = opt_.nu;
        const int two = nu >= 2 ? 1 : 0;
        const int extra = nu > 2 ? nu - 2 : 0;
        if (L == 0) return;
        mark(kSecRestrict);
        enqueue_restrict_chain(ctl, r);
        // all coarse levels smoothed in one launch (per sweep); the final sweep
        // writes c_l into the last column of the level's block carry
        mark(kSecCoarseSmooth);
        {
            const int two_f = two;
            if (extra == 0) {
                CoarseLevels<T> cl = coarse_arg(1);
                k_coarse_smooth<DIM, T><<<cl.blk_off[L], kBlock, 0, stream_>>>(ctl, cl, omega, 0, two_f);
            } else {
                CoarseLevels<T> cl = coarse_arg(0);     // first sweeps into c_
                k_coarse_smooth<DIM, T><<<cl.blk_off[L], kBlock, 0, stream_>>>(ctl, cl, omega, 0, two_f);
                for (int s2 = 0; s2 < extra; ++s2) {
                    const bool last = s2 == extra - 1;
                    const bool from_c = (s2 % 2) == 0;
                    for (int l = 0; l < L; ++l) {
                        cl.cin[l] = from_c ? c_[l].p : c2_[l].p;
                        if (last) {
                            cl.cout[l] = Y_[l].p + l;
                            cl.cstride[l] = even_up(l + 1);
                        } else {
                            cl.cout[l] = from_c ? c2_[l].p : c_[l].p;
                            cl.cstride[l] = 1;
                        }
                    }
                    k_coarse_smooth<DIM, T><<<cl.blk_off[L], kBlock, 0, stream_>>>(ctl, cl, omega, 1, two_f);
                }
            }
        }
        mark(kSecProlong);
        enqueue_prolong(ctl);
    }

    // prolongation chain Y_{l+1}[:, 0..l] = P Y_l: small levels in one block
    void enqueue_prolong(const Ctl* ctl) {
        const int L = L_;
        {
            int l = 0;
            ProlongChain<T> ch{};
            ch.l0 = 0;
            for (; l + 1 < L && N_[l + 1] <= kTailMax; ++l) {
                const int q = ch.count++;
                ch.nc[q] = n_axis[l];
                ch.nf[q] = n_axis[l + 1];
                ch.Nf[q] = N_[l + 1];
                ch.Yc[q] = Y_[l].p;
                ch.Yf[q] = Y_[l + 1].p;
            }
            if (ch.count > 0) k_prolong_head<DIM, T><<<1, kTailBlock, 0, stream_>>>(ctl, ch);
            for (; l + 1 < L; ++l) launch_prolong(ctl, l);
        }
    }

    double* part_init() { return part_.p; }
    double* part_rho() { return part_.p + (size_t)FB_ * 2; }
    double* part_W() { return part_.p + (size_t)FB_ * 3; }
    double* part_G() { return partG_.p; }

    // Q = A P and the Gram partials (spmm_blocks<NB>() partial rows at
    // part_G()): z-marching on 3D grids for blocks of <= 48 bytes per node,
    // row-mapped otherwise.
    // grid of the x/P update: one round of its resident blocks (5 per CU up
    // to 6 columns; wider blocks keep the fine grid)
    template <int NB>
    int xp_grid() const {
        return xp_blocks_per_cu<NB>() == xp_blocks_per_cu<1>() ? XPB_ : FB_;
    }

    // blocks of the W launch per stored slot: one round of the resident
    // blocks of that kernel instance (its occupancy), at most kGramBlocks
    template <int NB, int NE>
    int fw_grid() const {
        static const int per_cu = [] {
            int b = 0;
            HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_fine_W<DIM, T, NB, NE>, kBlock, 0));
            return std::max(b, 1);
        }();
        return fine_blocks(rows_.total, std::min(kGramBlocks, per_cu * kNumCU));
    }

    template <int NB>
    int spmm_blocks() const {
        if constexpr (DIM == 3 && zt_fits<T, NB>()) return SB_[zvar<NB>()];
        return FBG_;
    }
    // unit split of the z-marching kernel: 0 for 2 resident blocks per CU, 1 for 3
    template <int NB>
    int zvar() const {
        return (fop_.D ? zt_min_blocks<T, NB, true>() : zt_min_blocks<T, NB, false>()) - 2;
    }
    template <int NB>
    void launch_spmm(const Ctl* c, const T* P, T* Q, const double* r, hipStream_t s) {
        if constexpr (DIM == 3 && zt_fits<T, NB>()) {
            const long long pbytes = (long long)((P_.p + P_.n) - P) * (long long)sizeof(T);
            const int n = n_axis[L_], v = zvar<NB>();
            if (fop_.D)
                k_spmm_gram_z<T, NB, kZTY, true><<<SB_[v], kBlock, 0, s>>>(c, n, zntx_, zkz_[v], znkz_[v], fop_, P,
                                                                          pbytes, Q, r, part_G());
            else
                k_spmm_gram_z<T, NB, kZTY, false><<<SB_[v], kBlock, 0, s>>>(c, n, zntx_, zkz_[v], znkz_[v], fop_, P,
                                                                           pbytes, Q, r, part_G());
        } else {
            k_spmm_gram<DIM, T, NB><<<FBG_, kBlock, 0, s>>>(c, rows_, fop_, P, Q, r, part_G());
        }
    }
    double* part_ref() { return part_.p + (size_t)FB_ * (kPartRow - 1); }
    double* d_alpha() { return small_.p; }
    // beta_j and G_j^+ of the window's slot j (kMaxNB^2 doubles each)
    double* d_beta(int j = 0) { return small_.p + kMaxNB + (size_t)j * kMaxNB * kMaxNB; }
    double* d_Gplus(int j = 0) { return small_.p + kMaxNB + (size_t)(kMaxWin + j) * kMaxNB * kMaxNB; }
    T* Pslot(int j) { return P_.p + (size_t)j * pstride_; }
    T* Qslot(int j) { return Q_.p + (size_t)j * pstride_; }
    // W partials of every stored slot: slot j of a launch with nbs blocks per
    // slot starts at j kMaxNB^2 nbs (nbs <= FBG_, for which it is sized)
    double* part_Wall() { return partWin_.p; }
    PWin<T> window() {
        PWin<T> w{};
        for (int j = 0; j < m_; ++j) w.p[j] = Pslot(j);
        return w;
    }
    PWin<T> single() {
        PWin<T> w{};
        w.p[0] = Pslot(0);
        return w;
    }

    void enqueue_init(double tol) {
        const int N = N_[L_];
        k_init_residual<DIM><<<FB_, kBlock, 0, stream_>>>(rows_, f64_, b_.p, x_.p, r_.p, part_init());
        k_reduce_init<<<1, kRedBlock, 0, stream_>>>(ctl_, part_init(), FB_, tol, hist_cap_ ? rhist_.p : nullptr);
        k_zero_if<<<FB_, kBlock, 0, stream_>>>(ctl_, x_.p, N);
        if (method_ != AMGMPCG_METHOD_MPCG) {
            // comparison methods: p_0 = z_0 = B r_0, one direction
            T* z = precondition(ctl_, r_.p);
            k_xP1<T><<<FB_, kBlock, 0, stream_>>>(ctl_, N, Pslot(0), z, x_.p, d_alpha(), d_beta(), 1);
            launch_spmm<1>(ctl_, Pslot(0), Qslot(0), r_.p, stream_);
            k_reduce_alpha<1><<<1, kRedBlock, 0, stream_>>>(ctl_, part_G(), spmm_blocks<1>(), d_Gplus(0), d_alpha(),
                                                         hist_cap_ ? ahist_.p : nullptr);
            return;
        }
        enqueue_mg(ctl_, r_.p);
        dispatch_nb([&](auto nbc) {
            constexpr int NB = decltype(nbc)::value;
            [[maybe_unused]] constexpr int NE = decltype(nbc)::ne;
            const int nc = L_ > 0 ? n_axis[L_ - 1] : 1;
            k_update_xP<DIM, T, NB, NE><<<xp_grid<NB>(), kBlock, 0, stream_>>>(ctl_, rows_, fine_Y(), nc, cL_final_, dl(),
                                                                       dflag(), window(), m_, 0, 0, x_.p, d_alpha(),
                                                                       d_beta(), 1);
            launch_spmm<NB>(ctl_, Pslot(0), Qslot(0), r_.p, stream_);
            k_reduce_alpha<NB><<<1, kRedBlock, 0, stream_>>>(ctl_, part_G(), spmm_blocks<NB>(), d_Gplus(0), d_alpha(),
                                                          hist_cap_ ? ahist_.p : nullptr);
        });
    }

    // Iteration j (0-based count of x updates): P_j sits in slot j mod m and
    // P_{j+1} goes into slot (j+1) mod m.
    void enqueue_iteration(hipStream_t s, int j) {
        const int N = N_[L_];
        const int cur = j % m_, nxt = (j + 1) % m_;
        hipStream_t saved = stream_;
        stream_ = s;
        if (method_ != AMGMPCG_METHOD_MPCG) {
            enqueue_iteration_pcg(s);
            stream_ = saved;
            return;
        }
        dispatch_nb([&](auto nbc) {
            constexpr int NB = decltype(nbc)::value;
            [[maybe_unused]] constexpr int NE = decltype(nbc)::ne;
            const int nc = L_ > 0 ? n_axis[L_ - 1] : 1;
            mark(kSecUpdateR);
            k_update_r<T, NB><<<FB_, kBlock, 0, s>>>(ctl_, N, Qslot(cur), d_alpha(), r_.p, part_rho());
            enqueue_mg(ctl_, r_.p);
            mark(kSecFineW);
            // W_j for every stored block of the window in one launch
            const int fw = fw_grid<NB, NE>();
            k_fine_W<DIM, T, NB, NE><<<m_ * fw, kBlock, 0, s>>>(
                ctl_, rows_, fine_Y(), nc, cL_final_, dl(), dflag(), Qslot(0), pstride_, part_Wall(),
                (size_t)kMaxNB * kMaxNB * fw, fw);
            mark(kSecReduceBeta);
            k_reduce_beta<NB><<<1, kRedBlock, 0, s>>>(ctl_, part_rho(), FB_, part_Wall(), fw, m_, cur,
                                                   d_Gplus(0), d_beta(0), hist_cap_ ? rhist_.p : nullptr,
                                                   mixed_ ? 1 : 0);
            mark(kSecUpdateXP);
            if (prof_on_)
                launch_with_events(k_update_xP<DIM, T, NB, NE>, dim3(xp_grid<NB>()), dim3(kBlock), s, xp_events(),
                                   xp_ev_[1], ctl_, rows_, fine_Y(), nc, cL_final_, dl(), dflag(), window(), m_, cur,
                                   nxt, x_.p, d_alpha(), d_beta(0), 0);
            else
                k_update_xP<DIM, T, NB, NE><<<xp_grid<NB>(), kBlock, 0, s>>>(ctl_, rows_, fine_Y(), nc, cL_final_, dl(),
                                                                dflag(), window(), m_, cur, nxt, x_.p, d_alpha(),
                                                                d_beta(0), 0);
            if (mixed_) {
                mark(kSecRefresh);
                k_refresh<DIM><<<FB_, kBlock, 0, s>>>(ctl_, rows_, f64_, b_.p, x_.p, r_.p, part_ref());
                k_refresh_reduce<<<1, kRedBlock, 0, s>>>(ctl_, part_ref(), FB_, hist_cap_ ? rhist_.p : nullptr);
            }
            mark(kSecSpmmGram);
            launch_spmm<NB>(ctl_, Pslot(nxt), Qslot(nxt), r_.p, s);
            mark(kSecReduceAlpha);
            k_reduce_alpha<NB><<<1, kRedBlock, 0, s>>>(ctl_, part_G(), spmm_blocks<NB>(), d_Gplus(nxt), d_alpha(),
                                                    hist_cap_ ? ahist_.p : nullptr);
            mark(kSecEnd);
        });
        stream_ = saved;
    }

    // One iteration of a comparison method (CG, one direction, m = 1): the
    // MPCG iteration with the block replaced by z = B r.
    void enqueue_iteration_pcg(hipStream_t s) {
        const int N = N_[L_];
        mark(kSecUpdateR);
        k_update_r<T, 1><<<FB_, kBlock, 0, s>>>(ctl_, N, Qslot(0), d_alpha(), r_.p, part_rho());
        T* z = precondition(ctl_, r_.p);
        mark(kSecFineW);
        k_W1<T><<<FB_, kBlock, 0, s>>>(ctl_, N, Qslot(0), z, part_Wall());
        mark(kSecReduceBeta);
        k_reduce_beta<1><<<1, kRedBlock, 0, s>>>(ctl_, part_rho(), FB_, part_Wall(), FB_, 1, 0, d_Gplus(0),
                                              d_beta(0), hist_cap_ ? rhist_.p : nullptr, mixed_ ? 1 : 0);
        mark(kSecUpdateXP);
        if (prof_on_)
            launch_with_events(k_xP1<T>, dim3(FB_), dim3(kBlock), s, xp_events(), xp_ev_[1], ctl_, N, Pslot(0), z,
                               x_.p, d_alpha(), d_beta(0), 0);
        else
            k_xP1<T><<<FB_, kBlock, 0, s>>>(ctl_, N, Pslot(0), z, x_.p, d_alpha(), d_beta(0), 0);
        if (mixed_) {
            mark(kSecRefresh);
            k_refresh<DIM><<<FB_, kBlock, 0, s>>>(ctl_, rows_, f64_, b_.p, x_.p, r_.p, part_ref());
            k_refresh_reduce<<<1, kRedBlock, 0, s>>>(ctl_, part_ref(), FB_, hist_cap_ ? rhist_.p : nullptr);
        }
        mark(kSecSpmmGram);
        launch_spmm<1>(ctl_, Pslot(0), Qslot(0), r_.p, s);
        mark(kSecReduceAlpha);
        k_reduce_alpha<1><<<1, kRedBlock, 0, s>>>(ctl_, part_G(), spmm_blocks<1>(), d_Gplus(0), d_alpha(),
                                               hist_cap_ ? ahist_.p : nullptr);
        mark(kSecEnd);
    }

    // z = B r of a comparison method; returns the device vector holding z.
    T* precondition(const Ctl* ctl, const double* r) {
        if (method_ == AMGMPCG_METHOD_ADDITIVE_PCG) {
            enqueue_mg(ctl, r);
            mark(kSecFineW);
            dispatch_plain([&](auto nlc) {
                constexpr int NL = decltype(nlc)::value;
                const int nc = L_ > 0 ? n_axis[L_ - 1] : 1;
                k_sum_z<DIM, T, NL><<<FB_, kBlock, 0, stream_>>>(ctl, rows_, fine_Y(), nc, cL_final_, zv_.p);
            });
            return zv_.p;
        }
        return enqueue_vcycle(ctl, r);
    }

    // ---- V-cycle (multiplicative MG, Sec. 2.1) -------------------------
    // damped-Jacobi sweeps on the finest level: `count` sweeps from zero
    // (count >= 1), or `count` sweeps from `start`; results ping-pong between
    // vcL_ and vtL_, the buffer holding the result is returned.
    T* vc_fine_from_zero(const Ctl* ctl, const double* r, int count) {
        const T omega = T(opt_.omega);
        k_fine_smooth<DIM, T, double><<<FB_, kBlock, 0, stream_>>>(ctl, rows_, fop_, r, vcL_.p, omega,
                                                                   count >= 2 ? 1 : 0);
        return vc_fine_sweeps(ctl, r, vcL_.p, count - std::min(count, 2));
    }
    T* vc_fine_sweeps(const Ctl* ctl, const double* r, T* cur, int count) {
        const T omega = T(opt_.omega);
        for (int s = 0; s < count; ++s) {
            T* nxt = cur == vcL_.p ? vtL_.p : vcL_.p;
            k_fine_sweep<DIM, T, double><<<FB_, kBlock, 0, stream_>>>(ctl, rows_, fop_, r, cur, nxt, omega);
            cur = nxt;
        }
        return cur;
    }
    T* vc_coarse_sweeps(const Ctl* ctl, int l, T* cur, int count) {
        const T omega = T(opt_.omega);
        CoarseOp<T> op{n_axis[l], N_[l], coef_[l].p, cst_[l]};
        const int blocks = (N_[l] + kBlock - 1) / kBlock;
        for (int s = 0; s < count; ++s) {
            T* nxt = cur == vc_[l].p ? vt_[l].p : vc_[l].p;
            k_vc_coarse<DIM, T><<<blocks, kBlock, 0, stream_>>>(ctl, op, vg_[l].p, cur, nxt, omega, 1);
            cur = nxt;
        }
        return cur;
    }

    // One V-cycle for A c = r from c = 0: nu sweeps before and after the
    // coarse correction on every level but the coarsest (2 nu sweeps from
    // zero); the restriction kernels also write the first sweep from zero of
    // the coarser level.  Returns the vector holding c on the finest level.
    T* enqueue_vcycle(const Ctl* ctl, const double* r) {
        const T omega = T(opt_.omega);
        const int nu = vnu_, L = L_;
        mark(kSecFineSmooth);
        if (L == 0) return vc_fine_from_zero(ctl, r, 2 * nu);
        T* cf = vc_fine_from_zero(ctl, r, nu);
        mark(kSecRestrict);
        k_fine_resid<DIM, T, double><<<FB_, kBlock, 0, stream_>>>(ctl, rows_, fop_, r, cf, vrL_.p);
        k_restrict<DIM, T, T><<<(N_[L - 1] + kBlock - 1) / kBlock, kBlock, 0, stream_>>>(
            ctl, vrL_.p, n_axis[L], vg_[L - 1].p, n_axis[L - 1], N_[L - 1], diag(L - 1), vc_[L - 1].p, omega, cst_[L - 1]);
        std::vector<T*> c(L, nullptr);
        for (int l = L - 1; l >= 1; --l) {
            c[l] = vc_coarse_sweeps(ctl, l, vc_[l].p, nu - 1);
            CoarseOp<T> op{n_axis[l], N_[l], coef_[l].p, cst_[l]};
            k_vc_coarse<DIM, T><<<(N_[l] + kBlock - 1) / kBlock, kBlock, 0, stream_>>>(ctl, op, vg_[l].p, c[l],
                                                                                     vr_[l].p, omega, 2);
            k_restrict<DIM, T, T><<<(N_[l - 1] + kBlock - 1) / kBlock, kBlock, 0, stream_>>>(
                ctl, vr_[l].p, n_axis[l], vg_[l - 1].p, n_axis[l - 1], N_[l - 1], diag(l - 1), vc_[l - 1].p, omega, cst_[l - 1]);
        }
        mark(kSecCoarseSmooth);
        c[0] = vc_coarse_sweeps(ctl, 0, vc_[0].p, 2 * nu - 1);
        mark(kSecProlong);
        for (int l = 1; l < L; ++l) {
            k_prolong_add<DIM, T><<<(N_[l] + kBlock - 1) / kBlock, kBlock, 0, stream_>>>(ctl, c[l - 1], n_axis[l - 1],
                                                                                       c[l], n_axis[l], N_[l]);
            c[l] = vc_coarse_sweeps(ctl, l, c[l], nu);
        }
        k_prolong_add<DIM, T><<<(N_[L] + kBlock - 1) / kBlock, kBlock, 0, stream_>>>(ctl, c[L - 1], n_axis[L - 1], cf,
                                                                                   n_axis[L], N_[L]);
        return vc_fine_sweeps(ctl, r, cf, nu);
    }

    // ---- per-section timing inside real iterations --------------------
    // mark(sec) records an event before the launches of section sec; a
    // section lasts until the next mark.  A no-op outside profile_solve, in
    // particular during graph capture.
    // The event pair bound to the x/P update's dispatch; start event returned.
    hipEvent_t xp_events() {
        for (hipEvent_t& e : xp_ev_)
            if (!e) HIPCHK(hipEventCreate(&e));
        xp_rec_ = true;
        return xp_ev_[0];
    }

    void mark(int sec) {
        if (!prof_on_) return;
        if (prof_n_ == (int)prof_ev_.size()) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e));
            prof_ev_.push_back(e);
        }
        HIPCHK(hipEventRecord(prof_ev_[prof_n_], stream_));
        prof_sec_.resize(prof_n_ + 1);
        prof_sec_[prof_n_++] = sec;
    }

    // As solve(), with each iteration launched eagerly between events: the
    // average duration (ms) of each section over the iterations that ran in
    // full (not the last, whose SpMM and alpha step the stop flag skips).
    int profile_solve(const double* b_dev, double* x_dev, double tol, int maxit, amgmpcg_info* info, double* ms,
                      int cap, int* samples) override {
        const int N = N_[L_];
        if (maxit <= 0) maxit = opt_.maxit;
        Ctl& c = *hctl_in_;
        std::memset(&c, 0, sizeof(Ctl));
        c.maxit = maxit;
        c.hist_cap = std::min(hist_cap_, maxit);
        c.drop2 = opt_.refresh_drop * opt_.refresh_drop;
        c.tau = tau_;
        HIPCHK(hipMemcpyAsync(ctl_, hctl_in_, sizeof(Ctl), hipMemcpyHostToDevice, stream_));
        HIPCHK(hipMemcpyAsync(b_.p, b_dev, (size_t)N * sizeof(double), hipMemcpyDeviceToDevice, stream_));
        HIPCHK(hipMemcpyAsync(x_.p, x_dev, (size_t)N * sizeof(double), hipMemcpyDeviceToDevice, stream_));
        clear_window();
        enqueue_init(tol);
        HIPCHK(hipGetLastError());
        double sum[kSecCount] = {0.0};
        int full = 0;
        for (int it = 0; it <= maxit; ++it) {
            HIPCHK(hipMemcpyAsync(hctl_, ctl_, sizeof(Ctl), hipMemcpyDeviceToHost, stream_));
            HIPCHK(hipStreamSynchronize(stream_));
            if (hctl_->state != 0) break;
            prof_on_ = true;
            prof_n_ = 0;
            xp_rec_ = false;
            enqueue_iteration(stream_, it);
            prof_on_ = false;
            HIPCHK(hipGetLastError());
            HIPCHK(hipMemcpyAsync(hctl_, ctl_, sizeof(Ctl), hipMemcpyDeviceToHost, stream_));
            HIPCHK(hipStreamSynchronize(stream_));
            if (hctl_->state != 0) continue;   // the stopping iteration: partly skipped
            ++full;
            for (int k = 0; k + 1 < prof_n_; ++k) {
                float t = 0.f;
                HIPCHK(hipEventElapsedTime(&t, prof_ev_[k], prof_ev_[k + 1]));
                sum[prof_sec_[k]] += t;
            }
            float t = 0.f;
            HIPCHK(hipEventElapsedTime(&t, prof_ev_[0], prof_ev_[prof_n_ - 1]));
            sum[kSecEnd] += t;
            if (xp_rec_) {
                HIPCHK(hipEventElapsedTime(&t, xp_ev_[0], xp_ev_[1]));
                sum[kSecXPKernel] += t;
            }
        }
        HIPCHK(hipMemcpyAsync(x_dev, x_.p, (size_t)N * sizeof(double), hipMemcpyDeviceToDevice, stream_));
        HIPCHK(hipMemcpyAsync(hctl_, ctl_, sizeof(Ctl), hipMemcpyDeviceToHost, stream_));
        HIPCHK(hipStreamSynchronize(stream_));
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
            info->solve_ms = 0.0;
            info->relres_true = -1.0;
        }
        for (int k = 0; k < kSecCount && k < cap; ++k) ms[k] = full ? sum[k] / full : 0.0;
        if (samples) *samples = full;
        return kSecCount;
    }


    void capture_graph() {
        if (!cap_stream_) HIPCHK(hipStreamCreateWithFlags(&cap_stream_, hipStreamNonBlocking));
        HIPCHK(hipStreamBeginCapture(cap_stream_, hipStreamCaptureModeThreadLocal));
        for (int k = 0; k < kpoll_; ++k) enqueue_iteration(cap_stream_, k);
        hipError_t launch_err = hipGetLastError();
        HIPCHK(hipStreamEndCapture(cap_stream_, &graph_));
        HIPCHK(launch_err);
        HIPCHK(hipGraphInstantiate(&exec_, graph_, nullptr, nullptr, 0));
        graph_ready_ = true;
    }

    enum : int {
        kSecUpdateR,
        kSecFineSmooth,
        kSecRestrict,
        kSecCoarseSmooth,
        kSecProlong,
        kSecLearned,
        kSecFineW,
        kSecReduceBeta,
        kSecUpdateXP,
        kSecRefresh,
        kSecSpmmGram,
        kSecReduceAlpha,
        kSecEnd,          // slot of the whole iteration
        kSecXPKernel,     // the x/P update launch alone, timed by its dispatch
        kSecCount
    };
    bool prof_on_ = false;
    hipStream_t side_ = nullptr;
    hipEvent_t ev_fork_ = nullptr, ev_join_ = nullptr;
    int prof_n_ = 0;
    std::vector<hipEvent_t> prof_ev_;
    std::vector<int> prof_sec_;
    hipEvent_t xp_ev_[2] = {nullptr, nullptr};   // the x/P update's own dispatch (profile_solve)
    bool xp_rec_ = false;

    amgmpcg_options opt_;
    hipStream_t stream_;
    hipStream_t cap_stream_ = nullptr;
    hipGraph_t graph_ = nullptr;
    hipGraphExec_t exec_ = nullptr;
    bool graph_ready_ = false;
    bool mixed_ = false;
    int L_ = 0, FB_ = 1, FBG_ = 1, XPB_ = 1, hist_cap_ = 0, last_iters_ = 0;
    int method_ = AMGMPCG_METHOD_MPCG, vnu_ = 1;   // solution method; V-cycle sweeps per side
    // z-marching SpMM: x tiles; per resident-block count (2, 3): planes per
    // unit, z chunks, units (= blocks)
    int zntx_ = 1, zkz_[2] = {1, 1}, znkz_[2] = {1, 1}, SB_[2] = {1, 1};
    int m_ = 1, kpoll_ = 1;      // truncation window; iterations per captured graph (a multiple of m)
    size_t pstride_ = 0;         // elements per direction block slot
    double tau_ = 0.0;
    std::vector<int> N_;
    FineOp<T> fop_{};
    Rows rows_{};
    FineOp<double> f64_{};
    DevBuf<T> fD_, fex_, fey_, fez_, fiD_;
    DevBuf<double> gD_, gex_, gey_, gez_, giD_;
    std::vector<DevBuf<T>> coef_, g_, c1_, c_, c2_, Y_;
    T* cL_final_ = nullptr;
    DevBuf<double> x_, r_, b_, part_, small_, ahist_, rhist_, partWin_, partG_;
    DevBuf<T> P_, Q_, cL_, cL2_, dl_;
    DevBuf<T> zv_, vcL_, vtL_, vrL_;
    std::vector<int> cst_;                             // per coarse level: constant stencil (coef_ holds 3^d values)                   // comparison methods: z = B r; fine V-cycle vectors
    std::vector<DevBuf<T>> vg_, vc_, vt_, vr_;         // coarse V-cycle vectors (rhs, iterate x2, residual)
    DevBuf<double> xt_;
    DevBuf<unsigned short> lk_;
    Ctl* ctl_ = nullptr;
    Ctl* ctl_free_ = nullptr;
    Ctl* ctl_proj_ = nullptr;
    Ctl* hctl_proj_ = nullptr;
    Ctl* hctl_ = nullptr;
    Ctl* hctl_in_ = nullptr;
    hipEvent_t ev0_ = nullptr, ev1_ = nullptr;
};


}  // namespace amg
