// Host-side hierarchy construction (Sec. 2.1): the finest FD operator as a
// 3^d-point stencil, Galerkin coarse operators A_c = R A_f P with
// R = 2^-d P^T (tensor linear interpolation, coarse node J on fine node 2J+1),
// symmetrised by mirroring the upper triangle.  Multithreaded over coarse
// planes; deterministic (each coarse entry is summed by one thread in a
// fixed order).
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <stdexcept>
#include <thread>
#include <vector>
#include <utility>

namespace amg {
namespace host {

struct StencilLevel {
    int dim = 0, n = 0;
    int64_t N = 0;
    std::vector<double> coef;   // S * N, coef[s*N + idx] = A(idx, idx + o_s)
    int S() const { return dim == 2 ? 9 : 27; }
    int center() const { return dim == 2 ? 4 : 13; }
};

// Face data of the finest operator: diagonal and +x/+y/+z couplings
// (positive numbers, e[idx] = -A(idx, idx + e)), all h^-2 scaled.
struct FineFaces {
    std::vector<double> D, ex, ey, ez;
};

inline int64_t ipow(int64_t a, int e) {
    int64_t r = 1;
    while (e-- > 0) r *= a;
    return r;
}

template <typename F>
inline void parallel_for(int count, F&& body) {
    int nt = (int)std::thread::hardware_concurrency();
    nt = std::max(1, std::min(nt, std::min(count, 32)));
    if (nt == 1) {
        for (int i = 0; i < count; ++i) body(i);
        return;
    }
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t)
        th.emplace_back([&, t]() {
            for (int i = t; i < count; i += nt) body(i);
        });
    for (auto& x : th) x.join();
}

// Harmonic-mean FD operator.  kappa: (n+2)^dim node values (x fastest) or
// nullptr for kappa == 1.
inline FineFaces fine_faces(int dim, int n, const double* kappa) {
    const int64_t N = ipow(n, dim);
    const double h2inv = double(n + 1) * double(n + 1);
    FineFaces f;
    f.D.assign(N, 0.0);
    f.ex.assign(N, 0.0);
    f.ey.assign(N, 0.0);
    f.ez.assign(dim == 3 ? N : 0, 0.0);
    const int m = n + 2;
    auto K = [&](int i, int j, int k) -> double {   // node-grid coords incl. boundary
        if (!kappa) return 1.0;
        return kappa[i + (int64_t)m * (j + (int64_t)m * (dim == 3 ? k : 0))];
    };
    auto hm = [](double a, double b) { return 2.0 * a * b / (a + b); };
    const int nz = dim == 3 ? n : 1;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                const int64_t idx = i + (int64_t)n * (j + (int64_t)n * k);
                const int I = i + 1, J = j + 1, Kk = dim == 3 ? k + 1 : 0;
                const double kc = K(I, J, Kk);
                double d = 0.0;
                const double fxm = hm(kc, K(I - 1, J, Kk)), fxp = hm(kc, K(I + 1, J, Kk));
                const double fym = hm(kc, K(I, J - 1, Kk)), fyp = hm(kc, K(I, J + 1, Kk));
                d += fxm + fxp + fym + fyp;
                f.ex[idx] = h2inv * fxp;
                f.ey[idx] = h2inv * fyp;
                if (dim == 3) {
                    const double fzm = hm(kc, K(I, J, Kk - 1)), fzp = hm(kc, K(I, J, Kk + 1));
                    d += fzm + fzp;
                    f.ez[idx] = h2inv * fzp;
                }
                f.D[idx] = h2inv * d;
            }
    return f;
}

inline StencilLevel faces_to_stencil(int dim, int n, const FineFaces& f) {
    StencilLevel L;
    L.dim = dim;
    L.n = n;
    L.N = ipow(n, dim);
    const int S = L.S();
    L.coef.assign((size_t)S * L.N, 0.0);
    const int nz = dim == 3 ? n : 1;
    auto sidx = [&](int dx, int dy, int dz) { return dim == 2 ? (dy + 1) * 3 + (dx + 1) : (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1); };
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                const int64_t idx = i + (int64_t)n * (j + (int64_t)n * k);
                const int64_t sy = n, sz = (int64_t)n * n;
                L.coef[(size_t)sidx(0, 0, 0) * L.N + idx] = f.D[idx];
                if (i > 0) L.coef[(size_t)sidx(-1, 0, 0) * L.N + idx] = -f.ex[idx - 1];
                if (i < n - 1) L.coef[(size_t)sidx(1, 0, 0) * L.N + idx] = -f.ex[idx];
                if (j > 0) L.coef[(size_t)sidx(0, -1, 0) * L.N + idx] = -f.ey[idx - sy];
                if (j < n - 1) L.coef[(size_t)sidx(0, 1, 0) * L.N + idx] = -f.ey[idx];
                if (dim == 3) {
                    if (k > 0) L.coef[(size_t)sidx(0, 0, -1) * L.N + idx] = -f.ez[idx - sz];
                    if (k < n - 1) L.coef[(size_t)sidx(0, 0, 1) * L.N + idx] = -f.ez[idx];
                }
            }
    return L;
}

// Galerkin product R A P for one level; nc = floor(nf / 2).
// True if every node's stencil equals the stencil of the middle node with
// the couplings to nodes outside the grid dropped (exact comparison); then
// the level can be stored as those 3^d values.  Galerkin products of a
// constant-coefficient operator have this form on grids of odd size.
inline bool constant_with_truncation(const StencilLevel& L) {
    const int n = L.n, dim = L.dim;
    const int c = n / 2;
    const int64_t ref = c + (int64_t)n * (c + (dim == 3 ? (int64_t)n * c : 0));
    for (int64_t idx = 0; idx < L.N; ++idx) {
        const int i = (int)(idx % n), j = (int)((idx / n) % n), k = dim == 3 ? (int)(idx / ((int64_t)n * n)) : 0;
        int s = 0;
        for (int dz = (dim == 3 ? -1 : 0); dz <= (dim == 3 ? 1 : 0); ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx, ++s) {
                    const bool in = i + dx >= 0 && i + dx < n && j + dy >= 0 && j + dy < n &&
                                    (dim == 2 || (k + dz >= 0 && k + dz < n));
                    const double want = in ? L.coef[(size_t)s * L.N + ref] : 0.0;
                    if (L.coef[(size_t)s * L.N + idx] != want) return false;
                }
    }
    return true;
}

// ------------------------------------------------------ sparse hierarchy
// General hierarchies (Sec. 2.1 with given transfer operators): CSR
// matrices on the host, Galerkin products R A P by row-wise sparse products.

struct Csr {
    int n = 0, m = 0;            // rows, columns
    std::vector<int> ptr, col;   // ptr: n + 1
    std::vector<double> val;
    int64_t nnz() const { return (int64_t)col.size(); }
};

// The sliced layout the device kernels read a CSR matrix in: slices of 64
// consecutive rows, each padded to its longest row and stored column by
// column (entry k of row 64 s + l at off[s] + 64 k + l).  A row's entries
// come in CSR order, then padding of weight 0 at the row's first column
// (column 0 for an empty row), so a row sum over the layout is the CSR one
// followed by exact zeros.  False when the layout would not fit int32
// offsets.
struct Sliced {
    std::vector<int> off, wid, col;
    std::vector<double> val;
};

inline bool csr_sliced(const Csr& M, Sliced& S) {
    const int ns = (M.n + 63) / 64;
    S.off.assign(ns, 0);
    S.wid.assign(ns, 0);
    long long total = 0;
    for (int s = 0; s < ns; ++s) {
        int w = 0;
        for (int r = s * 64; r < std::min(M.n, s * 64 + 64); ++r) w = std::max(w, M.ptr[r + 1] - M.ptr[r]);
        S.off[s] = (int)total;
        S.wid[s] = w;
        total += 64LL * w;
        if (total > INT32_MAX) return false;
    }
    S.col.assign((size_t)std::max<long long>(total, 1), 0);
    S.val.assign((size_t)std::max<long long>(total, 1), 0.0);
    for (int s = 0; s < ns; ++s)
        for (int l = 0; l < 64; ++l) {
            const int r = s * 64 + l;
            if (r >= M.n) break;
            const int b = M.ptr[r], len = M.ptr[r + 1] - b;
            for (int k = 0; k < S.wid[s]; ++k) {
                const size_t e = (size_t)S.off[s] + 64 * (size_t)k + l;
                if (k < len) {
                    S.col[e] = M.col[b + k];
                    S.val[e] = M.val[b + k];
                } else {
                    S.col[e] = len > 0 ? M.col[b] : 0;
                }
            }
        }
    return true;
}

inline Csr csr_transpose(const Csr& A, double scale = 1.0) {
    Csr T;
    T.n = A.m;
    T.m = A.n;
    T.ptr.assign(T.n + 1, 0);
    for (int c : A.col) ++T.ptr[c + 1];
    for (int i = 0; i < T.n; ++i) T.ptr[i + 1] += T.ptr[i];
    T.col.resize(A.col.size());
    T.val.resize(A.col.size());
    std::vector<int> next(T.ptr.begin(), T.ptr.end() - 1);
    for (int i = 0; i < A.n; ++i)
        for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
            const int q = next[A.col[k]]++;
            T.col[q] = i;
            T.val[q] = scale * A.val[k];
        }
    return T;
}

// C = A B, each row summed in ascending order of A's entries, columns sorted.
inline Csr csr_multiply(const Csr& A, const Csr& B) {
    if (A.m != B.n) throw std::invalid_argument("inner dimensions differ");
    Csr C;
    C.n = A.n;
    C.m = B.m;
    std::vector<std::vector<int>> cols(A.n);
    std::vector<std::vector<double>> vals(A.n);
    const int nt = std::max(1, std::min(16, (int)std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t)
        th.emplace_back([&, t] {
            std::vector<double> acc(B.m, 0.0);
            std::vector<char> used(B.m, 0);
            std::vector<int> list;
            for (int i = t; i < A.n; i += nt) {
                list.clear();
                for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
                    const int j = A.col[k];
                    const double a = A.val[k];
                    for (int q = B.ptr[j]; q < B.ptr[j + 1]; ++q) {
                        const int c = B.col[q];
                        if (!used[c]) {
                            used[c] = 1;
                            acc[c] = 0.0;
                            list.push_back(c);
                        }
                        acc[c] += a * B.val[q];
                    }
                }
                std::sort(list.begin(), list.end());
                cols[i] = list;
                vals[i].resize(list.size());
                for (size_t q = 0; q < list.size(); ++q) {
                    vals[i][q] = acc[list[q]];
                    used[list[q]] = 0;
                }
            }
        });
    for (auto& x : th) x.join();
    C.ptr.assign(C.n + 1, 0);
    for (int i = 0; i < C.n; ++i) C.ptr[i + 1] = C.ptr[i] + (int)cols[i].size();
    C.col.reserve(C.ptr[C.n]);
    C.val.reserve(C.ptr[C.n]);
    for (int i = 0; i < C.n; ++i) {
        C.col.insert(C.col.end(), cols[i].begin(), cols[i].end());
        C.val.insert(C.val.end(), vals[i].begin(), vals[i].end());
    }
    return C;
}

// Upper triangle (with the diagonal) kept and mirrored: a symmetric matrix.
inline Csr csr_symmetrise_upper(const Csr& A) {
    Csr U;
    U.n = A.n;
    U.m = A.m;
    U.ptr.assign(A.n + 1, 0);
    for (int i = 0; i < A.n; ++i) {
        for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
            if (A.col[k] >= i) {
                U.col.push_back(A.col[k]);
                U.val.push_back(A.val[k]);
            }
        U.ptr[i + 1] = (int)U.col.size();
    }
    // mirror: entries (i, j), j > i, also as (j, i)
    std::vector<std::vector<std::pair<int, double>>> rows(A.n);
    for (int i = 0; i < U.n; ++i)
        for (int k = U.ptr[i]; k < U.ptr[i + 1]; ++k) {
            rows[i].push_back({U.col[k], U.val[k]});
            if (U.col[k] != i) rows[U.col[k]].push_back({i, U.val[k]});
        }
    Csr S;
    S.n = A.n;
    S.m = A.m;
    S.ptr.assign(A.n + 1, 0);
    for (int i = 0; i < A.n; ++i) {
        std::sort(rows[i].begin(), rows[i].end());
        for (auto& e : rows[i]) {
            S.col.push_back(e.first);
            S.val.push_back(e.second);
        }
        S.ptr[i + 1] = (int)S.col.size();
    }
    return S;
}

// Galerkin coarse operator R A P with R = scale P^T, stored symmetrised.
inline Csr csr_galerkin(const Csr& A, const Csr& P, double scale) {
    const Csr AP = csr_multiply(A, P);
    const Csr R = csr_transpose(P, scale);
    return csr_symmetrise_upper(csr_multiply(R, AP));
}

inline std::vector<double> csr_diagonal(const Csr& A) {
    std::vector<double> d(A.n, 0.0);
    for (int i = 0; i < A.n; ++i)
        for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
            if (A.col[k] == i) d[i] += A.val[k];
    return d;
}

// A == A^T up to rtol relative to the largest |a_ij| (same pattern not required).
inline bool csr_symmetric(const Csr& A, double rtol) {
    const Csr T = csr_transpose(A);
    double amax = 0.0;
    for (double v : A.val) amax = std::max(amax, std::fabs(v));
    std::vector<double> row(A.m, 0.0);
    for (int i = 0; i < A.n; ++i) {
        for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k) row[A.col[k]] += A.val[k];
        for (int k = T.ptr[i]; k < T.ptr[i + 1]; ++k) row[T.col[k]] -= T.val[k];
        bool ok = true;
        for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k) ok = ok && std::fabs(row[A.col[k]]) <= rtol * amax;
        for (int k = T.ptr[i]; k < T.ptr[i + 1]; ++k) ok = ok && std::fabs(row[T.col[k]]) <= rtol * amax;
        for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k) row[A.col[k]] = 0.0;
        for (int k = T.ptr[i]; k < T.ptr[i + 1]; ++k) row[T.col[k]] = 0.0;
        if (!ok) return false;
    }
    return true;
}

// A constant 2D 9-point stencil w (w[(dy+1)*3 + dx+1] = A(idx, idx + dx + n dy))
// on the n x n interior nodes; couplings to nodes outside the grid dropped
// (homogeneous Dirichlet).
inline StencilLevel constant_stencil9(int n, const double* w) {
    StencilLevel L;
    L.dim = 2;
    L.n = n;
    L.N = ipow(n, 2);
    L.coef.assign((size_t)9 * L.N, 0.0);
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            const int64_t idx = i + (int64_t)n * j;
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    if (i + dx < 0 || i + dx >= n || j + dy < 0 || j + dy >= n) continue;
                    const int sidx = (dy + 1) * 3 + (dx + 1);
                    L.coef[(size_t)sidx * L.N + idx] = w[sidx];
                }
        }
    return L;
}

inline StencilLevel galerkin(const StencilLevel& F) {
    const int dim = F.dim, nf = F.n, nc = nf / 2;
    if (nc < 1) throw std::invalid_argument("grid too small for another level");
    StencilLevel C;
    C.dim = dim;
    C.n = nc;
    C.N = ipow(nc, dim);
    const int S = F.S();
    C.coef.assign((size_t)S * C.N, 0.0);
    const int nzc = dim == 3 ? nc : 1;
    const double rscale = dim == 3 ? 0.125 : 0.25;
    // per-axis parents of a fine coordinate
    auto par = [&](int f, int* J, double* w) -> int {
        if (f & 1) {
            J[0] = (f - 1) / 2;
            w[0] = 1.0;
            return 1;
        }
        int c = 0;
        const int Jm = f / 2;
        if (Jm - 1 >= 0) { J[c] = Jm - 1; w[c++] = 0.5; }
        if (Jm < nc) { J[c] = Jm; w[c++] = 0.5; }
        return c;
    };
    parallel_for(nzc, [&](int cz) {
        for (int cy = 0; cy < nc; ++cy)
            for (int cx = 0; cx < nc; ++cx) {
                const int64_t I = cx + (int64_t)nc * (cy + (int64_t)nc * cz);
                double acc[27] = {0};
                const int zlo = dim == 3 ? -1 : 0, zhi = dim == 3 ? 1 : 0;
                for (int az = zlo; az <= zhi; ++az) {
                    const int fz = dim == 3 ? 2 * cz + 1 + az : 0;
                    if (dim == 3 && fz >= nf) continue;
                    const double wz = az ? 0.5 : 1.0;
                    for (int ay = -1; ay <= 1; ++ay) {
                        const int fy = 2 * cy + 1 + ay;
                        if (fy >= nf) continue;
                        const double wy = ay ? 0.5 : 1.0;
                        for (int ax = -1; ax <= 1; ++ax) {
                            const int fx = 2 * cx + 1 + ax;
                            if (fx >= nf) continue;
                            const double wi = (ax ? 0.5 : 1.0) * wy * wz;
                            const int64_t fidx = fx + (int64_t)nf * (fy + (int64_t)nf * fz);
                            int s = 0;
                            for (int oz = zlo; oz <= zhi; ++oz)
                                for (int oy = -1; oy <= 1; ++oy)
                                    for (int ox = -1; ox <= 1; ++ox, ++s) {
                                        const double a = F.coef[(size_t)s * F.N + fidx];
                                        if (a == 0.0) continue;
                                        const int jx = fx + ox, jy = fy + oy, jz = fz + oz;
                                        if (jx < 0 || jx >= nf || jy < 0 || jy >= nf) continue;
                                        if (dim == 3 && (jz < 0 || jz >= nf)) continue;
                                        int Jx[2], Jy[2], Jz[2] = {0, 0};
                                        double wx_[2], wy_[2], wz_[2] = {1.0, 1.0};
                                        const int nx_ = par(jx, Jx, wx_), ny_ = par(jy, Jy, wy_);
                                        const int nz_ = dim == 3 ? par(jz, Jz, wz_) : 1;
                                        for (int c3 = 0; c3 < nz_; ++c3)
                                            for (int c2 = 0; c2 < ny_; ++c2)
                                                for (int c1 = 0; c1 < nx_; ++c1) {
                                                    const int dx = Jx[c1] - cx, dy = Jy[c2] - cy;
                                                    const int dz = dim == 3 ? Jz[c3] - cz : 0;
                                                    const int so = dim == 2 ? (dy + 1) * 3 + (dx + 1)
                                                                            : (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
                                                    acc[so] += wi * a * (wx_[c1] * wy_[c2] * wz_[c3]);
                                                }
                                    }
                        }
                    }
                }
                for (int s = 0; s < S; ++s) C.coef[(size_t)s * C.N + I] = rscale * acc[s];
            }
    });
    // symmetrise: entries below the diagonal (s < centre) mirror the upper ones
    const int ctr = C.center();
    std::vector<double> sym(C.coef);
    for (int cz = 0; cz < nzc; ++cz)
        for (int cy = 0; cy < nc; ++cy)
            for (int cx = 0; cx < nc; ++cx) {
                const int64_t I = cx + (int64_t)nc * (cy + (int64_t)nc * cz);
                int s = 0;
                const int zlo = dim == 3 ? -1 : 0, zhi = dim == 3 ? 1 : 0;
                for (int oz = zlo; oz <= zhi; ++oz)
                    for (int oy = -1; oy <= 1; ++oy)
                        for (int ox = -1; ox <= 1; ++ox, ++s) {
                            if (s >= ctr) continue;
                            const int jx = cx + ox, jy = cy + oy, jz = cz + oz;
                            const bool in = jx >= 0 && jx < nc && jy >= 0 && jy < nc &&
                                            (dim == 2 || (jz >= 0 && jz < nc));
                            double v = 0.0;
                            if (in) {
                                const int64_t Jn = jx + (int64_t)nc * (jy + (int64_t)nc * (dim == 3 ? jz : 0));
                                v = C.coef[(size_t)(S - 1 - s) * C.N + Jn];
                            }
                            sym[(size_t)s * C.N + I] = v;
                        }
            }
    // neighbours outside the grid carry no coefficient
    for (int cz = 0; cz < nzc; ++cz)
        for (int cy = 0; cy < nc; ++cy)
            for (int cx = 0; cx < nc; ++cx) {
                const int64_t I = cx + (int64_t)nc * (cy + (int64_t)nc * cz);
                int s = 0;
                const int zlo = dim == 3 ? -1 : 0, zhi = dim == 3 ? 1 : 0;
                for (int oz = zlo; oz <= zhi; ++oz)
                    for (int oy = -1; oy <= 1; ++oy)
                        for (int ox = -1; ox <= 1; ++ox, ++s) {
                            const int jx = cx + ox, jy = cy + oy, jz = cz + oz;
                            const bool in = jx >= 0 && jx < nc && jy >= 0 && jy < nc &&
                                            (dim == 2 || (jz >= 0 && jz < nc));
                            if (!in) sym[(size_t)s * C.N + I] = 0.0;
                        }
            }
    C.coef.swap(sym);
    return C;
}

}  // namespace host
}  // namespace amg
