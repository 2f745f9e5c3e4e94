"""The library's host setup code built with AddressSanitizer and
UndefinedBehaviorSanitizer (g++, CPU only) and run on seeded inputs:

* the structured Galerkin hierarchy (csrc/setup.hpp: fine_faces,
  faces_to_stencil, galerkin, constant_stencil9) on 2D/3D grids with
  random kappa, odd and even sizes, against the general route through CSR
  matrices (csr_multiply, csr_transpose, csr_symmetrise_upper, csr_galerkin)
  with tensor-product interpolation built independently in the driver: the
  two must give the same coarse operators to rounding;
* the sliced CSR layout (csr_sliced) on random matrices with empty rows,
  rectangular shapes and a ragged last slice: a row product over the layout
  equals the CSR one bit for bit;
* the batched layout (csrc/batched_layout.hpp) for the 512-problem workload
  table and ragged small batches: every block map entry lies inside its
  problem's level, the blocks of each range tile each problem's nodes
  exactly once and in order, the groups are the level counts in order, and
  the buffer offsets are disjoint and inside the totals.

Any out-of-bounds access, use after free or undefined behaviour aborts the
driver, and the test fails.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2402_12833_amd", "csrc")

DRIVER = r"""
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>
#include "setup.hpp"
#include "batched_layout.hpp"
using namespace amg::host;

static void fail(const char* what, long a = 0, long b = 0) {
    std::fprintf(stderr, "FAIL %s (%ld, %ld)\n", what, a, b);
    std::exit(3);
}

// deterministic pseudo-random numbers in [0, 1)
static unsigned long long g_state = 12345;
static double urand() {
    g_state = g_state * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(g_state >> 11) * (1.0 / 9007199254740992.0);
}

// A structured level as a CSR matrix (the couplings inside the grid).
static Csr stencil_csr(const StencilLevel& L) {
    Csr A;
    A.n = A.m = (int)L.N;
    A.ptr.push_back(0);
    const int n = L.n, d = L.dim;
    for (int64_t idx = 0; idx < L.N; ++idx) {
        const int i = (int)(idx % n), j = (int)((idx / n) % n), k = d == 3 ? (int)(idx / ((int64_t)n * n)) : 0;
        int s = 0;
        for (int dz = (d == 3 ? -1 : 0); dz <= (d == 3 ? 1 : 0); ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx, ++s) {
                    const int a = i + dx, b = j + dy, c = k + dz;
                    if (a < 0 || a >= n || b < 0 || b >= n || c < 0 || c >= (d == 3 ? n : 1)) continue;
                    const double v = L.coef[(size_t)s * L.N + idx];
                    if (v == 0.0) continue;
                    A.col.push_back((int)(a + (int64_t)n * (b + (int64_t)n * c)));
                    A.val.push_back(v);
                }
        A.ptr.push_back((int)A.col.size());
    }
    return A;
}

// Tensor linear interpolation from nc to nf = any size >= 2 nc nodes per
// axis: coarse node J on fine node 2J+1, a fine node between two coarse
// nodes takes 1/2 from each, boundary neighbours dropped.
static Csr interp(int dim, int nc, int nf) {
    auto w1 = [&](int f, int* J, double* w) {
        int c = 0;
        if (f % 2 == 1) { J[c] = (f - 1) / 2; w[c++] = 1.0; }
        else {
            if (f / 2 - 1 >= 0 && f / 2 - 1 < nc) { J[c] = f / 2 - 1; w[c++] = 0.5; }
            if (f / 2 < nc) { J[c] = f / 2; w[c++] = 0.5; }
        }
        return c;
    };
    Csr P;
    const int64_t Nf = ipow(nf, dim), Nc = ipow(nc, dim);
    P.n = (int)Nf;
    P.m = (int)Nc;
    P.ptr.push_back(0);
    for (int64_t idx = 0; idx < Nf; ++idx) {
        const int i = (int)(idx % nf), j = (int)((idx / nf) % nf), k = dim == 3 ? (int)(idx / ((int64_t)nf * nf)) : 0;
        int Ji[2], Jj[2], Jk[2] = {0, 0};
        double wi[2], wj[2], wk[2] = {1.0, 0.0};
        const int ci = w1(i, Ji, wi), cj = w1(j, Jj, wj), ck = dim == 3 ? w1(k, Jk, wk) : 1;
        for (int c = 0; c < ck; ++c)
            for (int b = 0; b < cj; ++b)
                for (int a = 0; a < ci; ++a) {
                    P.col.push_back((int)(Ji[a] + (int64_t)nc * (Jj[b] + (int64_t)nc * Jk[c])));
                    P.val.push_back(wi[a] * wj[b] * wk[c]);
                }
        P.ptr.push_back((int)P.col.size());
    }
    return P;
}

static double csr_max_diff(const Csr& A, const Csr& B, double* scale) {
    double dmax = 0.0, amax = 0.0;
    std::vector<double> row(A.m, 0.0);
    for (int i = 0; i < A.n; ++i) {
        for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
            row[A.col[k]] += A.val[k];
            amax = std::fmax(amax, std::fabs(A.val[k]));
        }
        for (int k = B.ptr[i]; k < B.ptr[i + 1]; ++k) row[B.col[k]] -= B.val[k];
        for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k) { dmax = std::fmax(dmax, std::fabs(row[A.col[k]])); row[A.col[k]] = 0.0; }
        for (int k = B.ptr[i]; k < B.ptr[i + 1]; ++k) { dmax = std::fmax(dmax, std::fabs(row[B.col[k]])); row[B.col[k]] = 0.0; }
    }
    *scale = amax;
    return dmax;
}

static int galerkin_cases() {
    struct Case { int dim, n, nl; bool kappa; bool st9; };
    const Case cases[] = {{2, 31, 4, false, false}, {2, 30, 3, true, false}, {2, 45, 4, true, false},
                          {3, 17, 3, true, false}, {3, 20, 3, false, false}, {3, 15, 3, true, false},
                          {2, 31, 4, false, true}, {2, 100, 4, true, false}};
    int checked = 0;
    for (const Case& c : cases) {
        std::vector<double> kap;
        if (c.kappa) {
            kap.resize((size_t)ipow(c.n + 2, c.dim));
            for (double& v : kap) v = std::exp(4.0 * (urand() - 0.5));
        }
        std::vector<StencilLevel> lev(c.nl);
        if (c.st9) {
            const double w[9] = {-0.25, -0.5, -0.25, -0.5, 3.0, -0.5, -0.25, -0.5, -0.25};
            lev[c.nl - 1] = constant_stencil9(c.n, w);
        } else {
            FineFaces f = fine_faces(c.dim, c.n, c.kappa ? kap.data() : nullptr);
            lev[c.nl - 1] = faces_to_stencil(c.dim, c.n, f);
        }
        for (int l = c.nl - 2; l >= 0; --l) lev[l] = galerkin(lev[l + 1]);
        Csr A = stencil_csr(lev[c.nl - 1]);
        for (int l = c.nl - 2; l >= 0; --l) {
            const Csr P = interp(c.dim, lev[l].n, lev[l + 1].n);
            A = csr_galerkin(A, P, std::ldexp(1.0, -c.dim));
            const Csr S = stencil_csr(lev[l]);
            double scale = 0.0;
            const double d = csr_max_diff(S, A, &scale);
            if (!(d <= 1e-12 * scale)) fail("structured and CSR Galerkin differ", c.n, l);
            if (!csr_symmetric(A, 1e-14)) fail("CSR Galerkin not symmetric", c.n, l);
            const std::vector<double> D = csr_diagonal(A);
            for (double v : D) if (!(v > 0.0)) fail("non-positive diagonal", c.n, l);
            if (lev[l].N != (int64_t)ipow(lev[l].n, c.dim)) fail("level size", c.n, l);
            ++checked;
        }
        (void)constant_with_truncation(lev[0]);
    }
    return checked;
}

static int sliced_cases() {
    int checked = 0;
    const int shapes[][2] = {{0, 5}, {1, 1}, {63, 40}, {64, 64}, {65, 30}, {200, 17}, {129, 300}};
    for (const auto& sh : shapes) {
        Csr M;
        M.n = sh[0];
        M.m = sh[1];
        M.ptr.push_back(0);
        for (int i = 0; i < M.n; ++i) {
            const int k = urand() < 0.2 ? 0 : 1 + (int)(urand() * std::min(M.m, 19));
            std::vector<int> cols;
            for (int q = 0; q < k; ++q) cols.push_back((int)(urand() * M.m));
            std::sort(cols.begin(), cols.end());
            cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
            for (int c : cols) { M.col.push_back(c); M.val.push_back(urand() - 0.5); }
            M.ptr.push_back((int)M.col.size());
        }
        Sliced S;
        if (!csr_sliced(M, S)) fail("sliced layout refused", M.n, M.m);
        std::vector<double> x(M.m > 0 ? M.m : 1);
        for (double& v : x) v = urand();
        for (int i = 0; i < M.n; ++i) {
            double a = 0.0, b = 0.0;
            for (int k = M.ptr[i]; k < M.ptr[i + 1]; ++k) a += M.val[k] * x[M.col[k]];
            const int s = i / 64, l = i % 64;
            for (int k = 0; k < S.wid[s]; ++k) {
                const size_t e = (size_t)S.off[s] + 64 * (size_t)k + l;
                if (e >= S.col.size()) fail("sliced entry out of range", i, k);
                b += S.val[e] * x[S.col[e]];
            }
            if (a != b) fail("sliced row product differs", i, 0);
        }
        ++checked;
    }
    return checked;
}

// Invariants of the batched layout; prints a summary line.
static int layout_case(const char* path, int dim, int chunk, int block, int part_rows) {
    FILE* f = std::fopen(path, "rb");
    if (!f) fail("no table");
    int cnt = 0;
    if (std::fread(&cnt, 4, 1, f) != 1) fail("table");
    std::vector<int> n(cnt), nl(cnt);
    if ((int)std::fread(n.data(), 4, cnt, f) != cnt || (int)std::fread(nl.data(), 4, cnt, f) != cnt) fail("table");
    std::fclose(f);
    const BatchLayout L = batch_layout(dim, n, nl, chunk, block, part_rows);
    // order: a stable sort by levels
    std::vector<int> seen(cnt, 0);
    for (int i = 0; i < cnt; ++i) {
        const int q = L.pos[i];
        if (q < 0 || q >= cnt || seen[q]++) fail("pos is not a permutation", i, q);
        if (L.inst[q].problem != i) fail("instance problem", q, i);
    }
    for (int q = 1; q < cnt; ++q) {
        const BatchProblem &a = L.inst[q - 1], &b = L.inst[q];
        if (a.nlev > b.nlev || (a.nlev == b.nlev && a.problem > b.problem)) fail("instance order", q, 0);
    }
    int gq = 0;
    for (const BatchGroup& G : L.groups) {
        if (G.first != gq || G.count < 1) fail("groups not contiguous", G.first, gq);
        for (int q = G.first; q < G.first + G.count; ++q)
            if (L.inst[q].nlev != G.nlev) fail("group level", q, G.nlev);
        gq += G.count;
    }
    if (gq != cnt) fail("groups do not cover", gq, cnt);
    // offsets: disjoint, inside the totals
    auto disjoint = [&](const char* what, std::vector<std::pair<size_t, size_t>> iv, size_t total) {
        std::sort(iv.begin(), iv.end());
        size_t end = 0;
        for (auto& p : iv) {
            if (p.first < end) fail(what, (long)p.first, (long)end);
            end = p.first + p.second;
        }
        if (end > total) fail(what, (long)end, (long)total);
    };
    std::vector<std::pair<size_t, size_t>> fine, P, coef, vec, Y, part;
    for (int q = 0; q < cnt; ++q) {
        const BatchProblem& I = L.inst[q];
        const int64_t N = I.N[I.nlev - 1];
        if (N != ipow(n[I.problem], dim)) fail("fine size", q, 0);
        if (L.offs[I.problem + 1] - L.offs[I.problem] != (size_t)N || I.fine_off != L.offs[I.problem]) fail("offs", q, 0);
        fine.push_back({I.fine_off, (size_t)N});
        P.push_back({I.P_off, (size_t)batch_even_up(I.nlev) * (size_t)N});
        for (int l = 0; l + 1 < I.nlev; ++l) {
            if (I.n[l] != I.n[l + 1] / 2 || I.n[l] < 1) fail("level sizes", q, l);
            coef.push_back({I.coef_off[l], (size_t)(dim == 2 ? 9 : 27) * (size_t)I.N[l]});
            vec.push_back({I.vec_off[l], (size_t)I.N[l]});
            Y.push_back({I.Y_off[l], (size_t)batch_even_up(l + 1) * (size_t)I.N[l]});
        }
        if (I.pcnt != (int)((N + chunk - 1) / chunk)) fail("pcnt", q, I.pcnt);
        part.push_back({I.part_off, (size_t)I.pcnt * part_rows});
    }
    disjoint("fine offsets", fine, L.offs[cnt]);
    disjoint("P offsets", P, L.nP);
    disjoint("coef offsets", coef, L.ncoef);
    disjoint("vector offsets", vec, L.nvec);
    disjoint("carry offsets", Y, L.nY);
    disjoint("partial offsets", part, L.npart);
    // every range tiles its instances' level nodes exactly once, in order
    auto tiles = [&](const BatchRange& R, int q0, int q1, int depth, bool carry) {
        if (R.off < 0 || R.off + R.cnt > (int)L.maps.size()) fail("range outside the map", R.off, R.cnt);
        int e = R.off;
        for (int q = q0; q < q1; ++q) {
            const BatchProblem& I = L.inst[q];
            const int l = depth < 0 ? I.nlev - 1 : I.nlev - 1 - depth;
            if (l < 0 || (carry && l == 0)) continue;
            const int Nl = (int)I.N[l];
            int next = 0, j = 0;
            while (next < Nl) {
                if (e >= R.off + R.cnt) fail("range ends early", q, next);
                const BatchBlock& B = L.maps[e++];
                if (B.inst != q || B.blk != j++ || B.start != next || B.end <= B.start || B.end > Nl)
                    fail("block map entry", q, B.start);
                if (B.end - B.start > (depth < 0 ? chunk : block)) fail("block too long", q, B.end - B.start);
                next = B.end;
            }
        }
        if (e != R.off + R.cnt) fail("range has extra entries", e, R.off + R.cnt);
    };
    tiles(L.all, 0, cnt, -1, false);
    for (const BatchGroup& G : L.groups) tiles(G.fine, G.first, G.first + G.count, -1, false);
    int dmax = 0;
    for (int q = 0; q < cnt; ++q) dmax = std::max(dmax, L.inst[q].nlev - 1);
    if (dmax != L.dmax) fail("dmax", dmax, L.dmax);
    for (int d = 1; d <= L.dmax; ++d) {
        tiles(L.dep[d], 0, cnt, d, false);
        tiles(L.pro[d], 0, cnt, d, true);
    }
    std::printf("layout %d %zu %zu %zu %zu %zu %zu %d %zu\n", cnt, L.offs[cnt], L.nP, L.ncoef, L.nY, L.npart,
                L.maps.size(), L.dmax, L.groups.size());
    return 0;
}

int main(int argc, char** argv) {
    if (argc >= 2 && std::strcmp(argv[1], "galerkin") == 0) {
        const int g = galerkin_cases();
        const int s = sliced_cases();
        std::printf("galerkin %d sliced %d\n", g, s);
        return 0;
    }
    if (argc == 7 && std::strcmp(argv[1], "layout") == 0)
        return layout_case(argv[2], std::atoi(argv[3]), std::atoi(argv[4]), std::atoi(argv[5]), std::atoi(argv[6]));
    return 2;
}
"""

SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    d = tmp_path_factory.mktemp("sanitized")
    src = d / "drv.cpp"
    src.write_text(DRIVER)
    exe = d / "drv"
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", *SAN, "-pthread", "-I", CSRC, str(src), "-o", str(exe)],
                   check=True)
    return d, exe


def run(exe, *args):
    env = dict(os.environ, ASAN_OPTIONS="abort_on_error=1:detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([str(exe), *map(str, args)], capture_output=True, text=True, env=env, timeout=600)
    assert res.returncode == 0, res.stdout + res.stderr
    return res.stdout


def test_galerkin_and_sliced_layout_under_sanitizers(driver):
    _, exe = driver
    out = run(exe, "galerkin").split()
    assert out[0] == "galerkin" and int(out[1]) == 20 and out[2] == "sliced" and int(out[3]) == 7


def write_table(path, sides, levels):
    a = np.array([len(sides), *sides, *levels], dtype=np.int32)
    a.tofile(path)


@pytest.mark.parametrize("table", ["batched2d_512", "ragged"])
def test_batched_layout_under_sanitizers(driver, table):
    d, exe = driver
    if table == "batched2d_512":
        inst = W.batched_instances()
        sides = [t.n for t in inst]
        levels = [t.nlevels for t in inst]
    else:
        # the shapes of the batched GPU parity case: sides 2..127, 1..5 levels
        sides = [31, 7, 45, 64, 100, 33, 15, 63, 2, 20, 127, 50, 31]
        levels = [W.batched_levels(n) if n >= 31 else max(1, min(3, int(np.log2(n + 1)) - 1)) for n in sides]
        levels[-1] = 1
    path = d / f"{table}.bin"
    write_table(path, sides, levels)
    # the solver's constants: 1024-node fine blocks, 256-node coarse blocks,
    # 6 partial-sum rows per problem
    out = run(exe, "layout", path, 2, 1024, 256, 6).split()
    assert out[0] == "layout"
    cnt, total, nP, ncoef, nY, npart, nmaps, dmax, ngroups = map(int, out[1:])
    # the same totals computed here from the table
    ev = lambda k: (k + 1) // 2 * 2  # noqa: E731
    assert cnt == len(sides) and total == sum(n * n for n in sides)
    assert nP == sum(ev(l) * n * n for n, l in zip(sides, levels))
    coarse = [[(n >> (l - 1 - q)) ** 2 for q in range(l - 1)] for n, l in zip(sides, levels)]
    assert ncoef == 9 * sum(sum(c) for c in coarse)
    assert nY == sum(sum(ev(q + 1) * c[q] for q in range(len(c))) for c in coarse)
    pc = [(n * n + 1023) // 1024 for n in sides]
    assert npart == 6 * sum(pc)
    assert dmax == max(levels) - 1 and ngroups == len(set(levels))
    if table == "batched2d_512":
        assert total == 13108367
