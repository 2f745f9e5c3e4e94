"""Host checks of the sliced layout the CSR kernels read (slices of 64 rows,
each padded to its longest row, stored column by column).

The conversion is host C++ (csrc/setup.hpp, csr_sliced); this test compiles
a small driver around it with g++ and checks, on seeded random matrices with
empty rows, ragged last slices and rectangular shapes:
  * offsets and widths follow from the row lengths;
  * every row's entries appear in CSR order, bit for bit;
  * padding has weight +0.0 and a valid column (the row's first, 0 if empty);
  * so a row product over the layout equals the CSR one bit for bit;
  * a layout that would not fit int32 offsets is refused.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2402_12833_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <vector>
#include "setup.hpp"
using namespace amg::host;

int main(int argc, char** argv) {
    Csr M;
    Sliced S;
    if (argc == 2) {                      // one row longer than int32 offsets allow
        M.n = 1; M.m = 1; M.ptr = {0, 33554432};
        std::printf("%d\n", csr_sliced(M, S) ? 1 : 0);
        return 0;
    }
    FILE* f = std::fopen(argv[1], "rb");
    std::fread(&M.n, 4, 1, f);
    std::fread(&M.m, 4, 1, f);
    M.ptr.resize(M.n + 1);
    std::fread(M.ptr.data(), 4, M.n + 1, f);
    M.col.resize(M.ptr[M.n]);
    M.val.resize(M.ptr[M.n]);
    std::fread(M.col.data(), 4, M.col.size(), f);
    std::fread(M.val.data(), 8, M.val.size(), f);
    std::fclose(f);
    int ok = csr_sliced(M, S) ? 1 : 0;
    int ns = (int)S.off.size(), tot = (int)S.col.size();
    FILE* g = std::fopen(argv[2], "wb");
    std::fwrite(&ok, 4, 1, g);
    std::fwrite(&ns, 4, 1, g);
    std::fwrite(&tot, 4, 1, g);
    std::fwrite(S.off.data(), 4, ns, g);
    std::fwrite(S.wid.data(), 4, ns, g);
    std::fwrite(S.col.data(), 4, tot, g);
    std::fwrite(S.val.data(), 8, tot, g);
    std::fclose(g);
    return 0;
}
"""

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    d = tmp_path_factory.mktemp("sliced")
    src = d / "drv.cpp"
    src.write_text(DRIVER)
    exe = d / "drv"
    subprocess.run(["g++", "-std=c++17", "-O1", "-pthread", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    return d, exe


def random_csr(rng, n, m, pempty):
    ptr = [0]
    cols, vals = [], []
    for _ in range(n):
        k = 0 if rng.random() < pempty else int(rng.integers(1, min(m, 19) + 1))
        c = np.sort(rng.choice(m, size=k, replace=False))
        cols.extend(c.tolist())
        vals.extend(rng.standard_normal(k).tolist())
        ptr.append(len(cols))
    return np.array(ptr, np.int32), np.array(cols, np.int32), np.array(vals, np.float64)


def run(driver, n, m, ptr, col, val):
    d, exe = driver
    fin, fout = d / "in.bin", d / "out.bin"
    with open(fin, "wb") as f:
        np.array([n, m], np.int32).tofile(f)
        ptr.tofile(f)
        col.tofile(f)
        val.tofile(f)
    subprocess.run([str(exe), str(fin), str(fout)], check=True)
    raw = open(fout, "rb").read()
    ok, ns, tot = np.frombuffer(raw, np.int32, 3)
    o = 12
    off = np.frombuffer(raw, np.int32, ns, o); o += 4 * ns
    wid = np.frombuffer(raw, np.int32, ns, o); o += 4 * ns
    scol = np.frombuffer(raw, np.int32, tot, o); o += 4 * tot
    sval = np.frombuffer(raw, np.float64, tot, o)
    return ok, off, wid, scol, sval


@pytest.mark.parametrize("n,m,pempty,seed", [
    (200, 77, 0.2, 1),      # rectangular, ragged last slice, empty rows
    (64, 64, 0.0, 2),       # one full slice
    (1, 5, 0.0, 3),         # a single row
    (130, 300, 0.5, 4),     # wide, many empty rows
    (0, 3, 0.0, 5),         # no rows
])
def test_sliced_layout(driver, n, m, pempty, seed):
    rng = np.random.default_rng(seed)
    ptr, col, val = random_csr(rng, n, m, pempty)
    ok, off, wid, scol, sval = run(driver, n, m, ptr, col, val)
    assert ok == 1
    ns = (n + 63) // 64
    assert len(off) == len(wid) == ns
    lens = np.diff(ptr)
    for s in range(ns):
        assert wid[s] == lens[64 * s:64 * s + 64].max()
        assert off[s] == (0 if s == 0 else off[s - 1] + 64 * wid[s - 1])
    assert len(scol) == max(1, int(64 * wid.sum()))
    assert np.all((scol >= 0) & (scol < max(m, 1)))
    x = rng.standard_normal(m)
    for r in range(n):
        s, l = divmod(r, 64)
        b, k = ptr[r], lens[r]
        e = off[s] + 64 * np.arange(wid[s]) + l
        assert np.array_equal(scol[e[:k]], col[b:b + k])
        assert np.array_equal(sval[e[:k]].view(np.int64), val[b:b + k].view(np.int64))
        pad = e[k:]
        assert np.all(sval[pad].view(np.int64) == 0)          # +0.0 exactly
        assert np.all(scol[pad] == (col[b] if k > 0 else 0))
        dense = 0.0
        for j in range(b, b + k):
            dense += val[j] * x[col[j]]
        sliced = 0.0
        for j in e:
            sliced += sval[j] * x[scol[j]]
        assert sliced == dense


def test_sliced_refuses_int32_overflow(driver):
    _, exe = driver
    out = subprocess.run([str(exe), "big"], check=True, capture_output=True, text=True).stdout
    assert out.strip() == "0"
