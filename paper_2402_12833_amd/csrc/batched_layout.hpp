// Layout of a batch of structured problems in the batched solver's device
// buffers, computed on the host: the order of the problems in the instance
// table (sorted by number of levels, so that each level count is one group of
// consecutive entries), every problem's offsets into the shared vector,
// direction-block, operator, carry and partial-sum arrays, and the block maps
// that assign each block of a batched launch one problem's node range.  Host
// C++ only (no device code), so that the layout can be checked on the CPU.
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <vector>

namespace amg {
namespace host {

constexpr int kBatchMaxLevels = 8;

// One block of a batched launch: nodes [start, end) of level l of the
// instance at position inst (l is implied by the map the block belongs to);
// blk numbers the blocks of one instance in that map from 0.
struct BatchBlock {
    int inst, blk, start, end;
};

// Entries [off, off + cnt) of the block map.
struct BatchRange {
    int off = 0, cnt = 0;
};

// Instances first .. first + count - 1 have nlev levels; fine: their
// finest-level blocks.
struct BatchGroup {
    int nlev, first, count;
    BatchRange fine;
};

// One problem at its position in the instance table.  Offsets count
// elements of the arrays they index.
struct BatchProblem {
    int problem;                      // index in the caller's order
    int nlev;
    int n[kBatchMaxLevels];           // nodes per axis, level 0 coarsest
    int64_t N[kBatchMaxLevels];       // nodes per level
    size_t fine_off;                  // x, r, b, cL: the caller-order concatenation
    size_t P_off;                     // P and Q: even_up(nlev) values per fine node
    size_t coef_off[kBatchMaxLevels];  // coarse level l < nlev - 1: 3^dim coefficients per node
    size_t vec_off[kBatchMaxLevels];   // g and c1 of coarse level l: one value per node
    size_t Y_off[kBatchMaxLevels];     // block carry of coarse level l: even_up(l + 1) per node
    size_t part_off;                   // part_rows rows of pcnt partial sums
    int pcnt;                          // finest-level blocks (chunk nodes each)
};

struct BatchLayout {
    std::vector<size_t> offs;         // caller order: problem i's fine nodes start at offs[i]
    std::vector<int> pos;             // problem i -> its position in the instance table
    std::vector<BatchProblem> inst;   // by position
    std::vector<BatchGroup> groups;
    size_t nP = 0, ncoef = 0, nvec = 0, nY = 0, npart = 0;
    std::vector<BatchBlock> maps;
    BatchRange all;                   // every instance's finest-level blocks
    BatchRange dep[kBatchMaxLevels];  // depth d below the finest level: that level's nodes
    BatchRange pro[kBatchMaxLevels];  // the same where that level is not the coarsest
    int dmax = 0;                     // deepest depth over all groups
};

inline int batch_even_up(int k) { return (k + 1) / 2 * 2; }

inline int64_t batch_ipow(int64_t a, int e) {
    int64_t r = 1;
    while (e-- > 0) r *= a;
    return r;
}

// The layout of problems with n[i] nodes per axis and nlev[i] levels (1 ..
// kBatchMaxLevels, coarse sizes n / 2^k, all >= 1; the caller validates),
// fine blocks of `chunk` nodes, coarse blocks of `block` nodes, part_rows
// partial-sum rows per problem.  Buffers are laid out in the caller's order,
// the instance table in level order (stable).
inline BatchLayout batch_layout(int dim, const std::vector<int>& n, const std::vector<int>& nlev, int chunk,
                                int block, int part_rows) {
    const int cnt = (int)n.size();
    const int S = dim == 2 ? 9 : 27;
    BatchLayout L;
    L.offs.assign(cnt + 1, 0);
    std::vector<int> order(cnt);
    for (int i = 0; i < cnt; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return nlev[a] < nlev[b]; });
    L.pos.resize(cnt);
    for (int q = 0; q < cnt; ++q) L.pos[order[q]] = q;
    for (int q = 0; q < cnt; ++q) {
        const int nl = nlev[order[q]];
        if (L.groups.empty() || L.groups.back().nlev != nl) L.groups.push_back(BatchGroup{nl, q, 0, {}});
        ++L.groups.back().count;
    }
    L.inst.resize(cnt);
    for (int i = 0; i < cnt; ++i) {
        BatchProblem& I = L.inst[L.pos[i]];
        I = BatchProblem{};
        I.problem = i;
        I.nlev = nlev[i];
        I.n[I.nlev - 1] = n[i];
        for (int l = I.nlev - 2; l >= 0; --l) I.n[l] = I.n[l + 1] / 2;
        for (int l = 0; l < I.nlev; ++l) I.N[l] = batch_ipow(I.n[l], dim);
        const int64_t N = I.N[I.nlev - 1];
        I.fine_off = L.offs[i];
        L.offs[i + 1] = L.offs[i] + (size_t)N;
        I.P_off = L.nP;
        L.nP += (size_t)batch_even_up(I.nlev) * (size_t)N;
        for (int l = 0; l + 1 < I.nlev; ++l) {
            I.coef_off[l] = L.ncoef;
            L.ncoef += (size_t)S * (size_t)I.N[l];
            I.vec_off[l] = L.nvec;
            L.nvec += (size_t)I.N[l];
            I.Y_off[l] = L.nY;
            L.nY += (size_t)batch_even_up(l + 1) * (size_t)I.N[l];
        }
        I.pcnt = (int)((N + chunk - 1) / chunk);
        I.part_off = L.npart;
        L.npart += (size_t)I.pcnt * (size_t)part_rows;
    }
    auto fine = [&](int q0, int q1) {
        for (int q = q0; q < q1; ++q) {
            const BatchProblem& I = L.inst[q];
            const int N = (int)I.N[I.nlev - 1];
            for (int j = 0; j < I.pcnt; ++j) L.maps.push_back(BatchBlock{q, j, j * chunk, std::min(N, (j + 1) * chunk)});
        }
    };
    L.all.off = (int)L.maps.size();
    fine(0, cnt);
    L.all.cnt = (int)L.maps.size() - L.all.off;
    for (BatchGroup& G : L.groups) {
        G.fine.off = (int)L.maps.size();
        fine(G.first, G.first + G.count);
        G.fine.cnt = (int)L.maps.size() - G.fine.off;
    }
    // per depth below the finest level, over all groups: that coarse level's
    // nodes (restriction and smoothing), and the same for the problems where
    // it is not the coarsest level (the block carry into it)
    for (const BatchGroup& G : L.groups) L.dmax = std::max(L.dmax, G.nlev - 1);
    for (int d = 1; d <= L.dmax; ++d) {
        for (int pass = 0; pass < 2; ++pass) {
            BatchRange& R = pass == 0 ? L.dep[d] : L.pro[d];
            R.off = (int)L.maps.size();
            for (const BatchGroup& G : L.groups) {
                const int l = G.nlev - 1 - d;
                if (l < 0 || (pass == 1 && l == 0)) continue;
                for (int q = G.first; q < G.first + G.count; ++q) {
                    const int Nl = (int)L.inst[q].N[l];
                    for (int j = 0, s0 = 0; s0 < Nl; ++j, s0 += block)
                        L.maps.push_back(BatchBlock{q, j, s0, std::min(Nl, s0 + block)});
                }
            }
            R.cnt = (int)L.maps.size() - R.off;
        }
    }
    return L;
}

}  // namespace host
}  // namespace amg
