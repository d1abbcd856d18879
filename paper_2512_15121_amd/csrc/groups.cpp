// Grouped product form of a CSR operator (setup, host side).
//
// Rows with identical column lists are grouped (at most GROUP_ROWS rows per
// group); a block holds groups of one size g, at most 8 / g entries per
// thread of the product kernel and at most GROUP_THREADS rows, with its
// distinct columns in at most GROUP_THREADS runs of consecutive ids (staged
// in LDS by the kernel).  Blocks are ordered by their first row, so the
// XCD-contiguous block ranges of the kernel still cover contiguous parts of
// the mesh.  Values are reordered on the device into the planes of each
// block.  The form is built only where it removes at least a fifth of the
// slot stream; otherwise the operator keeps the CSR form.
#include <algorithm>
#include <numeric>

#include "kernels.h"

namespace giamg {

namespace {

constexpr int MAX_RUNS = GROUP_THREADS;   // one run descriptor per lane of a block
constexpr int RUN_LEN = 64;              // entries a wave copies with one load

int64_t max_entries(int g) { return (int64_t)GROUP_THREADS * (GROUP_CAP / GROUP_THREADS / g); }

// largest group size whose block can hold a group of m entries (0: none)
int group_cap(int64_t m) {
    for (int g = GROUP_ROWS; g >= 1; --g)
        if (m <= max_entries(g)) return g;
    return 0;
}

struct Group {
    int32_t first;              // smallest row
    int32_t g;
    int64_t m;                  // entries (the common row length)
    int32_t rows[GROUP_ROWS];   // ascending
};

// distinct columns of groups [q0, q1), sorted
void block_columns(const std::vector<Group>& groups, size_t q0, size_t q1, const std::vector<int64_t>& rp,
                   const std::vector<int32_t>& ci, std::vector<int32_t>& cols) {
    cols.clear();
    for (size_t q = q0; q < q1; ++q) {
        const int64_t s = rp[groups[q].rows[0]];
        cols.insert(cols.end(), ci.begin() + s, ci.begin() + s + groups[q].m);
    }
    std::sort(cols.begin(), cols.end());
    cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
}

// runs of consecutive ids in a sorted distinct list, each at most RUN_LEN long;
// fn(first index into cols, length)
template <typename Fn>
int64_t for_runs(const std::vector<int32_t>& cols, Fn fn) {
    int64_t nr = 0;
    size_t i = 0;
    while (i < cols.size()) {
        size_t j = i + 1;
        while (j < cols.size() && j - i < (size_t)RUN_LEN && cols[j] == cols[j - 1] + 1) ++j;
        fn(i, (int)(j - i));
        ++nr;
        i = j;
    }
    return nr;
}

}  // namespace

std::vector<std::vector<int32_t>> identical_row_classes(const std::vector<int64_t>& rp,
                                                        const std::vector<int32_t>& ci, int64_t n) {
    std::vector<uint64_t> h((size_t)n);
    parallel_for(n, 4096, [&](int64_t a, int64_t b) {
        for (int64_t r = a; r < b; ++r) {
            uint64_t x = 0x9e3779b97f4a7c15ull * (uint64_t)(rp[r + 1] - rp[r] + 1);
            for (int64_t j = rp[r]; j < rp[r + 1]; ++j) {
                x ^= (uint64_t)(uint32_t)ci[j] + 0x9e3779b97f4a7c15ull + (x << 6) + (x >> 2);
                x *= 0xbf58476d1ce4e5b9ull;
            }
            h[r] = x;
        }
    });
    std::vector<int32_t> order((size_t)n);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(),
              [&](int32_t a, int32_t b) { return h[a] != h[b] ? h[a] < h[b] : a < b; });
    auto same = [&](int32_t a, int32_t b) {
        const int64_t la = rp[a + 1] - rp[a];
        return la == rp[b + 1] - rp[b] &&
               std::equal(ci.data() + rp[a], ci.data() + rp[a] + la, ci.data() + rp[b]);
    };
    std::vector<std::vector<int32_t>> out, cls;
    for (size_t i = 0; i < order.size();) {
        size_t j = i;
        while (j < order.size() && h[order[j]] == h[order[i]]) ++j;
        cls.clear();
        for (size_t q = i; q < j; ++q) {   // rows in ascending order within equal hashes
            const int32_t r = order[q];
            bool put = false;
            for (auto& c : cls)
                if (same(c.front(), r)) {
                    c.push_back(r);
                    put = true;
                    break;
                }
            if (!put) cls.push_back({r});
        }
        for (auto& c : cls) out.push_back(std::move(c));
        i = j;
    }
    std::sort(out.begin(), out.end(), [](const std::vector<int32_t>& a, const std::vector<int32_t>& b) {
        return a.front() < b.front();
    });
    return out;
}

bool build_grouping(DevCSR& d, const std::vector<int64_t>& rp, const std::vector<int32_t>& ci,
                    hipStream_t s) {
    d.release_grouping();
    const int64_t n = d.nrows;
    if (n <= 0 || d.nnz <= 0 || (int64_t)rp.size() != n + 1 || (int64_t)ci.size() != d.nnz) return false;
    if (d.nnz >= (int64_t(1) << 31)) return false;
    for (int64_t r = 0; r < n; ++r)
        if (rp[r + 1] - rp[r] > GROUP_CAP) return false;   // long rows: CSR form

    // 1. classes of rows with identical column lists, split into groups
    std::vector<Group> groups;
    groups.reserve((size_t)n);
    int64_t entries = 0;
    for (const auto& c : identical_row_classes(rp, ci, n)) {
        const int64_t m = rp[c.front() + 1] - rp[c.front()];
        const int cap = group_cap(m);
        if (cap == 0) return false;
        for (size_t q = 0; q < c.size(); q += (size_t)cap) {   // full groups, then the rest
            Group gr{};
            gr.g = (int32_t)std::min(c.size() - q, (size_t)cap);
            gr.m = m;
            for (int k = 0; k < gr.g; ++k) gr.rows[k] = c[q + k];
            gr.first = gr.rows[0];
            groups.push_back(gr);
            entries += m;
        }
    }
    if (entries * 5 > d.nnz * 4) return false;   // saves less than a fifth of the slots

    // 2. groups of one size together, each size in row order
    std::sort(groups.begin(), groups.end(), [](const Group& a, const Group& b) {
        return a.g != b.g ? a.g > b.g : a.first < b.first;
    });

    // 3. blocks
    struct Blk {
        size_t q0, q1;
        int g;
        int64_t E;
        int R;
    };
    std::vector<Blk> blocks;
    std::vector<int32_t> cols;
    for (size_t q = 0; q < groups.size();) {
        const int g = groups[q].g;
        size_t q1 = q;
        int64_t E = 0;
        int R = 0;
        while (q1 < groups.size() && groups[q1].g == g && E + groups[q1].m <= max_entries(g) &&
               R + g <= GROUP_THREADS) {
            E += groups[q1].m;
            R += g;
            ++q1;
        }
        // q1 > q: one group always fits (group_cap); halve while the runs overflow
        for (;;) {
            block_columns(groups, q, q1, rp, ci, cols);
            if (for_runs(cols, [](size_t, int) {}) <= MAX_RUNS) break;
            if (q1 - q == 1) return false;   // one group with scattered columns: CSR form
            q1 = q + (q1 - q) / 2;
        }
        E = 0;
        for (size_t k = q; k < q1; ++k) E += groups[k].m;
        blocks.push_back({q, q1, g, E, (int)((q1 - q) * (size_t)g)});
        q = q1;
    }
    std::sort(blocks.begin(), blocks.end(),
              [&](const Blk& a, const Blk& b) { return groups[a.q0].first < groups[b.q0].first; });

    // 4. tables
    const int64_t nb = (int64_t)blocks.size();
    std::vector<GBlock> gb((size_t)nb + 1);
    std::vector<int32_t> rows_out, run_ptr((size_t)nb + 1), runs;
    std::vector<uint32_t> ggrp;
    std::vector<uint16_t> slots;
    std::vector<int64_t> src((size_t)d.nnz);
    rows_out.reserve((size_t)n);
    ggrp.reserve(groups.size());
    slots.reserve((size_t)entries);
    int64_t e0 = 0, v0 = 0;
    for (int64_t b = 0; b < nb; ++b) {
        const Blk& B = blocks[b];
        gb[b] = GBlock{e0, v0, (int32_t)rows_out.size(), (int32_t)ggrp.size(), B.g, 0};
        block_columns(groups, B.q0, B.q1, rp, ci, cols);
        if (runs.size() / 2 >= (size_t)1 << 30) return false;
        run_ptr[b] = (int32_t)(runs.size() / 2);
        for_runs(cols, [&](size_t i, int len) {
            runs.push_back(cols[i]);
            runs.push_back((int32_t)i | (len << 16));   // LDS slot of the run's first column
        });
        int64_t eb = 0;
        for (size_t q = B.q0; q < B.q1; ++q) {
            const Group& G = groups[q];
            ggrp.push_back((uint32_t)(eb << 16) | (uint32_t)G.m);
            for (int i = 0; i < G.g; ++i) rows_out.push_back(G.rows[i]);
            const int64_t s0 = rp[G.rows[0]];
            for (int64_t j = 0; j < G.m; ++j) {
                const int32_t c = ci[s0 + j];
                slots.push_back((uint16_t)(std::lower_bound(cols.begin(), cols.end(), c) - cols.begin()));
                for (int i = 0; i < G.g; ++i) src[v0 + i * B.E + eb + j] = rp[G.rows[i]] + j;
            }
            eb += G.m;
        }
        e0 += B.E;
        v0 += (int64_t)B.g * B.E;
    }
    run_ptr[nb] = (int32_t)(runs.size() / 2);
    gb[nb] = GBlock{e0, v0, (int32_t)rows_out.size(), (int32_t)ggrp.size(), 0, 0};
    GIAMG_REQUIRE(e0 == entries && v0 == d.nnz && (int64_t)rows_out.size() == n,
                  "grouped form does not cover the operator");

    // 5. upload; values reordered on the device
    d.gblk.alloc(4 * ((size_t)nb + 1));
    d.grows.alloc(rows_out.size());
    d.ggrp.alloc(ggrp.size());
    d.gslot.alloc(slots.size());
    d.grun_ptr.alloc(run_ptr.size());
    d.gruns.alloc(std::max<size_t>(runs.size(), 1));
    d.gval.alloc((size_t)d.nnz);
    DevBuf<int64_t> dsrc((size_t)d.nnz);
    GIAMG_HIP(hipMemcpyAsync(d.gblk.get(), gb.data(), gb.size() * sizeof(GBlock), hipMemcpyHostToDevice, s));
    GIAMG_HIP(hipMemcpyAsync(d.grows.get(), rows_out.data(), rows_out.size() * sizeof(int32_t),
                             hipMemcpyHostToDevice, s));
    GIAMG_HIP(hipMemcpyAsync(d.ggrp.get(), ggrp.data(), ggrp.size() * sizeof(uint32_t), hipMemcpyHostToDevice, s));
    GIAMG_HIP(hipMemcpyAsync(d.gslot.get(), slots.data(), slots.size() * sizeof(uint16_t),
                             hipMemcpyHostToDevice, s));
    GIAMG_HIP(hipMemcpyAsync(d.grun_ptr.get(), run_ptr.data(), run_ptr.size() * sizeof(int32_t),
                             hipMemcpyHostToDevice, s));
    if (!runs.empty())
        GIAMG_HIP(hipMemcpyAsync(d.gruns.get(), runs.data(), runs.size() * sizeof(int32_t),
                                 hipMemcpyHostToDevice, s));
    GIAMG_HIP(hipMemcpyAsync(dsrc.get(), src.data(), src.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
    launch_gather_values(d.nnz, dsrc.get(), d.val.get(), d.gval.get(), s);
    GIAMG_HIP(hipStreamSynchronize(s));
    d.gnblk = nb;
    d.gentries = entries;
    d.ggroups = (int64_t)ggrp.size();
    d.gnruns = (int64_t)(runs.size() / 2);
    return true;
}

void make_fp32_group_values(DevCSR& d, hipStream_t s) {
    if (d.gnblk <= 0) return;
    d.gval32.alloc((size_t)d.nnz);
    launch_convert<double, float>(d.nnz, d.gval.get(), d.gval32.get(), s);
}

}  // namespace giamg
