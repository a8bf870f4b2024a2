// Host side of the DDC handle: COO validation, the two orientations
// (counting sort by row, stable, multi-threaded), duplicate merging, row order
// (tiles of a row grid, or first column), block rows, row padding and entry
// interleaving, work units, the panel layout (column lists with 16-bit local
// indices, parts), 16-bit quantisation, and the upload into the caller's
// device workspace.
//
// The paper converts each angle-group sub-matrix D_m to CSR of D_m^T at
// initialisation (Sec. 2.2.2); here one GPU holds all of D, so both
// orientations of the whole matrix are built once from the host COO.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdlib>
#include <cstring>
#include <new>
#include <numeric>
#include <thread>

#include "common.hpp"

namespace dvmat {

static thread_local std::string g_last_error = "";

dvmat_status set_error(dvmat_status code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

dvmat_status check_hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return DVMAT_OK;
    return set_error(DVMAT_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

// Build phase timing on stderr when DVMAT_BUILD_VERBOSE is set.
static void phase(const char* what) {
    static const bool on = std::getenv("DVMAT_BUILD_VERBOSE") != nullptr;
    static auto t0 = std::chrono::steady_clock::now();
    if (!on) return;
    const auto t = std::chrono::steady_clock::now();
    fprintf(stderr, "[dvmat build] %-28s %8.3f s\n", what, std::chrono::duration<double>(t - t0).count());
    t0 = t;
}

static int host_threads() {
    int n = (int)std::thread::hardware_concurrency();
    if (const char* s = std::getenv("DVMAT_HOST_THREADS")) n = std::atoi(s);
    else if (const char* s2 = std::getenv("OMP_NUM_THREADS")) n = std::min(n, std::atoi(s2));
    return std::max(1, std::min(n, 64));
}

template <class F>
static void parallel_for(int64_t n, F&& f) {
    int T = host_threads();
    if (n < 1 << 16) T = 1;
    T = (int)std::min<int64_t>(T, std::max<int64_t>(1, n));
    std::vector<std::thread> th;
    for (int t = 0; t < T; ++t) {
        int64_t a = n * t / T, b = n * (t + 1) / T;
        th.emplace_back([&, a, b, t] { f(a, b, t); });
    }
    for (auto& x : th) x.join();
}


// IEEE binary16, round to nearest even (finite inputs; overflow -> inf).
static uint16_t float_to_half_bits(float f) {
    _Float16 h = (_Float16)f;
    uint16_t b;
    std::memcpy(&b, &h, 2);
    return b;
}
// bfloat16, round to nearest even (finite inputs).
static uint16_t float_to_bf16_bits(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7FFFu + lsb;
    return (uint16_t)(u >> 16);
}

// Layout options of one orientation (from dvmat_build_opts).
struct OrientOpts {
    int layout = 0;
    int row_order = 0;
    int slice_lanes = 0;     // 0: chosen from the mean row length
    int slice_entries = 4;   // entries per lane and step: 16 bytes of values
    int32_t grid[3] = {0, 0, 0};
    int32_t tile[3] = {0, 0, 0};
};

// Rows of one orientation, sorted by column with duplicates summed: row r's
// entries sit at [start[r], start[r] + len[r]) of col/val.
struct SortedRows {
    std::vector<int64_t> start;
    std::vector<int64_t> len;
    std::vector<int32_t> col;
    std::vector<float> val;
};

// Stable counting sort of COO by row key rk (per-thread histograms over
// contiguous entry chunks keep the input order inside a row), then per row:
// sort by column if needed and sum duplicate pairs.
static dvmat_status sort_rows(int64_t n_rows, int64_t nnz, const int32_t* rk, const int32_t* ck, const float* v,
                              SortedRows& out) {
    const int T = nnz >= (1 << 16) ? host_threads() : 1;
    try {
        std::vector<std::vector<int64_t>> hist(T);
        std::vector<std::thread> th;
        for (int t = 0; t < T; ++t) {
            th.emplace_back([&, t] {
                hist[t].assign(n_rows, 0);
                const int64_t a = nnz * t / T, b = nnz * (t + 1) / T;
                int64_t* h = hist[t].data();
                for (int64_t k = a; k < b; ++k) h[rk[k]]++;
            });
        }
        for (auto& x : th) x.join();
        th.clear();
        out.start.assign(n_rows + 1, 0);
        out.len.assign(n_rows, 0);
        parallel_for(n_rows, [&](int64_t a, int64_t b, int) {
            for (int64_t r = a; r < b; ++r) {
                int64_t c = 0;
                for (int t = 0; t < T; ++t) c += hist[t][r];
                out.len[r] = c;
            }
        });
        for (int64_t r = 0; r < n_rows; ++r) out.start[r + 1] = out.start[r] + out.len[r];
        parallel_for(n_rows, [&](int64_t a, int64_t b, int) {
            for (int64_t r = a; r < b; ++r) {
                int64_t pos = out.start[r];
                for (int t = 0; t < T; ++t) {
                    const int64_t c = hist[t][r];
                    hist[t][r] = pos;
                    pos += c;
                }
            }
        });
        out.col.resize(nnz);
        out.val.resize(nnz);
        for (int t = 0; t < T; ++t) {
            th.emplace_back([&, t] {
                const int64_t a = nnz * t / T, b = nnz * (t + 1) / T;
                int64_t* h = hist[t].data();
                for (int64_t k = a; k < b; ++k) {
                    const int64_t p = h[rk[k]]++;
                    out.col[p] = ck[k];
                    out.val[p] = v[k];
                }
            });
        }
        for (auto& x : th) x.join();
        hist.clear();
        hist.shrink_to_fit();
        parallel_for(n_rows, [&](int64_t a, int64_t b, int) {
            std::vector<int64_t> perm;
            std::vector<int32_t> tc;
            std::vector<float> tv;
            for (int64_t r = a; r < b; ++r) {
                const int64_t s0 = out.start[r], n = out.len[r];
                int32_t* c = out.col.data() + s0;
                float* fv = out.val.data() + s0;
                bool ok = true;
                for (int64_t k = 1; k < n; ++k)
                    if (c[k] <= c[k - 1]) { ok = false; break; }
                if (ok) continue;
                perm.resize(n);
                std::iota(perm.begin(), perm.end(), 0);
                std::stable_sort(perm.begin(), perm.end(), [&](int64_t x, int64_t y) { return c[x] < c[y]; });
                tc.resize(n);
                tv.resize(n);
                int64_t m = 0;
                for (int64_t k = 0; k < n; ++k) {
                    const int32_t cc = c[perm[k]];
                    const float vv = fv[perm[k]];
                    if (m > 0 && tc[m - 1] == cc) tv[m - 1] += vv;
                    else { tc[m] = cc; tv[m] = vv; ++m; }
                }
                std::copy(tc.begin(), tc.begin() + m, c);
                std::copy(tv.begin(), tv.begin() + m, fv);
                out.len[r] = m;
            }
        });
    } catch (const std::bad_alloc&) {
        return set_error(DVMAT_E_NOMEM, "host allocation failed while sorting %lld entries", (long long)nnz);
    }
    return DVMAT_OK;
}

// Block-row layout of one orientation.  B consecutive rows form a block row;
// its stored entries are the union of the rows' columns, each with B values
// (zero where a row lacks the column), so one column index and one gather of
// the vector serve B rows.  Block rows are padded with zero entries to a
// multiple of 4, and within every 256-entry chunk of a block row (the tail
// chunk: n entries) sorted entry l + q*(n/4) is stored at position 4*l + q: a
// lane's 16-byte column load then holds entries l, l+n/4, l+2n/4, l+3n/4 and
// each gather instruction of a wave covers n/4 consecutive sorted columns.
// Row order of one orientation: position p holds row perm[p] (empty: natural
// order).  Tiles of a row grid (panel layout) keep each tile's rows together
// in natural order; otherwise rows may be sorted by their first column (empty
// rows last) so rows touching the same part of the input vector run together.
// tile_of_pos: the tile of the row at each position (empty without a grid).
static dvmat_status order_rows(const SortedRows& sr, int64_t n_rows, int B, const OrientOpts& oo,
                               std::vector<int32_t>& perm, std::vector<int32_t>& tile_of_pos) {
    perm.clear();
    tile_of_pos.clear();
    const int64_t g0 = oo.grid[0], g1 = oo.grid[1], g2 = oo.grid[2];
    try {
        if (oo.layout >= 1 && (g0 | g1 | g2) != 0) {
            if (g0 < 1 || g1 < 1 || g2 < 1 || g0 * g1 * g2 != n_rows)
                return set_error(DVMAT_E_ARG, "row grid %lld x %lld x %lld does not match %lld rows", (long long)g0,
                                 (long long)g1, (long long)g2, (long long)n_rows);
            const int64_t t0 = oo.tile[0], t1 = oo.tile[1], t2 = oo.tile[2];
            if (t0 < 1 || t1 < 1 || t2 < 1 || t0 % B != 0)
                return set_error(DVMAT_E_ARG, "tile %lld x %lld x %lld: positive, first extent a multiple of %d",
                                 (long long)t0, (long long)t1, (long long)t2, B);
            const int64_t T0 = (g0 + t0 - 1) / t0, T1 = (g1 + t1 - 1) / t1, T2 = (g2 + t2 - 1) / t2;
            if (T0 * T1 * T2 >= (int64_t(1) << 31)) return set_error(DVMAT_E_ARG, "too many tiles");
            std::vector<int32_t> tile(n_rows);
            parallel_for(n_rows, [&](int64_t a, int64_t b, int) {
                for (int64_t r = a; r < b; ++r) {
                    const int64_t i = r % g0, j = (r / g0) % g1, k = r / (g0 * g1);
                    tile[r] = (int32_t)(((k / t2) * T1 + j / t1) * T0 + i / t0);
                }
            });
            perm.resize(n_rows);
            std::iota(perm.begin(), perm.end(), 0);
            std::stable_sort(perm.begin(), perm.end(), [&](int32_t a, int32_t b) { return tile[a] < tile[b]; });
            tile_of_pos.resize(n_rows);
            for (int64_t p = 0; p < n_rows; ++p) tile_of_pos[p] = tile[perm[p]];
        } else if (oo.row_order == 1) {
            perm.resize(n_rows);
            std::iota(perm.begin(), perm.end(), 0);
            auto key = [&](int32_t r) -> int64_t { return sr.len[r] > 0 ? sr.col[sr.start[r]] : INT64_MAX; };
            std::stable_sort(perm.begin(), perm.end(), [&](int32_t a, int32_t b) { return key(a) < key(b); });
        }
    } catch (const std::bad_alloc&) {
        return set_error(DVMAT_E_NOMEM, "host allocation failed while ordering %lld rows", (long long)n_rows);
    }
    return DVMAT_OK;
}

// Work units: consecutive block rows [b0, b1) up to a stored-value budget and
// kBlockRowsMax block rows; a longer block row is a unit of its own.
static void cut_units(const CsrHost& out, int64_t b0, int64_t b1, int64_t unit_cap, std::vector<int32_t>& blocks) {
    int64_t acc = 0;
    int32_t rows_in = 0;
    for (int64_t br = b0; br < b1; ++br) {
        const int64_t lp = (out.rowptr[br + 1] - out.rowptr[br]) * out.B;
        if (rows_in > 0 && (acc + lp > unit_cap || rows_in >= kBlockRowsMax)) {
            blocks.push_back((int32_t)br);
            acc = 0;
            rows_in = 0;
        }
        acc += lp;
        rows_in++;
    }
    blocks.push_back((int32_t)b1);
}

// Panels over the block rows (panel layout): a panel is a run of block rows of
// one tile whose columns number at most cap; each gets its sorted column list
// and every stored column index becomes the position in that list.  Returns
// DVMAT_E_SHAPE (no error text) when a single block row has more than cap
// columns: the caller then keeps the CSR layout.
static dvmat_status build_panels(CsrHost& out, int64_t n_cols, const std::vector<int32_t>& tile_of_pos, int64_t cap,
                                 int64_t unit_cap, int64_t part_cap, std::vector<int64_t>& pstart) {
    const int64_t n_br = out.n_brows;
    const int B = out.B;
    auto tile_of_br = [&](int64_t br) -> int64_t { return tile_of_pos.empty() ? 0 : tile_of_pos[br * B]; };
    // tiles: runs of block rows with the same tile id
    std::vector<int64_t> tstart;
    for (int64_t br = 0; br < n_br; ++br)
        if (br == 0 || tile_of_br(br) != tile_of_br(br - 1)) tstart.push_back(br);
    tstart.push_back(n_br);
    const int64_t n_tiles = (int64_t)tstart.size() - 1;
    // greedy cut of each tile (parallel over tiles).  Per thread, mark[c] holds
    // the id of the last panel that took column c and seen[c] the last block
    // row that looked at it; ids are global block row indices, so no clearing.
    std::vector<std::vector<int64_t>> cuts(n_tiles);
    std::atomic<int> too_wide(0);
    const int T = host_threads();
    std::vector<std::vector<int64_t>> marks(T), seens(T);
    parallel_for(n_tiles, [&](int64_t a, int64_t b, int t) {
        std::vector<int64_t>& mark = marks[t];
        std::vector<int64_t>& seen = seens[t];
        if (mark.empty()) {
            mark.assign(n_cols, -1);
            seen.assign(n_cols, -1);
        }
        for (int64_t ti = a; ti < b; ++ti) {
            int64_t pid = tstart[ti];         // panel id: its first block row
            int64_t count = 0;
            cuts[ti].push_back(tstart[ti]);
            for (int64_t br = tstart[ti]; br < tstart[ti + 1]; ++br) {
                const int32_t* c = out.col.data() + out.rowptr[br];
                const int64_t n = out.rowptr[br + 1] - out.rowptr[br];
                int64_t fresh = 0;                // distinct columns of this block row new to the panel
                for (int64_t k = 0; k < n; ++k)
                    if (mark[c[k]] != pid && seen[c[k]] != br) {
                        seen[c[k]] = br;
                        ++fresh;
                    }
                if (count + fresh > cap && br > pid) {
                    // close the panel before this block row; the row starts the next one
                    cuts[ti].push_back(br);
                    pid = br;
                    count = 0;
                    fresh = 0;
                    for (int64_t k = 0; k < n; ++k)
                        if (mark[c[k]] != pid) {
                            mark[c[k]] = pid;
                            ++fresh;
                        }
                } else {
                    for (int64_t k = 0; k < n; ++k) mark[c[k]] = pid;
                }
                count += fresh;
                if (count > cap) {                // a single block row wider than the budget
                    too_wide.store(1);
                    return;
                }
            }
        }
    });
    marks.clear();
    seens.clear();
    phase("panel cuts");
    if (too_wide.load()) return DVMAT_E_SHAPE;
    pstart.clear();
    for (auto& v : cuts)
        for (int64_t x : v) pstart.push_back(x);
    pstart.push_back(n_br);
    const int64_t n_pan = (int64_t)pstart.size() - 1;
    // column lists and local indices (parallel over panels)
    std::vector<std::vector<int32_t>> ul(n_pan);
    out.col16.assign(out.col.size(), 0);
    // per thread: stamp[c] = last panel that listed column c, lo[c] = its local index
    std::vector<std::vector<int64_t>> stamps(T);
    std::vector<std::vector<int32_t>> loc(T);
    parallel_for(n_pan, [&](int64_t a, int64_t b, int t) {
        std::vector<int64_t>& stamp = stamps[t];
        std::vector<int32_t>& lo = loc[t];
        if (lo.empty()) {
            lo.assign(n_cols, 0);
            stamp.assign(n_cols, -1);
        }
        for (int64_t p = a; p < b; ++p) {
            const int64_t e0 = out.rowptr[pstart[p]], e1 = out.rowptr[pstart[p + 1]];
            std::vector<int32_t>& u = ul[p];
            u.clear();
            for (int64_t k = e0; k < e1; ++k) {
                const int32_t c = out.col[k];
                if (stamp[c] != p) {
                    stamp[c] = p;
                    u.push_back(c);
                }
            }
            std::sort(u.begin(), u.end());
            for (size_t i = 0; i < u.size(); ++i) lo[u[i]] = (int32_t)i;
            for (int64_t k = e0; k < e1; ++k) out.col16[k] = (uint16_t)lo[out.col[k]];
        }
    });
    stamps.clear();
    loc.clear();
    phase("panel column lists");
    out.panel_u.assign(n_pan + 1, 0);
    out.max_panel_cols = 0;
    for (int64_t p = 0; p < n_pan; ++p) {
        out.panel_u[p + 1] = out.panel_u[p] + (int64_t)ul[p].size();
        out.max_panel_cols = std::max<int64_t>(out.max_panel_cols, (int64_t)ul[p].size());
    }
    out.ulist.resize(out.panel_u[n_pan]);
    parallel_for(n_pan, [&](int64_t a, int64_t b, int) {
        for (int64_t p = a; p < b; ++p) std::copy(ul[p].begin(), ul[p].end(), out.ulist.begin() + out.panel_u[p]);
    });
    // work units inside each panel
    out.blocks.clear();
    out.blocks.push_back(0);
    out.panel_units.assign(1, 0);
    for (int64_t p = 0; p < n_pan; ++p) {
        if (pstart[p + 1] > pstart[p]) cut_units(out, pstart[p], pstart[p + 1], unit_cap, out.blocks);
        out.panel_units.push_back((int32_t)out.blocks.size() - 1);
    }
    // parts: runs of a panel's units up to part_cap stored values (a panel
    // without units is one empty part, so every panel is visited)
    out.part_units.assign(1, 0);
    out.part_panel.clear();
    for (int64_t p = 0; p < n_pan; ++p) {
        const int32_t q0 = out.panel_units[p], q1 = out.panel_units[p + 1];
        int64_t acc = 0;
        for (int32_t q = q0; q < q1; ++q) {
            const int64_t lq = (out.rowptr[out.blocks[q + 1]] - out.rowptr[out.blocks[q]]) * out.B;
            if (q > q0 && acc + lq > part_cap) {
                out.part_units.push_back(q);
                out.part_panel.push_back((int32_t)p);
                acc = 0;
            }
            acc += lq;
        }
        out.part_units.push_back(q1);
        out.part_panel.push_back((int32_t)p);
    }
    out.layout = 1;
    phase("panel units");
    return DVMAT_OK;
}

// Sliced panels (layout 2), from the panel layout with one row per block row
// and no chunk interleave.  Each panel's rows, in their tile order, are first
// cut into parts: runs of whole lines of line_rows rows holding up to
// part_cap entries (a part is a workgroup's task, and the rows of one output
// line then share a workgroup, so its stores meet in one L2).  Inside each
// part the rows are sorted by length, longest first (stable), and cut into
// slices of C = 64 / W rows; a wave runs a slice with W lanes per row, all
// rows advancing together.  A slice of n_r rows and S steps stores, for step
// t, row i and lane w of that row, E entries (4 at FP32, 8 at 16 bits) at
// slice offset ((t*n_r + i)*W + w)*E + q, q = 0..E-1: the row's sorted entry
// EWt + qW + w, or a zero (local column 0, the row's first beamlet) past the
// row's end.  One 16-byte value load per lane and step thus streams the
// slice, and each gather instruction of a row's W lanes covers W consecutive
// sorted columns.  Rows without entries close each part in slices of up to
// 64 rows and no steps.  Afterwards rowptr holds each slice's first entry
// (int64, n_slices + 1), blocks each slice's first row position, perm the
// natural row of each position, panel_units each panel's first slice,
// part_units each part's first slice.  len_of_pos: entries of the row at
// each old position (before the panel layout's padding to a multiple of 4).
static dvmat_status build_slices(CsrHost& out, std::vector<float>& fvalb, const std::vector<int64_t>& pstart,
                                 const std::vector<int64_t>& len_of_pos, int W, int E, int64_t part_cap,
                                 int64_t line_rows) {
    const int C = kWaveSize / W;
    const int64_t n_pan = (int64_t)pstart.size() - 1;
    line_rows = std::max<int64_t>(line_rows, 1);
    // per panel: rows in slice order, the slices' row counts and steps, and
    // the first slice of each part (relative to the panel)
    std::vector<std::vector<int64_t>> order(n_pan);
    std::vector<std::vector<int32_t>> nrs(n_pan);
    std::vector<std::vector<int64_t>> steps(n_pan);
    std::vector<std::vector<int32_t>> part_first(n_pan);
    parallel_for(n_pan, [&](int64_t a, int64_t b, int) {
        for (int64_t p = a; p < b; ++p) {
            std::vector<int64_t>& o = order[p];
            o.resize(pstart[p + 1] - pstart[p]);
            std::iota(o.begin(), o.end(), pstart[p]);
            // parts: runs of whole lines up to part_cap entries (a line wider
            // than the budget is a part of its own)
            std::vector<size_t> cut{0};
            int64_t acc = 0;
            for (size_t l0 = 0; l0 < o.size(); l0 += line_rows) {
                const size_t l1 = std::min(o.size(), l0 + (size_t)line_rows);
                int64_t le = 0;
                for (size_t r = l0; r < l1; ++r) le += len_of_pos[o[r]];
                if (l0 > cut.back() && acc + le > part_cap) {
                    cut.push_back(l0);
                    acc = 0;
                }
                acc += le;
            }
            cut.push_back(o.size());
            for (size_t g = 0; g + 1 < cut.size(); ++g) {
                std::stable_sort(o.begin() + cut[g], o.begin() + cut[g + 1],
                                 [&](int64_t x, int64_t y) { return len_of_pos[x] > len_of_pos[y]; });
                part_first[p].push_back((int32_t)nrs[p].size());
                size_t i = cut[g];
                while (i < cut[g + 1]) {
                    const int64_t lmax = len_of_pos[o[i]];
                    const int cap_rows = lmax > 0 ? C : kWaveSize;
                    size_t j = i;
                    while (j < cut[g + 1] && (int64_t)(j - i) < cap_rows && (len_of_pos[o[j]] > 0) == (lmax > 0)) ++j;
                    nrs[p].push_back((int32_t)(j - i));
                    steps[p].push_back(((lmax + E - 1) / E + W - 1) / W);
                    i = j;
                }
            }
        }
    });
    // slice offsets
    std::vector<int64_t> first_slice(n_pan + 1, 0);
    for (int64_t p = 0; p < n_pan; ++p) first_slice[p + 1] = first_slice[p] + (int64_t)nrs[p].size();
    const int64_t n_sl = first_slice[n_pan];
    if (n_sl >= (int64_t(1) << 31)) return set_error(DVMAT_E_SHAPE, "too many slices");
    std::vector<int64_t> rowptr(n_sl + 1, 0);
    std::vector<int32_t> blocks(n_sl + 1, 0);
    {
        int64_t q = 0, e = 0, pos = 0;
        for (int64_t p = 0; p < n_pan; ++p)
            for (size_t k = 0; k < nrs[p].size(); ++k, ++q) {
                rowptr[q] = e;
                blocks[q] = (int32_t)pos;
                e += steps[p][k] * nrs[p][k] * W * E;
                pos += nrs[p][k];
            }
        rowptr[n_sl] = e;
        blocks[n_sl] = (int32_t)pos;
    }
    const int64_t ne = rowptr[n_sl];
    std::vector<uint16_t> col16(ne, 0);
    std::vector<int32_t> col(ne, 0);
    std::vector<float> val(ne, 0.0f);
    std::vector<int32_t> perm(out.n_rows);
    parallel_for(n_pan, [&](int64_t a, int64_t b, int) {
        for (int64_t p = a; p < b; ++p) {
            int64_t q = first_slice[p];
            size_t r = 0;
            for (size_t k = 0; k < nrs[p].size(); ++k, ++q) {
                const int nr = nrs[p][k];
                const int64_t S = steps[p][k];
                for (int i = 0; i < nr; ++i, ++r) {
                    const int64_t op = order[p][r];
                    perm[blocks[q] + i] = out.perm.empty() ? (int32_t)op : out.perm[op];
                    const int64_t s0 = out.rowptr[op], L = len_of_pos[op];
                    const int32_t c0 = L > 0 ? out.col[s0] : 0;
                    for (int64_t t = 0; t < S; ++t)
                        for (int w = 0; w < W; ++w)
                            for (int qq = 0; qq < E; ++qq) {
                                const int64_t sidx = E * W * t + qq * W + w;
                                const int64_t dst = rowptr[q] + ((t * nr + i) * W + w) * E + qq;
                                if (sidx < L) {
                                    col16[dst] = out.col16[s0 + sidx];
                                    col[dst] = out.col[s0 + sidx];
                                    val[dst] = fvalb[s0 + sidx];
                                } else {
                                    col[dst] = c0;      // a valid beamlet for the 16-bit scale; the value is zero
                                }
                            }
                }
            }
        }
    });
    // parts as cut above (a panel without rows is one empty part)
    out.part_units.assign(1, 0);
    out.part_panel.clear();
    for (int64_t p = 0; p < n_pan; ++p) {
        for (size_t g = 1; g < part_first[p].size(); ++g) {
            out.part_units.push_back((int32_t)(first_slice[p] + part_first[p][g]));
            out.part_panel.push_back((int32_t)p);
        }
        out.part_units.push_back((int32_t)first_slice[p + 1]);
        out.part_panel.push_back((int32_t)p);
    }
    out.panel_units.assign(first_slice.begin(), first_slice.end());
    out.rowptr.swap(rowptr);
    out.blocks.swap(blocks);
    out.col16.swap(col16);
    out.col.swap(col);
    fvalb.swap(val);
    out.perm.swap(perm);
    out.perm_runs = 0;
    out.slice_lanes = W;
    out.slice_entries = E;
    out.layout = 2;
    phase("slices");
    return DVMAT_OK;
}

// Lanes per row of the sliced layout when the caller leaves it open: the W in
// {4, 8, 16} whose slices take closest to 32 steps for a row of the mean
// non-empty length (E entries per lane and step).  Measured on the MI355X:
// single-arc voxel rows (872 entries) 8 lanes at FP32 and 4 at 16 bits,
// beamlet rows (1,723) 8 at 16 bits, the two-arc workload's longer rows 16
// (autograd evaluation 6.16 ms against 7.79 with 4).
static int auto_slice_lanes(const SortedRows& sr, int E) {
    int64_t n = 0, tot = 0;
    for (int64_t x : sr.len)
        if (x > 0) { ++n; tot += x; }
    if (n == 0) return 8;
    const double mean = (double)tot / (double)n;
    int best = 4;
    double err = 1e30;
    for (int w : {4, 8, 16}) {
        const double e = std::fabs(mean / (double)(w * E) - 32.0);
        if (e < err) { err = e; best = w; }
    }
    return best;
}

static dvmat_status build_blocked(const SortedRows& sr, int64_t n_rows, int64_t n_cols, int B, bool interleave,
                                  int64_t unit_cap, const OrientOpts& oo, int64_t panel_cols, int64_t part_cap,
                                  CsrHost& out, std::vector<float>& fvalb) {
    std::vector<int32_t> tile_of_pos;
    phase("start orientation");
    dvmat_status st0 = order_rows(sr, n_rows, B, oo, out.perm, tile_of_pos);
    if (st0) return st0;
    out.perm_runs = 0;
    if (!out.perm.empty()) {
        bool runs = true;
        for (int64_t p = 0; p < n_rows && runs; ++p)
            if (p % B != 0 && out.perm[p] != out.perm[p - 1] + 1) runs = false;
        out.perm_runs = runs ? 1 : 0;
    }
    phase("row order");
    try {
        const int64_t n_br = (n_rows + B - 1) / B;
        out.n_rows = n_rows;
        out.B = B;
        out.n_brows = n_br;
        out.layout = 0;
        auto row_at = [&](int64_t pos) -> int64_t { return out.perm.empty() ? pos : out.perm[pos]; };
        std::vector<int64_t> uni(n_br, 0);
        // union size of each block row (B-way merge of sorted column lists)
        parallel_for(n_br, [&](int64_t a, int64_t b, int) {
            int64_t pos[4], end[4];
            for (int64_t br = a; br < b; ++br) {
                const int nb = (int)std::min<int64_t>(B, n_rows - br * B);
                for (int q = 0; q < nb; ++q) {
                    pos[q] = sr.start[row_at(br * B + q)];
                    end[q] = pos[q] + sr.len[row_at(br * B + q)];
                }
                int64_t u = 0;
                for (;;) {
                    int32_t cmin = INT32_MAX;
                    for (int q = 0; q < nb; ++q)
                        if (pos[q] < end[q]) cmin = std::min(cmin, sr.col[pos[q]]);
                    if (cmin == INT32_MAX) break;
                    for (int q = 0; q < nb; ++q)
                        if (pos[q] < end[q] && sr.col[pos[q]] == cmin) pos[q]++;
                    ++u;
                }
                uni[br] = u;
            }
        });
        out.rowptr.assign(n_br + 1, 0);
        for (int64_t br = 0; br < n_br; ++br) out.rowptr[br + 1] = out.rowptr[br] + (uni[br] + kRowPad - 1) / kRowPad * kRowPad;
        const int64_t ne = out.rowptr[n_br];
        out.col.assign(ne, 0);
        fvalb.assign(ne * B, 0.0f);
        parallel_for(n_br, [&](int64_t a, int64_t b, int) {
            int64_t pos[4], end[4];
            std::vector<int32_t> tc;
            std::vector<float> tv;
            for (int64_t br = a; br < b; ++br) {
                const int nb = (int)std::min<int64_t>(B, n_rows - br * B);
                for (int q = 0; q < nb; ++q) {
                    pos[q] = sr.start[row_at(br * B + q)];
                    end[q] = pos[q] + sr.len[row_at(br * B + q)];
                }
                const int64_t s0 = out.rowptr[br], e0 = out.rowptr[br + 1];
                int32_t* c = out.col.data() + s0;
                float* fv = fvalb.data() + s0 * B;
                int64_t u = 0;
                for (;;) {
                    int32_t cmin = INT32_MAX;
                    for (int q = 0; q < nb; ++q)
                        if (pos[q] < end[q]) cmin = std::min(cmin, sr.col[pos[q]]);
                    if (cmin == INT32_MAX) break;
                    c[u] = cmin;
                    for (int q = 0; q < nb; ++q)
                        if (pos[q] < end[q] && sr.col[pos[q]] == cmin) fv[u * B + q] = sr.val[pos[q]++];
                    ++u;
                }
                const int32_t last = u > 0 ? c[u - 1] : 0;
                for (int64_t k = u; k < e0 - s0; ++k) c[k] = last;      // padding: valid column, zero values
                if (!interleave || oo.layout == 2) continue;
                const int64_t len = e0 - s0;
                for (int64_t base = 0; base < len; base += 256) {
                    const int64_t n = std::min<int64_t>(256, len - base);
                    const int64_t w = n / 4;
                    tc.assign(c + base, c + base + n);
                    tv.assign(fv + base * B, fv + (base + n) * B);
                    for (int64_t l = 0; l < w; ++l)
                        for (int q = 0; q < 4; ++q) {
                            c[base + 4 * l + q] = tc[l + q * w];
                            for (int bb = 0; bb < B; ++bb) fv[(base + 4 * l + q) * B + bb] = tv[(l + q * w) * B + bb];
                        }
                }
            }
        });
        phase("block rows");
        out.blocks.clear();
        out.blocks.push_back(0);
        bool csr = oo.layout == 0;
        if (!csr) {
            std::vector<int64_t> pstart;
            const dvmat_status sp = build_panels(out, n_cols, tile_of_pos, panel_cols, unit_cap, part_cap, pstart);
            if (sp == DVMAT_E_SHAPE) csr = true;             // a block row wider than the panel budget
            else if (sp) return sp;
            if (!csr && oo.layout == 2) {
                std::vector<int64_t> len_of_pos(n_rows);
                for (int64_t p = 0; p < n_rows; ++p) len_of_pos[p] = sr.len[row_at(p)];
                const int W = oo.slice_lanes != 0 ? oo.slice_lanes : auto_slice_lanes(sr, oo.slice_entries);
                // an output line: the first extent of a tile (rows of a tile run
                // in natural order, fastest axis first)
                const int64_t line = (oo.grid[0] | oo.grid[1] | oo.grid[2]) != 0 ? oo.tile[0] : 1;
                const dvmat_status ss =
                    build_slices(out, fvalb, pstart, len_of_pos, W, oo.slice_entries, part_cap, line);
                if (ss) return ss;
            }
        }
        if (csr) {
            out.layout = 0;
            out.blocks.assign(1, 0);
            if (n_br > 0) cut_units(out, 0, n_br, unit_cap, out.blocks);
        }
        out.nonempty = 0;
        for (int64_t r = 0; r < n_rows; ++r) out.nonempty += sr.len[r] > 0;
    } catch (const std::bad_alloc&) {
        return set_error(DVMAT_E_NOMEM, "host allocation failed while building block rows (%lld rows)",
                         (long long)n_rows);
    }
    return DVMAT_OK;
}

// Store the values in the requested type.  16-bit storage keeps v / s_j with
// s_j the scale of the value's beamlet: the column for the dose orientation,
// the row for the price orientation.
// The global column indices (h.col) are still present here in both layouts;
// the panel layout drops them afterwards.
static void encode_values(CsrHost& h, const std::vector<float>& fvalb, int32_t storage,
                          const std::vector<float>& scale, bool beamlet_is_row) {
    const int64_t ne = h.rowptr.empty() ? 0 : h.rowptr.back();
    const int B = h.B;
    if (storage == DVMAT_F32) {
        h.val.resize(ne * B * 4);
        std::memcpy(h.val.data(), fvalb.data(), ne * B * 4);
        return;
    }
    h.val.resize(ne * B * 2);
    uint16_t* q = reinterpret_cast<uint16_t*>(h.val.data());
    auto enc = [&](float x) { return storage == DVMAT_F16 ? float_to_half_bits(x) : float_to_bf16_bits(x); };
    if (h.layout == 2) {
        // slices: entry k of slice u with n_r rows belongs to row (k / E / W) % n_r of the slice
        const int W = h.slice_lanes, E = h.slice_entries;
        const int64_t n_sl = (int64_t)h.blocks.size() - 1;
        parallel_for(n_sl, [&](int64_t a, int64_t b, int) {
            for (int64_t u = a; u < b; ++u) {
                const int64_t nr = h.blocks[u + 1] - h.blocks[u];
                for (int64_t k = h.rowptr[u]; k < h.rowptr[u + 1]; ++k) {
                    const int64_t i = ((k - h.rowptr[u]) / E / W) % nr;
                    const float s = scale[beamlet_is_row ? h.perm[h.blocks[u] + i] : h.col[k]];
                    q[k] = enc(fvalb[k] / s);
                }
            }
        });
        return;
    }
    parallel_for(h.n_brows, [&](int64_t a, int64_t b, int) {
        for (int64_t br = a; br < b; ++br)
            for (int64_t k = h.rowptr[br]; k < h.rowptr[br + 1]; ++k)
                for (int bb = 0; bb < B; ++bb) {
                    const int64_t pos = std::min<int64_t>(br * B + bb, h.n_rows - 1);
                    const int64_t r = h.perm.empty() ? pos : h.perm[pos];
                    const float s = scale[beamlet_is_row ? r : h.col[k]];
                    const float x = fvalb[k * B + bb] / s;
                    q[k * B + bb] = enc(x);
                }
    });
}

}  // namespace dvmat

using namespace dvmat;

extern "C" {

const char* dvmat_last_error(void) { return dvmat::g_last_error.c_str(); }

int32_t dvmat_version(void) { return 0x000100; }

dvmat_status dvmat_ddc_default_opts(int32_t storage, dvmat_build_opts* opts) {
    if (!opts) return set_error(DVMAT_E_ARG, "dvmat_ddc_default_opts: NULL argument");
    if (storage != DVMAT_F32 && storage != DVMAT_F16 && storage != DVMAT_BF16)
        return set_error(DVMAT_E_ARG, "dvmat_ddc_default_opts: unknown storage %d", storage);
    // Beamlet rows sorted by first voxel keep their gathers local (CSR).
    opts->dose_block_rows = 0;          // 0: chosen at create for the layout and storage
    opts->price_block_rows = 0;
    opts->interleave = 1;
    opts->unit_entries = 0;             // 0: 2048 for CSR, 8192 for panels
    opts->dose_row_order = 0;
    opts->price_row_order = 1;
    opts->dose_layout = 0;
    opts->price_layout = 0;
    for (int i = 0; i < 3; ++i) {
        opts->dose_grid[i] = opts->price_grid[i] = 0;
        opts->dose_tile[i] = opts->price_tile[i] = 0;
    }
    opts->panel_cols = 12288;
    opts->part_entries = 131072;
    opts->dose_slice_lanes = 0;
    opts->price_slice_lanes = 0;
    if (const char* e = std::getenv("DVMAT_PANEL_COLS")) opts->panel_cols = std::atoi(e);
    if (const char* e = std::getenv("DVMAT_PART_ENTRIES")) opts->part_entries = std::atoi(e);
    if (const char* e = std::getenv("DVMAT_DOSE_ORDER")) opts->dose_row_order = std::atoi(e);
    if (const char* e = std::getenv("DVMAT_PRICE_ORDER")) opts->price_row_order = std::atoi(e);
    if (const char* e = std::getenv("DVMAT_DOSE_B")) opts->dose_block_rows = std::atoi(e);
    if (const char* e = std::getenv("DVMAT_PRICE_B")) opts->price_block_rows = std::atoi(e);
    if (const char* e = std::getenv("DVMAT_INTERLEAVE")) opts->interleave = std::atoi(e);
    if (const char* e = std::getenv("DVMAT_BLOCK_NNZ")) opts->unit_entries = std::atoi(e);
    return DVMAT_OK;
}

dvmat_status dvmat_ddc_create(int64_t n_vox, int64_t n_bl, int64_t nnz, const int32_t* row_vox,
                              const int32_t* col_bl, const float* val, int32_t storage, dvmat_ddc* out) {
    return dvmat_ddc_create_ex(n_vox, n_bl, nnz, row_vox, col_bl, val, storage, nullptr, out);
}

dvmat_status dvmat_ddc_create_ex(int64_t n_vox, int64_t n_bl, int64_t nnz, const int32_t* row_vox,
                                 const int32_t* col_bl, const float* val, int32_t storage,
                                 const dvmat_build_opts* opts, dvmat_ddc* out) {
    if (!out) return set_error(DVMAT_E_ARG, "dvmat_ddc_create: out is NULL");
    dvmat_build_opts o;
    if (opts) {
        o = *opts;
    } else if (dvmat_status st = dvmat_ddc_default_opts(storage, &o)) {
        return st;
    }
    // Block rows left at 0: the fastest measured on the full-scale single-arc
    // workload.  CSR: with 4-byte values B = 2 stores fewer bytes per non-zero
    // than B = 4 (the union of 4 voxel rows is looser), with 2-byte values the
    // gathers B = 4 saves win.  Panels: gathers are cheap LDS reads, so the
    // smaller block rows win (dose B = 1 at 4-byte, 2 at 2-byte values).
    {
        const bool f32 = storage == DVMAT_F32;
        if (o.dose_block_rows == 0)
            o.dose_block_rows = o.dose_layout == 2 ? 1 : o.dose_layout == 1 ? (f32 ? 1 : 2) : (f32 ? 2 : 4);
        if (o.price_block_rows == 0) o.price_block_rows = o.price_layout >= 1 ? 1 : (f32 ? 1 : 2);
        // sliced panels: lanes per row left at 0 are chosen from the rows'
        // mean length when the orientation is built (auto_slice_lanes)
        // work units: on panels the gathers are cheap and each unit's start
        // (bounds, row pointers, epilogue inputs) is the cost to amortise
        if (o.unit_entries == 0) o.unit_entries = (o.dose_layout >= 1 || o.price_layout >= 1) ? 8192 : 2048;
    }
    auto okB = [](int b) { return b == 1 || b == 2 || b == 4; };
    if (!okB(o.dose_block_rows) || !okB(o.price_block_rows) || (o.interleave != 0 && o.interleave != 1) ||
        o.unit_entries < 4 || o.unit_entries > (1 << 24) || (o.dose_row_order != 0 && o.dose_row_order != 1) ||
        (o.price_row_order != 0 && o.price_row_order != 1) || o.dose_layout < 0 || o.dose_layout > 2 ||
        o.price_layout < 0 || o.price_layout > 2 || o.panel_cols < 1 || o.panel_cols > 65536 ||
        o.part_entries < 1 || (o.dose_slice_lanes != 0 && !slice_lanes_ok(o.dose_slice_lanes)) ||
        (o.price_slice_lanes != 0 && !slice_lanes_ok(o.price_slice_lanes)) ||
        (o.dose_layout == 2 && o.dose_block_rows != 1) ||
        (o.price_layout == 2 && o.price_block_rows != 1))
        return set_error(DVMAT_E_ARG,
                         "dvmat_ddc_create: bad build options (block rows %d/%d, interleave %d, unit %d, layouts %d/%d, "
                         "slice lanes %d/%d)",
                         o.dose_block_rows, o.price_block_rows, o.interleave, o.unit_entries, o.dose_layout,
                         o.price_layout, o.dose_slice_lanes, o.price_slice_lanes);
    *out = nullptr;
    if (n_vox < 1 || n_vox >= (int64_t(1) << 31) || n_bl < 1 || n_bl >= (int64_t(1) << 31))
        return set_error(DVMAT_E_ARG, "dvmat_ddc_create: n_vox=%lld n_bl=%lld must be in [1, 2^31)",
                         (long long)n_vox, (long long)n_bl);
    if (nnz < 0) return set_error(DVMAT_E_ARG, "dvmat_ddc_create: nnz=%lld < 0", (long long)nnz);
    if (nnz > 0 && (!row_vox || !col_bl || !val))
        return set_error(DVMAT_E_ARG, "dvmat_ddc_create: NULL COO array with nnz=%lld", (long long)nnz);
    if (storage != DVMAT_F32 && storage != DVMAT_F16 && storage != DVMAT_BF16)
        return set_error(DVMAT_E_ARG, "dvmat_ddc_create: unknown storage %d", storage);
    // O(nnz) validation
    std::atomic<int64_t> bad_idx(-1), bad_val(-1);
    parallel_for(nnz, [&](int64_t a, int64_t b, int) {
        for (int64_t k = a; k < b; ++k) {
            if (row_vox[k] < 0 || row_vox[k] >= n_vox || col_bl[k] < 0 || col_bl[k] >= n_bl) {
                int64_t e = -1;
                bad_idx.compare_exchange_strong(e, k);
                return;
            }
            if (!std::isfinite(val[k])) {
                int64_t e = -1;
                bad_val.compare_exchange_strong(e, k);
                return;
            }
        }
    });
    if (bad_idx.load() >= 0) {
        int64_t k = bad_idx.load();
        return set_error(DVMAT_E_INDEX, "dvmat_ddc_create: entry %lld has (row %d, col %d) outside [0,%lld)x[0,%lld)",
                         (long long)k, row_vox[k], col_bl[k], (long long)n_vox, (long long)n_bl);
    }
    if (bad_val.load() >= 0)
        return set_error(DVMAT_E_ARG, "dvmat_ddc_create: entry %lld has a non-finite value",
                         (long long)bad_val.load());

    dvmat_ddc_s* d = new (std::nothrow) dvmat_ddc_s();
    if (!d) return set_error(DVMAT_E_NOMEM, "dvmat_ddc_create: host allocation failed");
    d->n_vox = n_vox;
    d->n_bl = n_bl;
    d->storage = storage;
    d->dose_cfg = initial_kernel_cfg();
    d->price_cfg = initial_kernel_cfg();
    d->value_bytes = storage == DVMAT_F32 ? 4 : 2;
    d->opts = o;
    dvmat_status st = DVMAT_OK;
    OrientOpts dose_oo, price_oo;
    dose_oo.layout = o.dose_layout;
    dose_oo.row_order = o.dose_row_order;
    dose_oo.slice_lanes = o.dose_slice_lanes;
    dose_oo.slice_entries = storage == DVMAT_F32 ? 4 : 8;
    price_oo.layout = o.price_layout;
    price_oo.row_order = o.price_row_order;
    price_oo.slice_lanes = o.price_slice_lanes;
    price_oo.slice_entries = storage == DVMAT_F32 ? 4 : 8;
    for (int i = 0; i < 3; ++i) {
        dose_oo.grid[i] = o.dose_grid[i];
        dose_oo.tile[i] = o.dose_tile[i];
        price_oo.grid[i] = o.price_grid[i];
        price_oo.tile[i] = o.price_tile[i];
    }
    {
        // dose orientation: rows = voxels, columns = beamlets
        SortedRows sr;
        std::vector<float> fvalb;
        phase("validate");
        if ((st = sort_rows(n_vox, nnz, row_vox, col_bl, val, sr))) { delete d; return st; }
        phase("sort dose rows");
        int64_t nnz_u = 0;
        for (int64_t x : sr.len) nnz_u += x;
        d->nnz = nnz_u;
        if (storage != DVMAT_F32) {
            // per-beamlet scale s_j = max_i |D_ij| (1 for an empty beamlet)
            const int T = host_threads();
            std::vector<std::vector<float>> mx(T);
            parallel_for(n_vox, [&](int64_t a, int64_t b, int t) {
                std::vector<float>& m = mx[t];
                m.assign(n_bl, 0.0f);
                for (int64_t r = a; r < b; ++r)
                    for (int64_t k = sr.start[r]; k < sr.start[r] + sr.len[r]; ++k)
                        m[sr.col[k]] = std::max(m[sr.col[k]], std::fabs(sr.val[k]));
            });
            d->host_scale.assign(n_bl, 0.0f);
            for (auto& m : mx)
                if (!m.empty())
                    for (int64_t j = 0; j < n_bl; ++j) d->host_scale[j] = std::max(d->host_scale[j], m[j]);
            for (auto& s : d->host_scale)
                if (!(s > 0.0f)) s = 1.0f;
        }
        if ((st = build_blocked(sr, n_vox, n_bl, o.dose_block_rows, o.interleave != 0, o.unit_entries, dose_oo, o.panel_cols, o.part_entries,
                                d->host_dose, fvalb))) {
            delete d;
            return st;
        }
        std::vector<int64_t>().swap(sr.start);
        std::vector<int64_t>().swap(sr.len);
        std::vector<int32_t>().swap(sr.col);
        std::vector<float>().swap(sr.val);
        encode_values(d->host_dose, fvalb, storage, d->host_scale, false);
        phase("encode dose values");
        if (d->host_dose.layout >= 1) std::vector<int32_t>().swap(d->host_dose.col);
    }
    {
        // price orientation: rows = beamlets, columns = voxels
        SortedRows sr;
        std::vector<float> fvalb;
        if ((st = sort_rows(n_bl, nnz, col_bl, row_vox, val, sr))) { delete d; return st; }
        phase("sort price rows");
        if ((st = build_blocked(sr, n_bl, n_vox, o.price_block_rows, o.interleave != 0, o.unit_entries, price_oo, o.panel_cols, o.part_entries,
                                d->host_price, fvalb))) {
            delete d;
            return st;
        }
        std::vector<int32_t>().swap(sr.col);
        std::vector<float>().swap(sr.val);
        encode_values(d->host_price, fvalb, storage, d->host_scale, true);
        phase("encode price values");
        if (d->host_price.layout >= 1) std::vector<int32_t>().swap(d->host_price.col);
    }

    // device workspace layout
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
    const CsrHost& hd = d->host_dose;
    const CsrHost& hp = d->host_price;
    d->off_dose_rowptr = take(hd.rowptr.size() * 8);
    d->off_dose_col = take(hd.layout >= 1 ? hd.col16.size() * 2 : hd.col.size() * 4);
    d->off_dose_val = take(hd.val.size());
    d->off_dose_blocks = take(hd.blocks.size() * 4);
    d->off_dose_perm = take(hd.perm.size() * 4);
    d->off_dose_ulist = take(hd.ulist.size() * 4);
    d->off_dose_panel_u = take(hd.panel_u.size() * 8);
    d->off_dose_panel_units = take(hd.panel_units.size() * 4);
    d->off_dose_part_units = take(hd.part_units.size() * 4);
    d->off_dose_part_panel = take(hd.part_panel.size() * 4);
    d->off_price_rowptr = take(hp.rowptr.size() * 8);
    d->off_price_col = take(hp.layout >= 1 ? hp.col16.size() * 2 : hp.col.size() * 4);
    d->off_price_val = take(hp.val.size());
    d->off_price_blocks = take(hp.blocks.size() * 4);
    d->off_price_perm = take(hp.perm.size() * 4);
    d->off_price_ulist = take(hp.ulist.size() * 4);
    d->off_price_panel_u = take(hp.panel_u.size() * 8);
    d->off_price_panel_units = take(hp.panel_units.size() * 4);
    d->off_price_part_units = take(hp.part_units.size() * 4);
    d->off_price_part_panel = take(hp.part_panel.size() * 4);
    if (storage != DVMAT_F32) {
        d->off_scale = take(n_bl * 4);
        d->off_xs = take(n_bl * 4 * kMaxRhs);
    }
    d->ws_bytes = std::max<size_t>(off, kAlign);
    d->dose.n_rows = n_vox;
    d->dose.B = hd.B;
    d->dose.nnz_pad = (int64_t)(hd.layout >= 1 ? hd.col16.size() : hd.col.size()) * hd.B;
    d->dose.layout = hd.layout;
    d->dose.slice_lanes = hd.slice_lanes;
    d->dose.n_panels = hd.layout >= 1 ? (int64_t)hd.panel_u.size() - 1 : 0;
    d->dose.max_panel_cols = hd.max_panel_cols;
    d->dose.n_parts = hd.layout >= 1 ? (int64_t)hd.part_panel.size() : 0;
    d->dose_panel_cols_total = hd.ulist.size();
    d->dose.n_blocks = (int64_t)hd.blocks.size() - 1;
    d->dose.nonempty = hd.nonempty;
    d->price.n_rows = n_bl;
    d->price.B = hp.B;
    d->price.nnz_pad = (int64_t)(hp.layout >= 1 ? hp.col16.size() : hp.col.size()) * hp.B;
    d->price.layout = hp.layout;
    d->price.slice_lanes = hp.slice_lanes;
    d->price.n_panels = hp.layout >= 1 ? (int64_t)hp.panel_u.size() - 1 : 0;
    if (hd.layout >= 1) d->dose_cfg.kind = KIND_PANEL;
    if (hp.layout >= 1) d->price_cfg.kind = KIND_PANEL;
    d->price.max_panel_cols = hp.max_panel_cols;
    d->price.n_parts = hp.layout >= 1 ? (int64_t)hp.part_panel.size() : 0;
    d->price_panel_cols_total = hp.ulist.size();
    d->price.n_blocks = (int64_t)hp.blocks.size() - 1;
    d->price.nonempty = hp.nonempty;
    *out = d;
    return DVMAT_OK;
}

dvmat_status dvmat_ddc_info(dvmat_ddc d, dvmat_ddc_info_t* info) {
    if (!d || !info) return set_error(DVMAT_E_ARG, "dvmat_ddc_info: NULL argument");
    info->n_vox = d->n_vox;
    info->n_bl = d->n_bl;
    info->nnz = d->nnz;
    info->nnz_pad_dose = d->dose.nnz_pad;
    info->nnz_pad_price = d->price.nnz_pad;
    info->n_blocks_dose = d->dose.n_blocks;
    info->n_blocks_price = d->price.n_blocks;
    info->nonempty_rows_dose = d->dose.nonempty;
    info->nonempty_rows_price = d->price.nonempty;
    info->storage = d->storage;
    info->value_bytes = d->value_bytes;
    info->workspace_bytes = d->ws_bytes;
    info->dose_kernel = d->dose_cfg.kind;
    info->dose_workgroups = d->dose_cfg.workgroups;
    info->price_kernel = d->price_cfg.kind;
    info->price_workgroups = d->price_cfg.workgroups;
    info->dose_tuned_ms = d->dose_tuned_ms;
    info->price_tuned_ms = d->price_tuned_ms;
    info->dose_block_rows = d->dose.B;
    info->price_block_rows = d->price.B;
    info->dose_row_order = d->opts.dose_row_order;
    info->price_row_order = d->opts.price_row_order;
    info->dose_layout = d->dose.layout;
    info->price_layout = d->price.layout;
    info->dose_panels = d->dose.n_panels;
    info->price_panels = d->price.n_panels;
    info->dose_panel_cols = d->dose.max_panel_cols;
    info->price_panel_cols = d->price.max_panel_cols;
    info->dose_panel_cols_total = d->dose_panel_cols_total;
    info->dose_panel_parts = d->dose.n_parts;
    info->price_panel_parts = d->price.n_parts;
    info->price_panel_cols_total = d->price_panel_cols_total;
    info->dose_slice_lanes = d->dose.layout == 2 ? d->dose.slice_lanes : 0;
    info->price_slice_lanes = d->price.layout == 2 ? d->price.slice_lanes : 0;
    return DVMAT_OK;
}

dvmat_status dvmat_ddc_bind(dvmat_ddc d, void* ws, size_t bytes, dvmat_stream stream) {
    if (!d || !ws) return set_error(DVMAT_E_ARG, "dvmat_ddc_bind: NULL argument");
    if (d->bound) return set_error(DVMAT_E_STATE, "dvmat_ddc_bind: handle already bound");
    if (reinterpret_cast<uintptr_t>(ws) % kAlign)
        return set_error(DVMAT_E_ARG, "dvmat_ddc_bind: workspace not %zu-byte aligned", kAlign);
    if (bytes < d->ws_bytes)
        return set_error(DVMAT_E_NOMEM, "dvmat_ddc_bind: workspace %zu bytes < required %zu", bytes, d->ws_bytes);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char* base = static_cast<char*>(ws);
    auto up = [&](size_t off, const void* src, size_t n) -> dvmat_status {
        if (n == 0) return DVMAT_OK;
        return check_hip(hipMemcpyAsync(base + off, src, n, hipMemcpyHostToDevice, s), "dvmat_ddc_bind: copy");
    };
    const CsrHost& hd = d->host_dose;
    const CsrHost& hp = d->host_price;
    dvmat_status st = DVMAT_OK;
    if ((st = up(d->off_dose_rowptr, hd.rowptr.data(), hd.rowptr.size() * 8))) return st;
    if (hd.layout >= 1) {
        if ((st = up(d->off_dose_col, hd.col16.data(), hd.col16.size() * 2))) return st;
        if ((st = up(d->off_dose_ulist, hd.ulist.data(), hd.ulist.size() * 4))) return st;
        if ((st = up(d->off_dose_panel_u, hd.panel_u.data(), hd.panel_u.size() * 8))) return st;
        if ((st = up(d->off_dose_panel_units, hd.panel_units.data(), hd.panel_units.size() * 4))) return st;
        if ((st = up(d->off_dose_part_units, hd.part_units.data(), hd.part_units.size() * 4))) return st;
        if ((st = up(d->off_dose_part_panel, hd.part_panel.data(), hd.part_panel.size() * 4))) return st;
    } else if ((st = up(d->off_dose_col, hd.col.data(), hd.col.size() * 4))) {
        return st;
    }
    if ((st = up(d->off_dose_val, hd.val.data(), hd.val.size()))) return st;
    if ((st = up(d->off_dose_blocks, hd.blocks.data(), hd.blocks.size() * 4))) return st;
    if ((st = up(d->off_dose_perm, hd.perm.data(), hd.perm.size() * 4))) return st;
    if ((st = up(d->off_price_rowptr, hp.rowptr.data(), hp.rowptr.size() * 8))) return st;
    if (hp.layout >= 1) {
        if ((st = up(d->off_price_col, hp.col16.data(), hp.col16.size() * 2))) return st;
        if ((st = up(d->off_price_ulist, hp.ulist.data(), hp.ulist.size() * 4))) return st;
        if ((st = up(d->off_price_panel_u, hp.panel_u.data(), hp.panel_u.size() * 8))) return st;
        if ((st = up(d->off_price_panel_units, hp.panel_units.data(), hp.panel_units.size() * 4))) return st;
        if ((st = up(d->off_price_part_units, hp.part_units.data(), hp.part_units.size() * 4))) return st;
        if ((st = up(d->off_price_part_panel, hp.part_panel.data(), hp.part_panel.size() * 4))) return st;
    } else if ((st = up(d->off_price_col, hp.col.data(), hp.col.size() * 4))) {
        return st;
    }
    if ((st = up(d->off_price_val, hp.val.data(), hp.val.size()))) return st;
    if ((st = up(d->off_price_blocks, hp.blocks.data(), hp.blocks.size() * 4))) return st;
    if ((st = up(d->off_price_perm, hp.perm.data(), hp.perm.size() * 4))) return st;
    if (d->storage != DVMAT_F32)
        if ((st = up(d->off_scale, d->host_scale.data(), d->host_scale.size() * 4))) return st;
    if ((st = check_hip(hipStreamSynchronize(s), "dvmat_ddc_bind: synchronize"))) return st;
    d->dose.rowptr = reinterpret_cast<const int64_t*>(base + d->off_dose_rowptr);
    d->dose.col = hd.layout >= 1 ? nullptr : reinterpret_cast<const int32_t*>(base + d->off_dose_col);
    if (hd.layout >= 1) {
        d->dose.col16 = reinterpret_cast<const uint16_t*>(base + d->off_dose_col);
        d->dose.ulist = reinterpret_cast<const int32_t*>(base + d->off_dose_ulist);
        d->dose.panel_u = reinterpret_cast<const int64_t*>(base + d->off_dose_panel_u);
        d->dose.panel_units = reinterpret_cast<const int32_t*>(base + d->off_dose_panel_units);
        d->dose.part_units = reinterpret_cast<const int32_t*>(base + d->off_dose_part_units);
        d->dose.part_panel = reinterpret_cast<const int32_t*>(base + d->off_dose_part_panel);
    }
    d->dose.val = base + d->off_dose_val;
    d->dose.blocks = reinterpret_cast<const int32_t*>(base + d->off_dose_blocks);
    d->dose.perm = hd.perm.empty() ? nullptr : reinterpret_cast<const int32_t*>(base + d->off_dose_perm);
    d->dose.perm_runs = hd.perm_runs;
    d->price.rowptr = reinterpret_cast<const int64_t*>(base + d->off_price_rowptr);
    d->price.col = hp.layout >= 1 ? nullptr : reinterpret_cast<const int32_t*>(base + d->off_price_col);
    if (hp.layout >= 1) {
        d->price.col16 = reinterpret_cast<const uint16_t*>(base + d->off_price_col);
        d->price.ulist = reinterpret_cast<const int32_t*>(base + d->off_price_ulist);
        d->price.panel_u = reinterpret_cast<const int64_t*>(base + d->off_price_panel_u);
        d->price.panel_units = reinterpret_cast<const int32_t*>(base + d->off_price_panel_units);
        d->price.part_units = reinterpret_cast<const int32_t*>(base + d->off_price_part_units);
        d->price.part_panel = reinterpret_cast<const int32_t*>(base + d->off_price_part_panel);
    }
    d->price.val = base + d->off_price_val;
    d->price.blocks = reinterpret_cast<const int32_t*>(base + d->off_price_blocks);
    d->price.perm = hp.perm.empty() ? nullptr : reinterpret_cast<const int32_t*>(base + d->off_price_perm);
    d->price.perm_runs = hp.perm_runs;
    if (d->storage != DVMAT_F32) {
        d->scale = reinterpret_cast<const float*>(base + d->off_scale);
        d->xs = reinterpret_cast<float*>(base + d->off_xs);
    }
    // release the host staging
    d->host_dose = CsrHost();
    d->host_price = CsrHost();
    d->bound = true;
    return DVMAT_OK;
}

dvmat_status dvmat_ddc_layout_array(dvmat_ddc d, int32_t orientation, int32_t which, void* dst, size_t cap,
                                    size_t* size) {
    if (!d || !size) return set_error(DVMAT_E_ARG, "dvmat_ddc_layout_array: NULL argument");
    if (d->bound) return set_error(DVMAT_E_STATE, "dvmat_ddc_layout_array: the host layout is released at bind");
    if (orientation != 0 && orientation != 1)
        return set_error(DVMAT_E_ARG, "dvmat_ddc_layout_array: orientation %d", orientation);
    const CsrHost& h = orientation == 0 ? d->host_dose : d->host_price;
    const void* src = nullptr;
    size_t n = 0;
    switch (which) {
        case 0: src = h.rowptr.data(); n = h.rowptr.size() * 8; break;
        case 1:
            if (h.layout >= 1) { src = h.col16.data(); n = h.col16.size() * 2; }
            else { src = h.col.data(); n = h.col.size() * 4; }
            break;
        case 2: src = h.val.data(); n = h.val.size(); break;
        case 3: src = h.blocks.data(); n = h.blocks.size() * 4; break;
        case 4: src = h.perm.data(); n = h.perm.size() * 4; break;
        case 5: src = h.ulist.data(); n = h.ulist.size() * 4; break;
        case 6: src = h.panel_u.data(); n = h.panel_u.size() * 8; break;
        case 7: src = h.panel_units.data(); n = h.panel_units.size() * 4; break;
        case 8: src = h.part_units.data(); n = h.part_units.size() * 4; break;
        case 9: src = h.part_panel.data(); n = h.part_panel.size() * 4; break;
        default: return set_error(DVMAT_E_ARG, "dvmat_ddc_layout_array: which %d", which);
    }
    *size = n;
    if (!dst) return DVMAT_OK;
    if (cap < n) return set_error(DVMAT_E_ARG, "dvmat_ddc_layout_array: %zu bytes < %zu", cap, n);
    if (n) std::memcpy(dst, src, n);
    return DVMAT_OK;
}

void dvmat_ddc_destroy(dvmat_ddc d) { delete d; }

}  // extern "C"
