// Host side of the DDC handle: COO validation, the two CSR orientations
// (counting sort by row, stable, multi-threaded), duplicate merging, row
// padding, row blocks, 16-bit quantisation, and the upload into the caller's
// device workspace.
//
// The paper converts each angle-group sub-matrix D_m to CSR of D_m^T at
// initialisation (Sec. 2.2.2); here one GPU holds all of D, so both CSR(D)
// and CSR(D^T) are built once from the host COO.
#include <hip/hip_runtime.h>

#include <algorithm>
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
static dvmat_status build_blocked(const SortedRows& sr, int64_t n_rows, int B, bool interleave, int64_t unit_cap,
                                  bool order_by_first_col, CsrHost& out, std::vector<float>& fvalb) {
    try {
        const int64_t n_br = (n_rows + B - 1) / B;
        out.n_rows = n_rows;
        out.B = B;
        out.n_brows = n_br;
        // optional row order: position p holds row perm[p]; rows sorted by their
        // first column (empty rows last), so rows touching the same part of the
        // input vector are processed together
        out.perm.clear();
        if (order_by_first_col) {
            out.perm.resize(n_rows);
            std::iota(out.perm.begin(), out.perm.end(), 0);
            auto key = [&](int32_t r) -> int64_t { return sr.len[r] > 0 ? sr.col[sr.start[r]] : INT64_MAX; };
            std::stable_sort(out.perm.begin(), out.perm.end(), [&](int32_t a, int32_t b) { return key(a) < key(b); });
        }
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
                if (!interleave) continue;
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
        // work units: consecutive block rows up to a stored-value budget and
        // kBlockRowsMax block rows; a longer block row is a unit of its own
        out.blocks.clear();
        out.blocks.push_back(0);
        int64_t acc = 0;
        int32_t rows_in = 0;
        for (int64_t br = 0; br < n_br; ++br) {
            const int64_t lp = (out.rowptr[br + 1] - out.rowptr[br]) * B;
            if (rows_in > 0 && (acc + lp > unit_cap || rows_in >= kBlockRowsMax)) {
                out.blocks.push_back((int32_t)br);
                acc = 0;
                rows_in = 0;
            }
            acc += lp;
            rows_in++;
        }
        out.blocks.push_back((int32_t)n_br);
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
static void encode_values(CsrHost& h, const std::vector<float>& fvalb, int32_t storage,
                          const std::vector<float>& scale, bool beamlet_is_row) {
    const int64_t ne = (int64_t)h.col.size();
    const int B = h.B;
    if (storage == DVMAT_F32) {
        h.val.resize(ne * B * 4);
        std::memcpy(h.val.data(), fvalb.data(), ne * B * 4);
        return;
    }
    h.val.resize(ne * B * 2);
    uint16_t* q = reinterpret_cast<uint16_t*>(h.val.data());
    parallel_for(h.n_brows, [&](int64_t a, int64_t b, int) {
        for (int64_t br = a; br < b; ++br)
            for (int64_t k = h.rowptr[br]; k < h.rowptr[br + 1]; ++k)
                for (int bb = 0; bb < B; ++bb) {
                    const int64_t pos = std::min<int64_t>(br * B + bb, h.n_rows - 1);
                    const int64_t r = h.perm.empty() ? pos : h.perm[pos];
                    const float s = scale[beamlet_is_row ? r : h.col[k]];
                    const float x = fvalb[k * B + bb] / s;
                    q[k * B + bb] = storage == DVMAT_F16 ? float_to_half_bits(x) : float_to_bf16_bits(x);
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
    // Fastest measured on the full-scale single-arc workload: with 4-byte
    // values B = 2 stores fewer bytes per non-zero than B = 4 (the union of 4
    // voxel rows is looser), with 2-byte values the gathers saved by B = 4
    // win.  Beamlet rows sorted by first voxel keep their gathers local.
    const bool f32 = storage == DVMAT_F32;
    opts->dose_block_rows = f32 ? 2 : 4;
    opts->price_block_rows = f32 ? 1 : 2;
    opts->interleave = 1;
    opts->unit_entries = 2048;
    opts->dose_row_order = 0;
    opts->price_row_order = 1;
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
    auto okB = [](int b) { return b == 1 || b == 2 || b == 4; };
    if (!okB(o.dose_block_rows) || !okB(o.price_block_rows) || (o.interleave != 0 && o.interleave != 1) ||
        o.unit_entries < 4 || o.unit_entries > (1 << 24) || (o.dose_row_order != 0 && o.dose_row_order != 1) ||
        (o.price_row_order != 0 && o.price_row_order != 1))
        return set_error(DVMAT_E_ARG, "dvmat_ddc_create: bad build options (block rows %d/%d, interleave %d, unit %d)",
                         o.dose_block_rows, o.price_block_rows, o.interleave, o.unit_entries);
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
    {
        // dose orientation: rows = voxels, columns = beamlets
        SortedRows sr;
        std::vector<float> fvalb;
        if ((st = sort_rows(n_vox, nnz, row_vox, col_bl, val, sr))) { delete d; return st; }
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
        if ((st = build_blocked(sr, n_vox, o.dose_block_rows, o.interleave != 0, o.unit_entries, o.dose_row_order == 1,
                                d->host_dose, fvalb))) {
            delete d;
            return st;
        }
        std::vector<int64_t>().swap(sr.start);
        std::vector<int64_t>().swap(sr.len);
        std::vector<int32_t>().swap(sr.col);
        std::vector<float>().swap(sr.val);
        encode_values(d->host_dose, fvalb, storage, d->host_scale, false);
    }
    {
        // price orientation: rows = beamlets, columns = voxels
        SortedRows sr;
        std::vector<float> fvalb;
        if ((st = sort_rows(n_bl, nnz, col_bl, row_vox, val, sr))) { delete d; return st; }
        if ((st = build_blocked(sr, n_bl, o.price_block_rows, o.interleave != 0, o.unit_entries, o.price_row_order == 1,
                                d->host_price, fvalb))) {
            delete d;
            return st;
        }
        std::vector<int32_t>().swap(sr.col);
        std::vector<float>().swap(sr.val);
        encode_values(d->host_price, fvalb, storage, d->host_scale, true);
    }

    // device workspace layout
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
    const CsrHost& hd = d->host_dose;
    const CsrHost& hp = d->host_price;
    d->off_dose_rowptr = take(hd.rowptr.size() * 8);
    d->off_dose_col = take(hd.col.size() * 4);
    d->off_dose_val = take(hd.val.size());
    d->off_dose_blocks = take(hd.blocks.size() * 4);
    d->off_dose_perm = take(hd.perm.size() * 4);
    d->off_price_rowptr = take(hp.rowptr.size() * 8);
    d->off_price_col = take(hp.col.size() * 4);
    d->off_price_val = take(hp.val.size());
    d->off_price_blocks = take(hp.blocks.size() * 4);
    d->off_price_perm = take(hp.perm.size() * 4);
    if (storage != DVMAT_F32) {
        d->off_scale = take(n_bl * 4);
        d->off_xs = take(n_bl * 4 * kMaxRhs);
    }
    d->ws_bytes = std::max<size_t>(off, kAlign);
    d->dose.n_rows = n_vox;
    d->dose.B = hd.B;
    d->dose.nnz_pad = (int64_t)hd.col.size() * hd.B;
    d->dose.n_blocks = (int64_t)hd.blocks.size() - 1;
    d->dose.nonempty = hd.nonempty;
    d->price.n_rows = n_bl;
    d->price.B = hp.B;
    d->price.nnz_pad = (int64_t)hp.col.size() * hp.B;
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
    if ((st = up(d->off_dose_col, hd.col.data(), hd.col.size() * 4))) return st;
    if ((st = up(d->off_dose_val, hd.val.data(), hd.val.size()))) return st;
    if ((st = up(d->off_dose_blocks, hd.blocks.data(), hd.blocks.size() * 4))) return st;
    if ((st = up(d->off_dose_perm, hd.perm.data(), hd.perm.size() * 4))) return st;
    if ((st = up(d->off_price_rowptr, hp.rowptr.data(), hp.rowptr.size() * 8))) return st;
    if ((st = up(d->off_price_col, hp.col.data(), hp.col.size() * 4))) return st;
    if ((st = up(d->off_price_val, hp.val.data(), hp.val.size()))) return st;
    if ((st = up(d->off_price_blocks, hp.blocks.data(), hp.blocks.size() * 4))) return st;
    if ((st = up(d->off_price_perm, hp.perm.data(), hp.perm.size() * 4))) return st;
    if (d->storage != DVMAT_F32)
        if ((st = up(d->off_scale, d->host_scale.data(), d->host_scale.size() * 4))) return st;
    if ((st = check_hip(hipStreamSynchronize(s), "dvmat_ddc_bind: synchronize"))) return st;
    d->dose.rowptr = reinterpret_cast<const int64_t*>(base + d->off_dose_rowptr);
    d->dose.col = reinterpret_cast<const int32_t*>(base + d->off_dose_col);
    d->dose.val = base + d->off_dose_val;
    d->dose.blocks = reinterpret_cast<const int32_t*>(base + d->off_dose_blocks);
    d->dose.perm = hd.perm.empty() ? nullptr : reinterpret_cast<const int32_t*>(base + d->off_dose_perm);
    d->price.rowptr = reinterpret_cast<const int64_t*>(base + d->off_price_rowptr);
    d->price.col = reinterpret_cast<const int32_t*>(base + d->off_price_col);
    d->price.val = base + d->off_price_val;
    d->price.blocks = reinterpret_cast<const int32_t*>(base + d->off_price_blocks);
    d->price.perm = hp.perm.empty() ? nullptr : reinterpret_cast<const int32_t*>(base + d->off_price_perm);
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

void dvmat_ddc_destroy(dvmat_ddc d) { delete d; }

}  // extern "C"
