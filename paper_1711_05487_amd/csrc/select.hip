// Plans and variant selection: realizing a set of optimizations as a concrete
// kernel plan (with its preprocessing), feature extraction (Sec. III-D), the
// profile-guided classifier with its micro-benchmarks and bounds (Sec. III-B,
// III-C), the class-to-optimization map (Sec. III-E, Table II), a small
// autotuner, and the exhaustive sweep over the 16-entry catalogue (the
// trivial optimizers of Sec. IV-D).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "internal.h"

namespace csr {

namespace {

using Clock = std::chrono::steady_clock;
double ms_since(Clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
}

constexpr double kCacheBytes = 256.0 * 1024 * 1024;  // MI355X Infinity Cache

struct DeviceBandwidth {
    double hbm = 0, cache = 0;
};

}  // namespace

// Catalogue of optimization sets: the baseline, the 5 singles and the 10
// pairs, the sets the trivial optimizers of Sec. IV-D sweep.
const int32_t kCatalogue[16] = {0,     1,     2,     4,     8,     16,    1 | 2, 1 | 4,
                                1 | 8, 1 | 16, 2 | 4, 2 | 8, 2 | 16, 4 | 8, 4 | 16, 8 | 16};

int catalogue_id(int32_t opts) {
    for (int k = 0; k < 16; ++k)
        if (kCatalogue[k] == opts) return k;
    return -1;
}

double plan_bytes(const csr_matrix_s *A, const Plan &P) {
    const double vb = (double)storage_bytes(A->storage);
    const double xb = A->storage == CSR_VAL_F64 ? 8.0 : 4.0;
    const double ib = P.idx == IDX_D16                                        ? 2.0
                      : (P.idx == IDX_D8 || P.idx == IDX_W8 || P.idx == IDX_R8 ||
                         P.idx == IDX_W9)
                          ? 1.0
                          : 4.0;
    double b = (double)A->nnz * (vb + ib) + 4.0 * (A->n_rows + 1) + xb * A->n_cols +
               xb * A->n_rows;
    if (P.opts & CSR_OPT_MERGE) {
        // tile table, carries written and read back by the fixup pass (none
        // on row-aligned tiles), and the tile bases of the merge codes
        const double T = (double)A->n_tiles;
        const double ab = A->storage == CSR_VAL_F64 ? 8.0 : 4.0;
        b += 2.0 * 4.0 * (T + 1) + (A->tiles_fixup ? 2.0 * ab * T : 0.0);
        if (P.idx != IDX_I32 && P.idx != IDX_R8) b += 4.0 * T;
        // window codes: the dictionaries (window entries read) and lengths;
        // run windows: one record per tile
        if (P.idx == IDX_W8) b += 2.0 * (double)A->wdict_entries + 4.0 * T;
        if (P.idx == IDX_W9) b += 2.0 * (double)A->wdict_entries + 4.0 * kWideWords * T;
        if (P.idx == IDX_R8) b += 4.0 * kRunWords * T;
        if (P.cblocks > 0) {
            // column blocks: every pass reads its row pointers and tile table
            // and writes y (the later ones read it back); the single pass's
            // row pointers and tile table are not read
            const double B = (double)P.cblocks;
            const double xb2 = A->storage == CSR_VAL_F64 ? 8.0 : 4.0;
            b -= 4.0 * (A->n_rows + 1) + 2.0 * 4.0 * (T + 1);
            b += 4.0 * (A->n_rows + 1) * B + 8.0 * (double)A->cb_tile_off[P.cblocks] +
                 xb2 * A->n_rows * (2.0 * B - 2.0);
            if (A->tiles_fixup)  // every pass's carries, not the single pass's
                b += 2.0 * ab * ((double)A->cb_tile_off[P.cblocks] - B - T);
            if (A->cb_split) {
                // passes after the first: row pointers, row list and y of
                // their rows only
                b -= 4.0 * (A->n_rows + 1) * (B - 1.0) + xb2 * A->n_rows * (2.0 * B - 2.0);
                for (int q = 1; q < P.cblocks; ++q)
                    b += 4.0 * (2.0 * (double)A->cb_rows[q] + 1.0) + 2.0 * xb2 * (double)A->cb_rows[q];
            }
        }
    }
    if (P.long_rows && A->n_long > 0) {
        const double ab = A->storage == CSR_VAL_F64 ? 8.0 : 4.0;
        b += 8.0 * A->n_long_chunks + 4.0 * (2.0 * A->n_long + 1) + 2.0 * ab * A->n_long_chunks;
    }
    return b;
}

void fill_info(const csr_matrix_s *A, const Plan &P, csr_plan_info_t *info) {
    info->opts = P.opts;
    info->lanes_per_row = P.G;
    info->merge_items = P.L;
    info->merge_slack = (P.opts & CSR_OPT_MERGE) ? (int32_t)A->tiles_slack : 0;
    info->delta_bits = P.idx == IDX_D16                                        ? 16
                       : (P.idx == IDX_D8 || P.idx == IDX_W8 || P.idx == IDX_R8) ? 8
                       : P.idx == IDX_W9                                           ? 9
                                                                                 : 32;
    info->window_codes = P.idx == IDX_W8 ? 1 : P.idx == IDX_R8 ? 2 : P.idx == IDX_W9 ? 3 : 0;
    info->column_blocks = P.cblocks;
    info->dynamic_rows = P.dyn;
    info->jit = P.jit;
    info->n_long_rows = P.long_rows ? A->n_long : 0;
    info->variant_id = catalogue_id(P.opts);
    info->format_bytes = plan_bytes(A, P);
}

// --------------------------------------------------------------------------
// Preprocessing of the individual remedies
// --------------------------------------------------------------------------
namespace {

csr_status_t build_delta(csr_matrix_s *A, hipStream_t s) {
    if (A->code_bits != 32) return CSR_OK;  // built already, or known ineligible (0)
    if (!A->rows_sorted) {
        A->code_bits = 0;
        return CSR_OK;
    }
    for (int bits : {8, 16}) {
        DevBuf flags, codes;
        csr_status_t st;
        // a failed step leaves code_bits at 32 (not built), so a later
        // call tries again
        if ((st = flags.alloc(sizeof(int32_t))) != CSR_OK) return st;
        if ((st = codes.alloc((size_t)A->nnz * (bits / 8) + kPadBytes)) != CSR_OK) return st;
        CSR_HIP(hipMemsetAsync(flags.p, 0, sizeof(int32_t), s));
        CSR_HIP(launch_delta_encode(A->rp.as<int32_t>(), A->col.as<int32_t>(), A->n_rows, bits,
                                    codes.p, flags.as<int32_t>(), s));
        int32_t h = 0;
        CSR_HIP(hipMemcpyAsync(&h, flags.p, sizeof(h), hipMemcpyDeviceToHost, s));
        CSR_HIP(hipStreamSynchronize(s));
        if (h == 0) {
            std::swap(A->codes.p, codes.p);
            std::swap(A->codes.bytes, codes.bytes);
            A->code_bits = bits;
            return CSR_OK;
        }
    }
    A->code_bits = 0;
    return CSR_OK;
}

csr_status_t build_tiles(csr_matrix_s *A, int L, hipStream_t s) {
    if (A->tiles_L == L) return CSR_OK;
    const int64_t slack = merge_slack(A, L);
    const int64_t T = merge_tile_count(A, L);
    // until the new table is complete, no table (and nothing built on one)
    // is valid
    A->tiles_L = 0;
    A->n_tiles = 0;
    A->mcodes_L = 0;
    A->wcodes_L = 0;
    A->wcode_state = 0;
    A->wruns_L = 0;
    A->wruns_state = 0;
    csr_status_t st;
    if ((st = A->tile_i.alloc(sizeof(int32_t) * (T + 1))) != CSR_OK) return st;
    if ((st = A->tile_j.alloc(sizeof(int32_t) * (T + 1))) != CSR_OK) return st;
    if ((st = A->carry.alloc((A->storage == CSR_VAL_F64 ? 8 : 4) * (size_t)(T + 1))) != CSR_OK)
        return st;
    CSR_HIP(launch_merge_partition(A->rp.as<int32_t>(), A->n_rows, A->nnz, L, slack, T,
                                   A->tile_i.as<int32_t>(), A->tile_j.as<int32_t>(), s));
    A->n_tiles = T;
    A->tiles_L = L;
    A->tiles_slack = slack;
    A->tiles_fixup = slack == 0;  // row-aligned tiles leave nothing to fix up
    return CSR_OK;
}

// Merge codes (MB remedy on the merge path, Table II): the narrowest width
// (8, else 16 bits) that holds every tile's column range; 32 = not eligible.
// The tile bases and the width come first; the codes themselves only when
// `encode` (window codes need the bases and the width check, not the codes).
csr_status_t build_merge_codes(csr_matrix_s *A, hipStream_t s, bool encode = true) {
    if (A->mcodes_L == A->tiles_L && A->mcode_bits != 0) {
        if (!encode || A->mcodes_encoded || A->mcode_bits == 32) return CSR_OK;
        csr_status_t st;
        const int bits = A->mcode_bits;
        if ((st = A->mcodes.alloc((size_t)A->nnz * (bits / 8) + kPadBytes)) != CSR_OK) return st;
        CSR_HIP(hipMemsetAsync(A->mcodes.as<char>() + (size_t)A->nnz * (bits / 8), 0, kPadBytes,
                               s));
        CSR_HIP(launch_merge_encode(A->col.as<int32_t>(), A->tile_j.as<int32_t>(), A->n_tiles,
                                    A->tile_base.as<int32_t>(), bits, A->mcodes.p, s));
        CSR_HIP(hipStreamSynchronize(s));
        A->mcodes_encoded = 1;
        return CSR_OK;
    }
    const int64_t T = A->n_tiles;
    A->mcodes_L = 0;  // not valid until the end
    A->mcode_bits = 0;
    A->mcodes_encoded = 0;
    csr_status_t st;
    if ((st = A->tile_base.alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(T, 1))) != CSR_OK)
        return st;
    DevBuf range;
    if ((st = range.alloc(sizeof(int32_t))) != CSR_OK) return st;
    CSR_HIP(hipMemsetAsync(range.p, 0, sizeof(int32_t), s));
    CSR_HIP(launch_merge_tile_range(A->col.as<int32_t>(), A->tile_j.as<int32_t>(), T,
                                    A->tile_base.as<int32_t>(), range.as<int32_t>(), s));
    int32_t r = 0;
    CSR_HIP(hipMemcpyAsync(&r, range.p, sizeof(r), hipMemcpyDeviceToHost, s));
    CSR_HIP(hipStreamSynchronize(s));
    const int bits = r < (1 << 8) ? 8 : r < (1 << 16) ? 16 : 32;
    if (bits != 32 && encode) {
        if ((st = A->mcodes.alloc((size_t)A->nnz * (bits / 8) + kPadBytes)) != CSR_OK) return st;
        CSR_HIP(hipMemsetAsync(A->mcodes.as<char>() + (size_t)A->nnz * (bits / 8), 0, kPadBytes,
                               s));
        CSR_HIP(launch_merge_encode(A->col.as<int32_t>(), A->tile_j.as<int32_t>(), T,
                                    A->tile_base.as<int32_t>(), bits, A->mcodes.p, s));
        CSR_HIP(hipStreamSynchronize(s));
        A->mcodes_encoded = 1;
    }
    A->mcode_bits = bits;
    A->mcodes_L = A->tiles_L;
    return CSR_OK;
}

// Window codes (MB and ML remedies on row-aligned merge tiles): needs the
// tile bases and every tile's column range below 2^16 (the merge codes'
// check), then every tile's window within kWindowMax entries.
csr_status_t build_window_codes(csr_matrix_s *A, hipStream_t s) {
    if (A->wcodes_L == A->tiles_L && A->wcode_state != 0) return CSR_OK;
    csr_status_t st;
    if ((st = build_merge_codes(A, s, false)) != CSR_OK) return st;
    A->wcodes_L = 0;  // not valid until the end
    A->wcode_state = 0;
    A->wcode_wide = 0;
    if (A->tiles_slack <= 0 || A->mcode_bits > 16) {
        A->wcodes_L = A->tiles_L;
        A->wcode_state = -1;
        return CSR_OK;
    }
    // tiles of 1,024 items: 9-bit ranks (windows of up to 512 entries)
    const bool wide = A->tiles_L == 16 * kMergeBlock;
    const int wmax = wide ? kWideWindowMax : kWindowMax;
    const int wrec = wide ? kWideWords : 1;
    const int64_t T = A->n_tiles;
    if ((st = A->wdict.alloc(sizeof(uint16_t) * wmax * (size_t)std::max<int64_t>(T, 1))) != CSR_OK)
        return st;
    if ((st = A->wlen.alloc(sizeof(int32_t) * wrec * (size_t)std::max<int64_t>(T, 1))) != CSR_OK)
        return st;
    if ((st = A->wcodes.alloc((size_t)A->nnz + kPadBytes)) != CSR_OK) return st;
    CSR_HIP(hipMemsetAsync(A->wcodes.as<char>() + A->nnz, 0, kPadBytes, s));
    DevBuf most;
    if ((st = most.alloc(sizeof(int32_t))) != CSR_OK) return st;
    CSR_HIP(hipMemsetAsync(most.p, 0, sizeof(int32_t), s));
    const int vec = A->storage == CSR_VAL_F64 ? 2 : 4;  // the merge kernel's elements per load
    CSR_HIP(launch_window_encode(A->col.as<int32_t>(), A->tile_j.as<int32_t>(),
                                 A->tile_base.as<int32_t>(), T, A->wdict.as<uint16_t>(),
                                 A->wlen.as<int32_t>(), A->wcodes.as<uint8_t>(),
                                 most.as<int32_t>(), s, wide ? vec : 0));
    int32_t m = 0;
    CSR_HIP(hipMemcpyAsync(&m, most.p, sizeof(m), hipMemcpyDeviceToHost, s));
    CSR_HIP(hipStreamSynchronize(s));
    if (m > wmax) {
        A->wcodes_L = A->tiles_L;
        A->wcode_state = -1;
        return CSR_OK;
    }
    std::vector<int32_t> wl((size_t)T * wrec);
    if (T > 0)
        CSR_HIP(hipMemcpyAsync(wl.data(), A->wlen.p, sizeof(int32_t) * wl.size(),
                               hipMemcpyDeviceToHost, s));
    CSR_HIP(hipStreamSynchronize(s));
    int64_t sum = 0;
    for (int64_t t = 0; t < T; ++t) sum += wl[(size_t)t * wrec];
    A->wdict_entries = sum;
    A->wcodes_L = A->tiles_L;
    A->wcode_wide = wide ? 1 : 0;
    A->wcode_state = 1;
    return CSR_OK;
}

// Run windows (IDX_R8): the window codes' dictionaries cut into runs of
// consecutive columns, one record per tile; eligible when no tile has more
// than kRunsMax runs (the codes are the window codes' ranks).
csr_status_t build_window_runs(csr_matrix_s *A, hipStream_t s) {
    if (A->wruns_L == A->tiles_L && A->wruns_state != 0) return CSR_OK;
    csr_status_t st;
    if ((st = build_window_codes(A, s)) != CSR_OK) return st;
    A->wruns_L = 0;  // not valid until the end
    A->wruns_state = 0;
    if (A->wcode_state != 1 || A->wcode_wide) {  // run records hold 8-bit ranks only
        A->wruns_L = A->tiles_L;
        A->wruns_state = -1;
        return CSR_OK;
    }
    const int64_t T = A->n_tiles;
    if ((st = A->wruns.alloc(sizeof(int32_t) * kRunWords * (size_t)std::max<int64_t>(T, 1))) !=
        CSR_OK)
        return st;
    DevBuf most;
    if ((st = most.alloc(sizeof(int32_t))) != CSR_OK) return st;
    CSR_HIP(hipMemsetAsync(most.p, 0, sizeof(int32_t), s));
    CSR_HIP(launch_window_runs(A->wdict.as<uint16_t>(), A->wlen.as<int32_t>(),
                               A->tile_base.as<int32_t>(), T, A->wruns.as<int32_t>(),
                               most.as<int32_t>(), s));
    int32_t m = 0;
    CSR_HIP(hipMemcpyAsync(&m, most.p, sizeof(m), hipMemcpyDeviceToHost, s));
    CSR_HIP(hipStreamSynchronize(s));
    A->wruns_L = A->tiles_L;
    A->wruns_state = m <= kRunsMax ? 1 : -1;
    return CSR_OK;
}

// Column blocks (the merge path's answer to x gathers that miss the L2, the
// latency bottleneck of Sec. III-A that the ML remedy targets): when x outgrows
// one XCD's L2, the rows are short (row-aligned tiles) and a row's columns
// spread over more x than a slab holds (the average row bandwidth bw_avg of
// Table I), the columns are cut into slabs of at most kSlabBytes of x and
// the product runs slab by slab, each pass gathering inside one slab (the
// L2 keeps it) and adding into y. Rows whose columns stay close (stencils,
// bands) already gather from a small window and would only pay the extra y
// traffic; so would rows with few nonzeros. Needs the features; 0 = one
// pass over all columns.
constexpr double kL2Bytes = 4.0 * 1024 * 1024;  // per XCD
constexpr double kSlabBytes = 2.0 * 1024 * 1024;

int column_blocks_for(const csr_matrix_s *A) {
    const double xb = A->storage == CSR_VAL_F64 ? 8.0 : 4.0;
    const double x_bytes = xb * A->n_cols;
    if (x_bytes <= kL2Bytes || A->n_rows == 0 || (double)A->nnz < 4.0 * A->n_rows) return 0;
    if (!A->has_features || A->feat.f[7] * xb <= kSlabBytes) return 0;
    const int B = (int)std::ceil(x_bytes / kSlabBytes);
    return std::min(B, 8);
}

csr_status_t build_colblocks(csr_matrix_s *A, int B, int L, hipStream_t s) {
    if (A->cb_B == B && A->cb_L == L) return CSR_OK;
    A->cb_B = 0;  // not valid until the end
    A->cb_L = 0;
    const int32_t n = A->n_rows;
    const int32_t width = (int32_t)((A->n_cols + (int64_t)B - 1) / B);
    const size_t vb = storage_bytes(A->storage);
    csr_status_t st;
    DevBuf cnt, off;
    if ((st = cnt.alloc(sizeof(int32_t) * (size_t)B * std::max(n, 1))) != CSR_OK) return st;
    CSR_HIP(launch_colblock_count(A->rp.as<int32_t>(), A->col.as<int32_t>(), n, B, width,
                                  cnt.as<int32_t>(), s));
    std::vector<int32_t> c((size_t)B * n), rpb((size_t)B * (n + 1));
    if (n > 0)
        CSR_HIP(hipMemcpyAsync(c.data(), cnt.p, sizeof(int32_t) * c.size(), hipMemcpyDeviceToHost, s));
    CSR_HIP(hipStreamSynchronize(s));
    std::vector<int64_t> nnz_off((size_t)B + 1, 0);
    for (int b = 0; b < B; ++b) {
        int32_t *r = rpb.data() + (size_t)b * (n + 1);
        int64_t run = 0;
        r[0] = 0;
        for (int32_t i = 0; i < n; ++i) {
            run += c[(size_t)b * n + i];
            r[i + 1] = (int32_t)run;
        }
        nnz_off[b + 1] = nnz_off[b] + run;
    }
    if ((st = A->cb_rp.alloc(sizeof(int32_t) * rpb.size())) != CSR_OK) return st;
    if ((st = A->cb_col.alloc(sizeof(int32_t) * (size_t)A->nnz + kPadBytes)) != CSR_OK) return st;
    if ((st = A->cb_val.alloc(vb * (size_t)A->nnz + kPadBytes)) != CSR_OK) return st;
    if ((st = off.alloc(sizeof(int64_t) * B)) != CSR_OK) return st;
    CSR_HIP(hipMemcpyAsync(A->cb_rp.p, rpb.data(), sizeof(int32_t) * rpb.size(),
                           hipMemcpyHostToDevice, s));
    CSR_HIP(hipMemcpyAsync(off.p, nnz_off.data(), sizeof(int64_t) * B, hipMemcpyHostToDevice, s));
    CSR_HIP(hipMemsetAsync(A->cb_col.as<char>() + sizeof(int32_t) * (size_t)A->nnz, 0, kPadBytes, s));
    CSR_HIP(hipMemsetAsync(A->cb_val.as<char>() + vb * (size_t)A->nnz, 0, kPadBytes, s));
    CSR_HIP(launch_colblock_scatter(A->rp.as<int32_t>(), A->col.as<int32_t>(), A->val.p, (int32_t)vb,
                                    n, B, width, A->cb_rp.as<int32_t>(), off.as<int64_t>(),
                                    A->cb_col.as<int32_t>(), A->cb_val.p, s));
    // each block's merge tiles (its rows are no longer than the matrix's, so
    // the matrix's slack keeps them row-aligned)
    const int64_t slack = merge_slack(A, L);
    // tiles that are not row-aligned: blocks after the first walk only the
    // rows with nonzeros in them (a row list; y is reached through it), so
    // that a block does not pay a path step for every row of the matrix
    const bool split = slack == 0;
    std::vector<int64_t> rows((size_t)B, n), rid_off((size_t)B + 1, 0), rrp_off((size_t)B + 1, 0);
    std::vector<int32_t> rid, rrp;
    if (split) {
        for (int b = 1; b < B; ++b) {
            const int32_t *cnt_b = c.data() + (size_t)b * n;
            rrp.push_back(0);
            int64_t run = 0, k = 0;
            for (int32_t i = 0; i < n; ++i) {
                if (cnt_b[i] == 0) continue;
                rid.push_back(i);
                run += cnt_b[i];
                rrp.push_back((int32_t)run);
                ++k;
            }
            rows[b] = k;
            rid_off[b + 1] = rid_off[b] + k;
            rrp_off[b + 1] = rrp_off[b] + k + 1;
        }
        if ((st = A->cb_rid.alloc(sizeof(int32_t) * std::max<size_t>(rid.size(), 1))) != CSR_OK)
            return st;
        if ((st = A->cb_rrp.alloc(sizeof(int32_t) * std::max<size_t>(rrp.size(), 1))) != CSR_OK)
            return st;
        if (!rid.empty())
            CSR_HIP(hipMemcpyAsync(A->cb_rid.p, rid.data(), sizeof(int32_t) * rid.size(),
                                   hipMemcpyHostToDevice, s));
        if (!rrp.empty())
            CSR_HIP(hipMemcpyAsync(A->cb_rrp.p, rrp.data(), sizeof(int32_t) * rrp.size(),
                                   hipMemcpyHostToDevice, s));
    }
    std::vector<int64_t> tiles((size_t)B), tile_off((size_t)B + 1, 0);
    for (int b = 0; b < B; ++b) {
        const int64_t total = rows[b] + (nnz_off[b + 1] - nnz_off[b]);
        tiles[b] = (total + (L - slack) - 1) / (L - slack);
        tile_off[b + 1] = tile_off[b] + tiles[b] + 1;
    }
    if ((st = A->cb_tile_i.alloc(sizeof(int32_t) * (size_t)tile_off[B])) != CSR_OK) return st;
    if ((st = A->cb_tile_j.alloc(sizeof(int32_t) * (size_t)tile_off[B])) != CSR_OK) return st;
    for (int b = 0; b < B; ++b) {
        const int32_t *rpb_dev = split && b > 0
                                     ? A->cb_rrp.as<int32_t>() + rrp_off[b]
                                     : A->cb_rp.as<int32_t>() + (size_t)b * (n + 1);
        CSR_HIP(launch_merge_partition(rpb_dev, (int32_t)rows[b], nnz_off[b + 1] - nnz_off[b], L,
                                       slack, tiles[b], A->cb_tile_i.as<int32_t>() + tile_off[b],
                                       A->cb_tile_j.as<int32_t>() + tile_off[b], s));
    }
    CSR_HIP(hipStreamSynchronize(s));
    A->cb_split = split ? 1 : 0;
    A->cb_rows = rows;
    A->cb_rid_off = rid_off;
    A->cb_rrp_off = rrp_off;
    A->cb_B = B;
    A->cb_width = width;
    A->cb_L = L;
    A->cb_nnz_off = nnz_off;
    A->cb_tile_off = tile_off;
    A->cb_tiles = tiles;
    return CSR_OK;
}

// Long rows: nnz_i > tau. The list (ascending) and the chunk layout are built
// on the host from a copy of row_ptr.
constexpr int32_t kLongChunk = 8192;

csr_status_t build_long_rows(csr_matrix_s *A, int64_t tau, hipStream_t s) {
    if (A->long_tau == tau) return CSR_OK;
    A->long_tau = -1;  // not valid until the end
    std::vector<int32_t> rp((size_t)A->n_rows + 1);
    CSR_HIP(hipMemcpyAsync(rp.data(), A->rp.p, sizeof(int32_t) * rp.size(),
                           hipMemcpyDeviceToHost, s));
    CSR_HIP(hipStreamSynchronize(s));
    std::vector<int32_t> rows, row_chunk{0}, chunks;
    for (int32_t i = 0; i < A->n_rows; ++i) {
        const int64_t k = (int64_t)rp[i + 1] - rp[i];
        if (k <= tau) continue;
        rows.push_back(i);
        for (int64_t b = rp[i]; b < rp[i + 1]; b += kLongChunk) {
            chunks.push_back((int32_t)b);
            chunks.push_back((int32_t)std::min<int64_t>(b + kLongChunk, rp[i + 1]));
        }
        row_chunk.push_back((int32_t)(chunks.size() / 2));
    }
    csr_status_t st;
    if ((st = A->long_list.alloc(sizeof(int32_t) * rows.size())) != CSR_OK) return st;
    if ((st = A->long_row_chunk.alloc(sizeof(int32_t) * row_chunk.size())) != CSR_OK) return st;
    if ((st = A->long_chunks.alloc(sizeof(int32_t) * chunks.size())) != CSR_OK) return st;
    if ((st = A->long_part.alloc(8 * (chunks.size() / 2))) != CSR_OK) return st;
    if (!rows.empty()) {
        CSR_HIP(hipMemcpyAsync(A->long_list.p, rows.data(), sizeof(int32_t) * rows.size(),
                               hipMemcpyHostToDevice, s));
        CSR_HIP(hipMemcpyAsync(A->long_row_chunk.p, row_chunk.data(),
                               sizeof(int32_t) * row_chunk.size(), hipMemcpyHostToDevice, s));
        CSR_HIP(hipMemcpyAsync(A->long_chunks.p, chunks.data(), sizeof(int32_t) * chunks.size(),
                               hipMemcpyHostToDevice, s));
        CSR_HIP(hipStreamSynchronize(s));
    }
    A->n_long = (int32_t)rows.size();
    A->n_long_chunks = (int64_t)chunks.size() / 2;
    A->long_tau = tau;
    return CSR_OK;
}

int64_t long_row_tau(const csr_matrix_s *A, const csr_config_t &cfg) {
    const double nnz_avg = A->n_rows ? (double)A->nnz / A->n_rows : 0.0;
    const double t = std::max(cfg.long_row_factor * nnz_avg, (double)cfg.long_row_floor);
    return (int64_t)t;
}

}  // namespace

csr_status_t inspect(csr_matrix_s *A, hipStream_t s);

bool plan_tables_ok(const csr_matrix_s *A, const Plan &P) {
    if (P.opts & CSR_OPT_MERGE) {
        if (P.cblocks > 0) return A->cb_B == P.cblocks && A->cb_L == P.L;
        if (A->tiles_L != P.L || A->n_tiles <= 0) return false;
        if (P.idx == IDX_W8) return A->wcode_state == 1 && A->wcodes_L == P.L && !A->wcode_wide;
        if (P.idx == IDX_W9) return A->wcode_state == 1 && A->wcodes_L == P.L && A->wcode_wide;
        if (P.idx == IDX_R8)
            return A->wcode_state == 1 && A->wcodes_L == P.L && A->wruns_state == 1 &&
                   A->wruns_L == P.L;
        if (P.idx == IDX_D8 || P.idx == IDX_D16)
            return A->mcodes_encoded && A->mcodes_L == P.L &&
                   A->mcode_bits == (P.idx == IDX_D8 ? 8 : 16);
        return true;
    }
    if ((P.idx == IDX_D8 || P.idx == IDX_D16) && A->code_bits != (P.idx == IDX_D8 ? 8 : 16))
        return false;
    if (P.long_rows && A->long_tau < 0) return false;
    if (P.dyn && !A->dyn_ctr.p) return false;
    return true;
}

// Realize an optimization mask as a concrete plan, building what it needs.
// Parameters not fixed by cfg take the defaults below; the autotuner varies
// them.
csr_status_t realize(csr_matrix_s *A, int32_t opts, const csr_config_t &cfg, Plan *out,
                     hipStream_t s) {
    Plan P;
    P.opts = opts;
    const double nnz_avg = A->n_rows ? (double)A->nnz / A->n_rows : 0.0;
    const int G0 = default_lanes_per_row(nnz_avg);
    P.G = G0;
    if (opts & CSR_OPT_UNROLL) {  // CMP: more rows per wave, independent accumulators
        P.G = G0 >= 2 ? G0 / 2 : 1;
        P.U = 4;
        P.R = 2;
    }
    if (opts & CSR_OPT_PREFETCH) {  // ML: streamed val/col, more gathers in flight
        P.nt = 1;
        P.R = 4;
    }
    if (cfg.rows_per_group > 0) P.G = cfg.rows_per_group;
    if (cfg.dynamic_rows != 0 && cfg.dynamic_rows != 1)
        return fail(CSR_ERR_INVALID_ARG, "dynamic_rows must be 0 or 1");
    if (cfg.dynamic_rows && !(opts & CSR_OPT_MERGE)) {
        // the row-split kernels' dynamic schedule: two counters, zeroed once
        // (the kernel leaves them zeroed)
        if (!A->dyn_ctr.p) {
            csr_status_t st0;
            if ((st0 = A->dyn_ctr.alloc(2 * sizeof(int32_t))) != CSR_OK) return st0;
            CSR_HIP(hipMemsetAsync(A->dyn_ctr.p, 0, 2 * sizeof(int32_t), s));
        }
        P.dyn = 1;
    }
    if (cfg.rows_in_flight > 0) P.R = cfg.rows_in_flight >= 4 ? 4 : cfg.rows_in_flight >= 2 ? 2 : 1;
    csr_status_t st;
    if (opts & CSR_OPT_MERGE) {
        // IMB (GPU counterpart of the runtime-chosen schedule). With DECOMP
        // as well, the merge path already balances long rows.
        int L = cfg.merge_items > 0 ? cfg.merge_items : 512;
        if (cfg.merge_items <= 0 && (opts & CSR_OPT_DELTA)) {
            // default tile size with codes: 1,024-item tiles when every
            // tile's window fits 9-bit ranks (fewer x-window cache lines per
            // nonzero; measured faster in every value storage), else 512
            if ((st = build_tiles(A, 16 * kMergeBlock, s)) != CSR_OK) return st;
            if (A->tiles_slack > 0) {
                if ((st = build_merge_codes(A, s, false)) != CSR_OK) return st;
                if (A->mcode_bits == 16) {
                    if ((st = build_window_codes(A, s)) != CSR_OK) return st;
                    if (A->wcode_state == 1 && A->wcode_wide) L = 16 * kMergeBlock;
                }
            }
        }
        if (!merge_items_supported(L))
            return fail(CSR_ERR_INVALID_ARG,
                        "merge_items must be a multiple of 256 from 256 to 2048");
        if ((st = build_tiles(A, L, s)) != CSR_OK) return st;
        P.L = L;
        if (opts & CSR_OPT_DELTA) {
            // MB: tile-base codes when every tile's column range fits 8 or
            // 16 bits (streamed, like the compressed arrays of the remedy);
            // on row-aligned tiles whose ranges need 16 bits, window codes
            // when every tile has at most kWindowMax distinct columns
            // (kWideWindowMax with 9-bit ranks on tiles of 1,024 items;
            // codes only at tile sizes where a lane's codes form whole loads)
            if ((st = build_merge_codes(A, s, false)) != CSR_OK) return st;
            const bool w8_fits = merge_codes_fit(L, 1);
            if (A->mcode_bits == 16 && A->tiles_slack > 0 && w8_fits) {
                if ((st = build_window_codes(A, s)) != CSR_OK) return st;
                // the same windows as runs of consecutive columns, when few
                // enough (their x loads then need no dictionary load first)
                if (A->wcode_state == 1 && cfg.window_runs == 1 &&
                    (st = build_window_runs(A, s)) != CSR_OK)
                    return st;
            }
            if (A->mcode_bits == 16 && A->wcode_state == 1 && w8_fits) {
                P.idx = A->wcode_wide ? IDX_W9
                        : cfg.window_runs == 1 && A->wruns_state == 1 && A->wruns_L == L
                            ? IDX_R8
                            : IDX_W8;
                P.nt = 1;
            } else if ((A->mcode_bits == 8 || A->mcode_bits == 16) &&
                       merge_codes_fit(L, A->mcode_bits / 8)) {
                if ((st = build_merge_codes(A, s, true)) != CSR_OK) return st;
                P.idx = A->mcode_bits == 8 ? IDX_D8 : IDX_D16;
                P.nt = 1;
            }
        }
        if (P.idx == IDX_I32 && (A->tiles_slack > 0 || cfg.split_row_blocks == 1)) {
            // int32 columns (no codes asked for, or the matrix is not
            // eligible for them): the merge path keeps its gathers inside
            // the L2, with column blocks when x outgrows it and the rows'
            // columns spread over it (on tiles that are not row-aligned
            // as well, unless turned off: every pass then carries its split
            // rows through the fixup, and the passes after the first walk
            // only the rows with nonzeros in their block)
            if (!A->has_features && (st = inspect(A, s)) != CSR_OK) return st;
            const int B = column_blocks_for(A);
            if (B >= 2) {
                if ((st = build_colblocks(A, B, L, s)) != CSR_OK) return st;
                P.cblocks = B;
            }
        }
        P.G = 0;
        P.U = 1;
        P.R = 1;
        if (!merge_items_prebuilt(L)) {
            // compile (or find) the run-time instance this plan launches, so
            // that a failed compilation is reported here and not at launch
            hipFunction_t f;
            const bool x32 = x_fits_32(A);
            st = P.cblocks ? jit_merge_kernel(A->device, A->storage, L / kMergeBlock, false, x32,
                                              IDX_I32, A->tiles_fixup == 0, &f)
                           : jit_merge_kernel(A->device, A->storage, L / kMergeBlock, P.nt != 0,
                                              x32, P.idx, A->tiles_fixup == 0, &f);
            if (st != CSR_OK) return st;
            P.jit = 1;
        }
    } else if (opts & CSR_OPT_DECOMP) {
        if ((st = build_long_rows(A, long_row_tau(A, cfg), s)) != CSR_OK) return st;
        P.long_rows = 1;
    }
    if ((opts & CSR_OPT_DELTA) && !(opts & CSR_OPT_MERGE)) {
        // MB: delta codes; when the matrix is not eligible only the wide-load
        // half of the remedy applies
        if ((st = build_delta(A, s)) != CSR_OK) return st;
        if (A->code_bits == 8 || A->code_bits == 16) {
            P.idx = A->code_bits == 8 ? IDX_D8 : IDX_D16;
            P.U = 1;
            P.R = 1;
        } else {
            P.U = 4;
        }
    }
    *out = P;
    return CSR_OK;
}

// --------------------------------------------------------------------------
// Timing
// --------------------------------------------------------------------------
namespace {

csr_status_t ensure_scratch(csr_matrix_s *A, hipStream_t s) {
    const size_t xb = A->storage == CSR_VAL_F64 ? 8 : 4;
    csr_status_t st;
    if (!A->scratch_x.p) {
        if ((st = A->scratch_x.alloc(xb * (size_t)A->n_cols)) != CSR_OK) return st;
        CSR_HIP(hipMemsetAsync(A->scratch_x.p, 0, A->scratch_x.bytes, s));
    }
    if (!A->scratch_y.p) {
        if ((st = A->scratch_y.alloc(xb * (size_t)A->n_rows)) != CSR_OK) return st;
    }
    return CSR_OK;
}

// `calls` back-to-back SpMVs between two events, `runs` times, after one
// untimed call. Returns the time per call as the reciprocal of the harmonic
// mean of the per-run rates (Sec. IV-A): the mean of the per-run times.
template <class Launch>
csr_status_t time_launches(Launch &&launch, int calls, int runs, hipStream_t s,
                           double *ms_per_call) {
    hipEvent_t e0, e1;
    CSR_HIP(hipEventCreate(&e0));
    hipError_t e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(e, "hipEventCreate");
    }
    e = launch();
    double sum = 0.0;
    for (int r = 0; r < runs && e == hipSuccess; ++r) {
        e = hipEventRecord(e0, s);
        for (int c = 0; c < calls && e == hipSuccess; ++c) e = launch();
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        sum += (double)ms / calls;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return hip_fail(e, "timed launches");
    *ms_per_call = sum / runs;
    return CSR_OK;
}

csr_status_t time_plan(csr_matrix_s *A, const Plan &P, int calls, int runs, hipStream_t s,
                       double *ms) {
    csr_status_t st = ensure_scratch(A, s);
    if (st != CSR_OK) return st;
    return time_launches([&] { return launch_spmv(A, P, A->scratch_x.p, A->scratch_y.p, s); },
                         calls, runs, s, ms);
}

bool opts_realizable(int32_t opts) { return (opts & ~31) == 0; }

csr_status_t ensure_row_index(csr_matrix_s *A, hipStream_t s) {
    if (A->scratch_col.p) return CSR_OK;
    csr_status_t st;
    if ((st = A->scratch_col.alloc(sizeof(int32_t) * (size_t)A->nnz + kPadBytes)) != CSR_OK)
        return st;
    CSR_HIP(launch_fill_row_index(A->rp.as<int32_t>(), A->n_rows, A->n_cols,
                                  A->scratch_col.as<int32_t>(), s));
    return CSR_OK;
}

// The micro-benchmarks of Sec. III-B on the baseline kernel (G lanes per
// row): which = 1 P_ML (colind := row index), 2 P_CMP (no colind, x[row]).
hipError_t launch_probe(const csr_matrix_s *A, int G, int which, const void *x, void *y,
                        hipStream_t s) {
    const void *col = which == 1 ? A->scratch_col.p : A->col.p;
    const int probe = which == 2 ? 1 : 0;
    const void *arr[8] = {A->rp.p, col, nullptr, A->val.p, x, y, nullptr, nullptr};
    switch (A->storage) {
    case CSR_VAL_F64:
        return launch_rowsplit_s0(G, IDX_I32, false, 1, 1, probe, arr, INT32_MAX, A->n_rows,
                                  A->n_cols, s);
    case CSR_VAL_F32:
        return launch_rowsplit_s1(G, IDX_I32, false, 1, 1, probe, arr, INT32_MAX, A->n_rows,
                                  A->n_cols, s);
    default:
        return launch_rowsplit_s2(G, IDX_I32, false, 1, 1, probe, arr, INT32_MAX, A->n_rows,
                                  A->n_cols, s);
    }
}

}  // namespace

// --------------------------------------------------------------------------
// B_max: triad bandwidth at an HBM-sized and an Infinity-Cache-sized
// footprint, measured once per device (Sec. III-B footnote on cache-resident
// working sets; Sec. IV-A, Table III).
// --------------------------------------------------------------------------
csr_status_t device_bandwidth(int device, hipStream_t s, double *hbm, double *cache) {
    static std::mutex mu;
    static std::map<int, DeviceBandwidth> known;
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = known.find(device);
        if (it != known.end()) {
            *hbm = it->second.hbm;
            *cache = it->second.cache;
            return CSR_OK;
        }
    }
    DeviceBandwidth d;
    csr_status_t st;
    // HBM: 3 x 1 GiB with non-temporal accesses. Cache: 3 x 48 MiB (inside
    // the 256 MB Infinity Cache) with ordinary accesses, so that repeated
    // passes hit there. The cache figure never goes below the HBM one.
    if ((st = triad_bandwidth((size_t)1 << 30, 3, true, s, &d.hbm)) != CSR_OK) return st;
    if ((st = triad_bandwidth((size_t)48 << 20, 5, false, s, &d.cache)) != CSR_OK) return st;
    if (d.cache < d.hbm) d.cache = d.hbm;
    std::lock_guard<std::mutex> lk(mu);
    known[device] = d;
    *hbm = d.hbm;
    *cache = d.cache;
    return CSR_OK;
}

// --------------------------------------------------------------------------
// Features (Sec. III-D, Table I)
// --------------------------------------------------------------------------
// The feature sweep's workspace (partials, long-row list, x-reuse samples),
// sized from the matrix's shape; allocated with the handle so that an
// inspection launches and reads back only.
csr_status_t feature_buffers(csr_matrix_s *A) {
    if (A->n_rows == 0) return CSR_OK;
    const double nnz_avg = (double)A->nnz / A->n_rows;
    const int G0 = default_lanes_per_row(nnz_avg);
    const int G = G0 >= 4 ? G0 / 4 : 1;
    const size_t n_slots = (size_t)(features_partials(A->n_rows, G) +
                                    features_long_capacity(A->nnz, G));
    const size_t n_long = (size_t)features_long_capacity(A->nnz, G) + 1;
    const size_t n_out = kFeatHeader + sizeof(int32_t) * 2 * (size_t)xreuse_samples(A->n_rows);
    csr_status_t st;
    if (A->feat_parts.bytes < sizeof(FeatPart) * n_slots &&
        (st = A->feat_parts.alloc(sizeof(FeatPart) * n_slots)) != CSR_OK)
        return st;
    if (A->feat_long.bytes < sizeof(int32_t) * n_long &&
        (st = A->feat_long.alloc(sizeof(int32_t) * n_long)) != CSR_OK)
        return st;
    const size_t n_bits = sizeof(uint32_t) * (((size_t)A->n_rows + 31) / 32);
    if (A->feat_bits.bytes < n_bits && (st = A->feat_bits.alloc(n_bits)) != CSR_OK) return st;
    if (A->feat_reuse.bytes < n_out && (st = A->feat_reuse.alloc(n_out)) != CSR_OK) return st;
    if (A->feat_host.bytes < n_out && (st = A->feat_host.alloc(n_out)) != CSR_OK) return st;
    return CSR_OK;
}

csr_status_t inspect(csr_matrix_s *A, hipStream_t s) {
    const auto t0 = Clock::now();
    csr_features_t F{};
    F.rows_sorted = A->rows_sorted;
    const int64_t N = A->n_rows;
    if (N > 0) {
        const double nnz_avg = (double)A->nnz / N;
        const int G0 = default_lanes_per_row(nnz_avg);
        const int G = G0 >= 4 ? G0 / 4 : 1;  // contiguous segments of about 4 entries per lane
        const int32_t n_parts = features_partials(A->n_rows, G);
        const int32_t n_samp = xreuse_samples(A->n_rows);
        csr_status_t st;
        if ((st = feature_buffers(A)) != CSR_OK) return st;  // allocated by csr_create
        CSR_HIP(launch_features(A->rp.as<int32_t>(), A->col.as<int32_t>(), A->n_rows, G,
                                A->feat_parts.as<FeatPart>(), n_parts, A->feat_long.as<int32_t>(),
                                A->feat_bits.as<uint32_t>(), A->feat_reuse.p, s));
        // one round trip when no row was long: the fold, the long-row count
        // and the x-reuse samples in one copy to pinned memory
        const size_t out_bytes = kFeatHeader + sizeof(int32_t) * 2 * (size_t)n_samp;
        const char *const h = static_cast<const char *>(A->feat_host.p);
        CSR_HIP(hipMemcpyAsync(A->feat_host.p, A->feat_reuse.p, out_bytes, hipMemcpyDeviceToHost, s));
        CSR_HIP(hipStreamSynchronize(s));
        FeatPart p;
        int32_t n_long = 0;
        std::memcpy(&p, h, sizeof(p));
        std::memcpy(&n_long, h + sizeof(FeatPart), sizeof(n_long));
        std::vector<int32_t> reuse(2 * (size_t)n_samp);
        if (n_samp > 0) std::memcpy(reuse.data(), h + kFeatHeader, sizeof(int32_t) * reuse.size());
        if (n_long != 0) {
            CSR_HIP(features_long_rows(A->rp.as<int32_t>(), A->col.as<int32_t>(), A->n_rows,
                                       A->nnz, G, A->feat_parts.as<FeatPart>(), n_parts,
                                       A->feat_long.as<int32_t>(), A->feat_bits.as<uint32_t>(),
                                       n_long, A->feat_reuse.p, s));
            CSR_HIP(hipMemcpyAsync(A->feat_host.p, A->feat_reuse.p, sizeof(p),
                                   hipMemcpyDeviceToHost, s));
            CSR_HIP(hipStreamSynchronize(s));
            std::memcpy(&p, h, sizeof(p));
        }
        int64_t shared = 0, distinct = 0;
        for (int32_t q = 0; q < n_samp; ++q) {
            shared += reuse[2 * q];
            distinct += reuse[2 * q + 1];
        }
        const int64_t s1 = A->nnz;
        const double dN = (double)N;
        // population variance from exact integer sums: (N*S2 - S1^2) / N^2
        auto ivar = [&](int64_t sum, int64_t sum2) {
            const __int128 num = (__int128)N * sum2 - (__int128)sum * sum;
            return (double)num / (dN * dN);
        };
        const double bytes = 12.0 * (double)A->nnz + 4.0 * (double)(N + 1) +
                             8.0 * (double)A->n_cols + 8.0 * (double)N;
        F.f[0] = dN;
        F.f[1] = p.nnz_min;
        F.f[2] = p.nnz_max;
        F.f[3] = (double)s1 / dN;
        F.f[4] = std::sqrt(std::max(0.0, ivar(s1, p.s_nnz2)));
        F.f[5] = p.bw_min;
        F.f[6] = p.bw_max;
        F.f[7] = (double)p.s_bw / dN;
        F.f[8] = std::sqrt(std::max(0.0, ivar(p.s_bw, p.s_bw2)));
        F.f[9] = p.sc_mean;
        F.f[10] = std::sqrt(std::max(0.0, p.sc_m2 / dN));
        F.f[11] = p.s_cl / dN;
        F.f[12] = (double)p.s_miss / dN;
        F.f[13] = bytes <= kCacheBytes ? 1.0 : 0.0;
        F.f[14] = p.s_len1 ? (double)p.s_bw / (double)p.s_len1 : 0.0;
        F.f[15] = distinct ? (double)shared / (double)distinct : 0.0;
        F.isum[0] = s1;
        F.isum[1] = p.s_nnz2;
        F.isum[2] = p.s_bw;
        F.isum[3] = p.s_bw2;
        F.isum[4] = p.s_miss;
        F.isum[5] = p.s_grp;
        F.isum[6] = shared;
        F.isum[7] = distinct;
    }
    A->feat = F;
    A->has_features = 1;
    A->t_inspect_ms = ms_since(t0);
    return CSR_OK;
}

// --------------------------------------------------------------------------
// Profile-guided classification (Sec. III-B bounds, Sec. III-C rule)
// --------------------------------------------------------------------------
namespace {

struct Bounds {
    double p_csr, p_mb, p_ml, p_imb, p_cmp, p_peak, b_max;
    int32_t ml_parts, ml_flagged;  // partition-aware ML test (cfg.ml_partitions > 0)
    double ml_part_max;
};

// Contiguous partitions of the baseline's row blocks (NG rows each) with
// about nnz/Q nonzeros each, the static one-dimensional partitioning of
// Sec. IV-A applied to blocks: bound[q] is the first block whose first
// nonzero index is at least floor(q * nnz / Q); bound[0] = 0 and
// bound[Q] = the number of blocks. Empty partitions (bound[q] = bound[q+1])
// occur where one block holds more than nnz/Q nonzeros.
std::vector<int32_t> ml_partition_bounds(const std::vector<int32_t> &rp, int NG, int Q) {
    const int64_t n = (int64_t)rp.size() - 1, nnz = rp.back();
    const int64_t nblk = (n + NG - 1) / NG;
    auto first_nz = [&](int64_t b) { return (int64_t)rp[(size_t)std::min(b * NG, n)]; };
    std::vector<int32_t> bound((size_t)Q + 1);
    for (int q = 0; q < Q; ++q) {
        const int64_t target = (int64_t)q * nnz / Q;
        int64_t lo = 0, hi = nblk;  // first b in [0, nblk] with first_nz(b) >= target
        while (lo < hi) {
            const int64_t mid = (lo + hi) / 2;
            if (first_nz(mid) >= target) hi = mid;
            else lo = mid + 1;
        }
        bound[q] = (int32_t)lo;
    }
    bound[Q] = (int32_t)nblk;
    return bound;
}

// Per partition: summed baseline block times over summed probe block times
// (t[b] baseline, t[nblk + b] probe); 0 for a partition without blocks or
// without measurable time.
std::vector<double> ml_partition_ratios(const std::vector<int64_t> &t,
                                        const std::vector<int32_t> &bound) {
    const size_t nblk = t.size() / 2;
    std::vector<double> r(bound.size() - 1, 0.0);
    for (size_t q = 0; q + 1 < bound.size(); ++q) {
        int64_t sc = 0, sm = 0;
        for (int64_t b = bound[q]; b < bound[q + 1]; ++b) {
            sc += t[b];
            sm += t[nblk + b];
        }
        if (sc > 0 && sm > 0) r[q] = (double)sc / (double)sm;
    }
    return r;
}

csr_status_t measure_bounds(csr_matrix_s *A, const csr_config_t &cfg, hipStream_t s, Bounds *B) {
    const int calls = cfg.timing_calls > 0 ? cfg.timing_calls : 32;
    const double flops = 2.0 * (double)A->nnz;
    csr_config_t dc;
    csr_config_default(&dc);
    Plan P0;
    csr_status_t st;
    if ((st = realize(A, 0, dc, &P0, s)) != CSR_OK) return st;
    double t_csr = 0, t_ml = 0, t_cmp = 0;
    if ((st = time_plan(A, P0, calls, 3, s, &t_csr)) != CSR_OK) return st;
    // P_ML: the baseline kernel on colind := row (same bytes, regular x)
    if ((st = ensure_row_index(A, s)) != CSR_OK) return st;
    if ((st = time_launches([&] { return launch_probe(A, P0.G, 1, A->scratch_x.p, A->scratch_y.p, s); },
                            calls, 3, s, &t_ml)) != CSR_OK)
        return st;
    // P_CMP: no column stream, x read at the row index
    if ((st = time_launches([&] { return launch_probe(A, P0.G, 2, A->scratch_x.p, A->scratch_y.p, s); },
                            calls, 3, s, &t_cmp)) != CSR_OK)
        return st;
    // P_IMB: per-CU busy spans of the instrumented baseline
    const int NG = kBlock / P0.G;
    const int64_t nblk = (A->n_rows + NG - 1) / NG;
    DevBuf rec;
    if ((st = rec.alloc(sizeof(int64_t) * 3 * (size_t)std::max<int64_t>(nblk, 1))) != CSR_OK)
        return st;
    // one instrumented launch (the baseline on `colp`), records copied to h
    auto instrumented = [&](const void *colp, std::vector<int64_t> &h) -> csr_status_t {
        const void *arr[8] = {A->rp.p, colp, nullptr, A->val.p, A->scratch_x.p,
                              A->scratch_y.p, rec.p, nullptr};
        hipError_t e;
        switch (A->storage) {
        case CSR_VAL_F64:
            e = launch_rowsplit_s0(P0.G, IDX_I32, false, 1, 1, 2, arr, INT32_MAX, A->n_rows,
                                   A->n_cols, s);
            break;
        case CSR_VAL_F32:
            e = launch_rowsplit_s1(P0.G, IDX_I32, false, 1, 1, 2, arr, INT32_MAX, A->n_rows,
                                   A->n_cols, s);
            break;
        default:
            e = launch_rowsplit_s2(P0.G, IDX_I32, false, 1, 1, 2, arr, INT32_MAX, A->n_rows,
                                   A->n_cols, s);
            break;
        }
        if (e != hipSuccess) return hip_fail(e, "instrumented baseline");
        h.assign(3 * (size_t)nblk, 0);
        if (nblk > 0) {
            CSR_HIP(hipMemcpyAsync(h.data(), rec.p, sizeof(int64_t) * h.size(),
                                   hipMemcpyDeviceToHost, s));
        }
        CSR_HIP(hipStreamSynchronize(s));
        return CSR_OK;
    };
    std::vector<int64_t> h;
    if ((st = instrumented(A->col.p, h)) != CSR_OK) return st;
    {
        std::map<int64_t, std::pair<int64_t, int64_t>> span;  // cu -> (min start, max end)
        for (int64_t b = 0; b < nblk; ++b) {
            auto it = span.find(h[3 * b + 2]);
            if (it == span.end()) span[h[3 * b + 2]] = {h[3 * b], h[3 * b + 1]};
            else {
                it->second.first = std::min(it->second.first, h[3 * b]);
                it->second.second = std::max(it->second.second, h[3 * b + 1]);
            }
        }
        // the "threads" of Sec. III-B are the compute units: each one's time
        // is the span from its first workgroup's start to its last one's end
        A->imb_spans.clear();
        for (auto &kv : span) A->imb_spans.push_back(kv.second.second - kv.second.first);
        A->imb_clock_hz = device_wall_clock_hz(A->device);
    }
    // Partition-aware ML (the extension proposed with the results of
    // Sec. IV-C): the P_ML comparison repeated on contiguous nnz-balanced
    // partitions of the row blocks, from per-block times of the instrumented
    // baseline and of the instrumented P_ML probe (shortest of kMlReps runs).
    A->mlp_bounds.clear();
    A->mlp_times.clear();
    A->mlp_ratios.clear();
    B->ml_parts = 0;
    B->ml_flagged = 0;
    B->ml_part_max = 0.0;
    if (cfg.ml_partitions > 0 && nblk > 0) {
        constexpr int kMlReps = 3;
        std::vector<int64_t> t((size_t)2 * nblk, INT64_MAX);
        for (int r = 0; r < kMlReps; ++r) {
            if (r > 0 && (st = instrumented(A->col.p, h)) != CSR_OK) return st;
            for (int64_t b = 0; b < nblk; ++b) t[b] = std::min(t[b], h[3 * b + 1] - h[3 * b]);
            if ((st = instrumented(A->scratch_col.p, h)) != CSR_OK) return st;
            for (int64_t b = 0; b < nblk; ++b)
                t[nblk + b] = std::min(t[nblk + b], h[3 * b + 1] - h[3 * b]);
        }
        std::vector<int32_t> rp_h((size_t)A->n_rows + 1);
        CSR_HIP(hipMemcpyAsync(rp_h.data(), A->rp.p, sizeof(int32_t) * rp_h.size(),
                               hipMemcpyDeviceToHost, s));
        CSR_HIP(hipStreamSynchronize(s));
        A->mlp_bounds = ml_partition_bounds(rp_h, NG, cfg.ml_partitions);
        A->mlp_ratios = ml_partition_ratios(t, A->mlp_bounds);
        A->mlp_times = std::move(t);
        for (double r : A->mlp_ratios) {
            if (r <= 0.0) continue;
            B->ml_parts += 1;
            if (r > cfg.t_ml_part) B->ml_flagged += 1;
            B->ml_part_max = std::max(B->ml_part_max, r);
        }
    }
    double b_hbm = 0, b_cache = 0;
    if ((st = device_bandwidth(A->device, s, &b_hbm, &b_cache)) != CSR_OK) return st;
    const double xb = A->storage == CSR_VAL_F64 ? 8.0 : 4.0;
    const double vb = (double)storage_bytes(A->storage);
    const double sx = xb * A->n_cols, sy = xb * A->n_rows;
    const double s_fmt = (double)A->nnz * (vb + 4.0) + 4.0 * (A->n_rows + 1);
    const double bmax = (s_fmt + sx + sy) <= kCacheBytes ? b_cache : b_hbm;
    B->b_max = bmax;
    A->bw_hbm = b_hbm;
    A->bw_cache = b_cache;
    B->p_csr = flops / (t_csr * 1e-3);
    B->p_ml = flops / (t_ml * 1e-3);
    B->p_cmp = flops / (t_cmp * 1e-3);
    // P_IMB = 2 NNZ / t_median, t_median the median span over the compute
    // units that ran work (for an even count the mean of the two middle
    // ones); without spans the baseline's own rate
    B->p_imb = B->p_csr;
    if (!A->imb_spans.empty()) {
        std::vector<int64_t> d = A->imb_spans;
        std::sort(d.begin(), d.end());
        const size_t m = d.size() / 2;
        const double med = d.size() % 2 ? (double)d[m] : 0.5 * ((double)d[m - 1] + (double)d[m]);
        if (med > 0) B->p_imb = flops / (med / A->imb_clock_hz);
    }
    B->p_mb = flops / ((s_fmt + sx + sy) / bmax);
    B->p_peak = flops / (((double)A->nnz * vb + sx + sy) / bmax);
    return CSR_OK;
}

}  // namespace

// The profile-guided classifier (Sec. III-C, Fig. 4). Every bottleneck
// class has its own test on the bounds of Sec. III-B, independent of the
// others, and a matrix belongs to every class whose test holds:
//   IMB  removing the imbalance would pay: P_IMB / P_CSR above t_imb;
//   ML   regular x accesses would pay: P_ML / P_CSR above t_ml;
//   MB   the baseline already streams near the bandwidth bound (P_CSR at
//        least t_mb P_MB, the reading of the paper's "approximately equal")
//        while dropping the index stream stays between the two
//        bandwidth bounds (P_MB < P_CMP < P_peak);
//   CMP  the no-index probe falls outside those bounds (P_CMP below P_MB or
//        above P_peak).
namespace {
struct ClassTest {
    int32_t cls;
    bool (*holds)(const double *p, const csr_config_t &cfg);  // p: csr, mb, ml, imb, cmp, peak
};
enum { B_CSR, B_MB, B_ML, B_IMB, B_CMP, B_PEAK };
constexpr ClassTest kClassTests[] = {
    {CSR_CLS_MB, [](const double *p, const csr_config_t &c) {
         return p[B_CSR] >= c.t_mb * p[B_MB] && p[B_MB] < p[B_CMP] && p[B_CMP] < p[B_PEAK];
     }},
    {CSR_CLS_ML, [](const double *p, const csr_config_t &c) { return p[B_ML] / p[B_CSR] > c.t_ml; }},
    {CSR_CLS_IMB, [](const double *p, const csr_config_t &c) { return p[B_IMB] / p[B_CSR] > c.t_imb; }},
    {CSR_CLS_CMP, [](const double *p, const csr_config_t &) {
         return p[B_CMP] < p[B_MB] || p[B_CMP] > p[B_PEAK];
     }},
};
}  // namespace

int32_t classify(double p_csr, double p_mb, double p_ml, double p_imb, double p_cmp,
                 double p_peak, const csr_config_t &cfg) {
    const double p[] = {p_csr, p_mb, p_ml, p_imb, p_cmp, p_peak};
    int32_t classes = 0;
    for (const ClassTest &t : kClassTests)
        if (t.holds(p, cfg)) classes |= t.cls;
    return classes;
}

// Table II: classes -> optimizations, applied jointly.
// map 0: as the paper's table; map 1: the pool as it pays on this GPU
// (measured over the suite): irregular x gathers go to the merge path (its
// window codes and column blocks keep gathers close), imbalance to the
// merge path with compressed column codes (the decomposition when long rows
// exist), and the computation class has no remedy that pays here.
int32_t remedies(int32_t classes, bool has_long_rows, int map) {
    int32_t o = 0;
    if (classes & CSR_CLS_MB) o |= CSR_OPT_DELTA;
    if (map == 1) {
        if (classes & CSR_CLS_ML) o |= CSR_OPT_MERGE | CSR_OPT_DELTA;
        if (classes & CSR_CLS_IMB)
            o |= has_long_rows ? CSR_OPT_DECOMP : (CSR_OPT_MERGE | CSR_OPT_DELTA);
        return o;
    }
    if (classes & CSR_CLS_ML) o |= CSR_OPT_PREFETCH;
    if (classes & CSR_CLS_IMB) o |= has_long_rows ? CSR_OPT_DECOMP : CSR_OPT_MERGE;
    if (classes & CSR_CLS_CMP) o |= CSR_OPT_UNROLL;
    return o;
}

namespace {

// A few parameter settings of the chosen optimization set, timed; the
// fastest is kept.
csr_status_t autotune(csr_matrix_s *A, int32_t opts, const csr_config_t &cfg, hipStream_t s,
                      Plan *best, csr_config_t *best_cfg) {
    const int calls = cfg.timing_calls > 0 ? cfg.timing_calls : 32;
    std::vector<csr_config_t> cands;
    const double nnz_avg = A->n_rows ? (double)A->nnz / A->n_rows : 0.0;
    const int G0 = default_lanes_per_row(nnz_avg);
    if (opts & CSR_OPT_MERGE) {
        std::vector<int> sizes = {256, 512, 1024};
        if (cfg.jit_tiles) sizes.insert(sizes.end(), {768, 1536});  // compiled at run time
        // column blocks on tiles that are not row-aligned: timed both ways
        // where they would apply
        if (!A->has_features) {
            csr_status_t st0 = inspect(A, s);
            if (st0 != CSR_OK) return st0;
        }
        const bool split_blocks = column_blocks_for(A) >= 2;
        for (int L : sizes) {
            csr_config_t c = cfg;
            c.merge_items = L;
            cands.push_back(c);
            if (opts & CSR_OPT_DELTA) {  // window codes: dictionary or run records
                csr_config_t w = c;
                w.window_runs = 1 - cfg.window_runs;
                cands.push_back(w);
            }
            if (split_blocks && merge_slack(A, L) == 0) {
                c.split_row_blocks = 1 - cfg.split_row_blocks;
                cands.push_back(c);
            }
        }
    } else {
        const int gs[3] = {G0, G0 >= 2 ? G0 / 2 : 1, G0 <= 32 ? G0 * 2 : 64};
        for (int g : gs)
            for (int r : {1, 4}) {
                csr_config_t c = cfg;
                c.rows_per_group = g;
                c.rows_in_flight = r;
                cands.push_back(c);
            }
        if (opts & CSR_OPT_DECOMP) {
            // imbalance: the dynamic schedule as well (Sec. IV-A's runtime-chosen
            // schedule on the row-parallel kernel)
            for (int g : gs) {
                csr_config_t c = cfg;
                c.rows_per_group = g;
                c.rows_in_flight = 1;
                c.dynamic_rows = 1;
                cands.push_back(c);
            }
        }
    }
    double best_ms = 1e300;
    size_t best_k = 0;
    bool best_plain_loads = false;
    for (size_t k = 0; k < cands.size(); ++k) {
        Plan Q;
        csr_status_t st = realize(A, opts, cands[k], &Q, s);
        if (st != CSR_OK) return st;
        // ML's streaming half (non-temporal val/col loads) is timed against
        // ordinary loads: on this GPU it often costs more than it saves.
        // Plans whose loads stream regardless (merge codes) or never
        // (column blocks) have one setting.
        const bool twin = (opts & CSR_OPT_PREFETCH) && Q.nt && !Q.cblocks &&
                          !(Q.G == 0 && Q.idx != IDX_I32);
        for (int plain_loads = 0; plain_loads <= (twin ? 1 : 0); ++plain_loads) {
            if (plain_loads) Q.nt = 0;
            double ms = 0;
            if ((st = time_plan(A, Q, calls, 2, s, &ms)) != CSR_OK) return st;
            if (ms < best_ms) {
                best_ms = ms;
                best_k = k;
                best_plain_loads = plain_loads != 0;
            }
        }
    }
    // The matrix holds one set of derived tables (tiles, long rows, codes),
    // rebuilt by each candidate: realize the winner again so that its tables
    // are the ones in place (cached per parameter, so this is cheap).
    csr_status_t st = realize(A, opts, cands[best_k], best, s);
    if (st == CSR_OK && best_plain_loads) best->nt = 0;
    *best_cfg = cands[best_k];
    return st;
}

}  // namespace

}  // namespace csr

using namespace csr;

// Feature-guided classifier (Sec. III-D): a CART tree over the 16 features
// that predicts the profile-guided classes; walked on the host.
namespace {
struct TreeNode {
    int32_t feature;  // -1 at a leaf
    double threshold; // go left when f[feature] <= threshold
    int32_t left, right;
    int32_t value;    // class mask at a leaf
};
std::mutex g_tree_mu;
std::vector<TreeNode> *const g_tree = new std::vector<TreeNode>;  // empty: no tree

// The class mask the tree predicts for the features f, -1 without a tree.
// Children always follow their parent, so the walk ends.
int32_t tree_classes(const double *f) {
    std::lock_guard<std::mutex> lk(g_tree_mu);
    if (g_tree->empty()) return -1;
    size_t k = 0;
    while ((*g_tree)[k].feature >= 0) {
        const TreeNode &n = (*g_tree)[k];
        k = (size_t)(f[n.feature] <= n.threshold ? n.left : n.right);
    }
    return (*g_tree)[k].value;
}
}  // namespace

extern "C" {

csr_status_t csr_tree_load(int32_t n_nodes, const int32_t *feature, const double *threshold,
                           const int32_t *left, const int32_t *right, const int32_t *value) {
    if (n_nodes < 1 || n_nodes > (1 << 20) || !feature || !threshold || !left || !right || !value)
        return fail(CSR_ERR_INVALID_ARG, "bad tree arrays");
    std::vector<TreeNode> t((size_t)n_nodes);
    for (int32_t k = 0; k < n_nodes; ++k) {
        TreeNode &n = t[(size_t)k];
        n = TreeNode{feature[k], threshold[k], left[k], right[k], value[k]};
        if (n.feature < -1 || n.feature >= 16)
            return fail(CSR_ERR_INVALID_ARG, "tree feature index out of range");
        if (n.feature >= 0) {
            if (!std::isfinite(n.threshold)) return fail(CSR_ERR_INVALID_ARG, "non-finite threshold");
            if (n.left <= k || n.left >= n_nodes || n.right <= k || n.right >= n_nodes)
                return fail(CSR_ERR_INVALID_ARG, "a child must follow its parent");
        } else if (n.value < 0 || n.value > 15) {
            return fail(CSR_ERR_INVALID_ARG, "leaf class mask out of range");
        }
    }
    std::lock_guard<std::mutex> lk(g_tree_mu);
    g_tree->swap(t);
    return CSR_OK;
}

csr_status_t csr_tree_unload(void) {
    std::lock_guard<std::mutex> lk(g_tree_mu);
    g_tree->clear();
    return CSR_OK;
}

csr_status_t csr_inspect(csr_matrix_t A, csr_features_t *out, void *stream) {
    if (!A || !out) return fail(CSR_ERR_INVALID_ARG, "NULL argument");
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (prev != A->device) (void)hipSetDevice(A->device);
    csr_status_t st = inspect(A, (hipStream_t)stream);
    if (prev >= 0 && prev != A->device) (void)hipSetDevice(prev);
    if (st != CSR_OK) return st;
    *out = A->feat;
    return CSR_OK;
}

namespace {
// After a failed selection: the candidates it built may have replaced the
// tables of the committed plan (they share the handle's tile table, codes,
// column blocks and long-row list). Rebuild them; if that fails too, fall
// back to the plain plan, which reads only row_ptr, col_idx and val. The
// failure's message is kept.
void restore_plan(csr_matrix_s *A, hipStream_t s) {
    if (plan_tables_ok(A, A->plan)) return;
    const std::string why = csr_last_error();
    Plan Q;
    const bool rebuilt = realize(A, A->plan.opts, A->plan_cfg, &Q, s) == CSR_OK &&
                         plan_tables_ok(A, A->plan);
    if (!rebuilt) {
        csr_config_t dc;
        csr_config_default(&dc);
        (void)realize(A, 0, dc, &Q, s);  // builds nothing
        A->plan = Q;
        A->plan_cfg = dc;
        A->info = csr_plan_info_t{};
        A->info.classes = -1;
        fill_info(A, Q, &A->info);
        A->version += 1;
    }
    (void)hipStreamSynchronize(s);
    set_error(why);
}
}  // namespace

csr_status_t csr_select(csr_matrix_t A, int32_t mode, const csr_config_t *cfg_in,
                        csr_plan_info_t *out, void *stream) {
    if (!A) return fail(CSR_ERR_INVALID_ARG, "NULL handle");
    csr_config_t cfg;
    if (cfg_in) cfg = *cfg_in;
    else csr_config_default(&cfg);
    if (cfg.remedy_map != 0 && cfg.remedy_map != 1)
        return fail(CSR_ERR_INVALID_ARG, "remedy_map must be 0 or 1");
    if (cfg.split_row_blocks != 0 && cfg.split_row_blocks != 1)
        return fail(CSR_ERR_INVALID_ARG, "split_row_blocks must be 0 or 1");
    if (!(cfg.ood_z >= 0.0) || !std::isfinite(cfg.ood_z))
        return fail(CSR_ERR_INVALID_ARG, "ood_z must be finite and >= 0");
    if (cfg.ml_partitions < 0 || cfg.ml_partitions > 4096 ||
        (cfg.ml_partitions > 0 && !(cfg.t_ml_part > 0.0)))
        return fail(CSR_ERR_INVALID_ARG, "ml_partitions must be in 0..4096 with t_ml_part > 0");
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (prev != A->device) (void)hipSetDevice(A->device);
    struct Restore {
        int prev, dev;
        ~Restore() {
            if (prev >= 0 && prev != dev) (void)hipSetDevice(prev);
        }
    } restore{prev, A->device};
    hipStream_t s = (hipStream_t)stream;
    const auto t0 = Clock::now();
    Plan P;
    csr_config_t used = cfg;  // the configuration P is realized with
    csr_plan_info_t info{};
    info.classes = -1;
    csr_status_t st = CSR_OK;
    double t_prep = 0.0;
    int32_t sel = mode;
    if (A->n_rows == 0 && sel >= CSR_SEL_PLAIN && sel <= CSR_SEL_TREE) {
        // a matrix without rows: every plan computes nothing, so the plain
        // one is kept without inspecting, timing or preprocessing anything
        if (sel == CSR_SEL_FORCED && !opts_realizable(cfg.forced_opts))
            return fail(CSR_ERR_INVALID_ARG, "unknown optimization bits");
        st = realize(A, 0, cfg, &P, s);
        sel = -1;
    }
    if (sel == CSR_SEL_TREE) {
        // features -> decision tree -> bottleneck classes -> Table II
        // remedies with default parameters (nothing timed); no tree -> the
        // profile-guided path
        if ((st = inspect(A, s)) != CSR_OK) return st;
        const int32_t cls = tree_classes(A->feat.f);
        if (cls >= 0) {
            info.classes = cls;
            const bool has_long = A->feat.f[2] > (double)long_row_tau(A, cfg);
            const auto tp = Clock::now();
            st = realize(A, remedies(cls, has_long, cfg.remedy_map), cfg, &P, s);
            t_prep = ms_since(tp);
            sel = -1;  // decided
        } else {
            info.fallback = 1;
            sel = CSR_SEL_PROFILE;
        }
    }
    switch (sel) {
    case -1:
        break;
    case CSR_SEL_PLAIN:
        st = realize(A, 0, cfg, &P, s);
        break;
    case CSR_SEL_FORCED:
        if (!opts_realizable(cfg.forced_opts))
            return fail(CSR_ERR_INVALID_ARG, "unknown optimization bits");
        st = realize(A, cfg.forced_opts, cfg, &P, s);
        break;
    case CSR_SEL_EXHAUSTIVE: {
        double best = 1e300;
        int best_k = 0;
        const int calls = cfg.timing_calls > 0 ? cfg.timing_calls : 32;
        // the catalogue lists the baseline and the singles first
        const int n_sets = cfg.exhaustive_set == 1 ? 6 : 16;
        if (cfg.exhaustive_set != 0 && cfg.exhaustive_set != 1) {
            st = fail(CSR_ERR_INVALID_ARG, "exhaustive_set must be 0 or 1");
            break;
        }
        for (int k = 0; k < n_sets && st == CSR_OK; ++k) {
            Plan Q;
            if ((st = realize(A, kCatalogue[k], cfg, &Q, s)) != CSR_OK) break;
            double ms = 0;
            if ((st = time_plan(A, Q, calls, 3, s, &ms)) != CSR_OK) break;
            if (ms < best) {
                best = ms;
                best_k = k;
            }
        }
        if (st == CSR_OK) st = realize(A, kCatalogue[best_k], cfg, &P, s);  // its tables in place
        break;
    }
    case CSR_SEL_LEARNED: {
        // features -> MLP -> catalogue variant with default parameters; no
        // model, non-finite features, or features outside the model's
        // training range -> the profile-guided path
        if ((st = inspect(A, s)) != CSR_OK) break;
        int32_t v = -1;
        st = learned_pick(A, s, cfg.ood_z, &v, &info.feature_z_max);
        if (st == CSR_OK && v >= 0 && v < 16) {
            const auto tp = Clock::now();
            st = realize(A, kCatalogue[v], cfg, &P, s);
            t_prep = ms_since(tp);
            break;
        }
        if (st != CSR_ERR_NOT_READY && st != CSR_OK) break;
        st = CSR_OK;
        info.fallback = 1;  // fell back to PROFILE
    }
        [[fallthrough]];
    case CSR_SEL_PROFILE: {
        Bounds B{};
        if ((st = measure_bounds(A, cfg, s, &B)) != CSR_OK) break;
        if (!A->has_features && (st = inspect(A, s)) != CSR_OK) break;
        int32_t cls = classify(B.p_csr, B.p_mb, B.p_ml, B.p_imb, B.p_cmp, B.p_peak, cfg);
        if (B.ml_flagged > 0) cls |= CSR_CLS_ML;  // partition-aware ML
        const bool has_long = A->feat.f[2] > (double)long_row_tau(A, cfg);
        const int32_t opts = remedies(cls, has_long, cfg.remedy_map);
        info.classes = cls;
        info.p_csr = B.p_csr;
        info.p_mb = B.p_mb;
        info.p_ml = B.p_ml;
        info.p_imb = B.p_imb;
        info.p_cmp = B.p_cmp;
        info.p_peak = B.p_peak;
        info.b_max = B.b_max;
        info.ml_partitions = B.ml_parts;
        info.ml_parts_flagged = B.ml_flagged;
        info.ml_part_max = B.ml_part_max;
        const auto tp = Clock::now();
        if (cfg.autotune) st = autotune(A, opts, cfg, s, &P, &used);
        else st = realize(A, opts, cfg, &P, s);
        t_prep = ms_since(tp);
        break;
    }
    default:
        return fail(CSR_ERR_UNSUPPORTED, "selection mode not available");
    }
    if (st != CSR_OK) {
        restore_plan(A, s);
        return st;
    }
    CSR_HIP(hipStreamSynchronize(s));
    A->plan = P;
    A->plan_cfg = used;
    A->version += 1;
    const int32_t fell_back = info.fallback;
    fill_info(A, P, &info);
    info.fallback = fell_back;
    info.t_select_ms = ms_since(t0) - t_prep;
    info.t_prep_ms = t_prep;
    A->info = info;
    if (out) *out = info;
    return CSR_OK;
}

csr_status_t csr_classify(const double *p, const csr_config_t *cfg_in, int32_t has_long_rows,
                          int32_t *classes, int32_t *opts) {
    if (!p || !classes || !opts) return fail(CSR_ERR_INVALID_ARG, "NULL argument");
    for (int k = 0; k < 6; ++k)
        if (!(p[k] > 0.0) || !std::isfinite(p[k]))
            return fail(CSR_ERR_INVALID_ARG, "bounds must be finite and positive");
    csr_config_t cfg;
    if (cfg_in) cfg = *cfg_in;
    else csr_config_default(&cfg);
    if (cfg.remedy_map != 0 && cfg.remedy_map != 1)
        return fail(CSR_ERR_INVALID_ARG, "remedy_map must be 0 or 1");
    *classes = classify(p[0], p[1], p[2], p[3], p[4], p[5], cfg);
    *opts = remedies(*classes, has_long_rows != 0, cfg.remedy_map);
    return CSR_OK;
}

csr_status_t csr_device_bandwidth(double *hbm, double *cache, void *stream) {
    if (!hbm || !cache) return fail(CSR_ERR_INVALID_ARG, "NULL argument");
    int dev = 0;
    CSR_HIP(hipGetDevice(&dev));
    return device_bandwidth(dev, (hipStream_t)stream, hbm, cache);
}

csr_status_t csr_debug_probe(csr_matrix_t A, int32_t which, const void *d_x, void *d_y,
                             void *stream) {
    if (!A || (which != 1 && which != 2) || (!d_x && A->n_cols > 0) || (!d_y && A->n_rows > 0))
        return fail(CSR_ERR_INVALID_ARG, "bad probe arguments");
    if (A->n_rows == 0) return CSR_OK;
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (prev != A->device) (void)hipSetDevice(A->device);
    hipStream_t s = (hipStream_t)stream;
    const double nnz_avg = (double)A->nnz / A->n_rows;
    csr_status_t st = which == 1 ? ensure_row_index(A, s) : CSR_OK;
    if (st == CSR_OK) {
        const hipError_t e = launch_probe(A, default_lanes_per_row(nnz_avg), which, d_x, d_y, s);
        if (e != hipSuccess) st = hip_fail(e, "probe");
    }
    if (prev >= 0 && prev != A->device) (void)hipSetDevice(prev);
    return st;
}

}  // extern "C"
