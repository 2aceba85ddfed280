// Constant-time size model (Section 4.1).
//
// The paper fits SSRS = round(a_s - b_s ln r) and SRS = round(a_r - b_r ln r)
// by logarithmic regression over the best sizes of a sweep, rounds to nearest
// with halves toward +infinity, then adjusts the sizes per row-density case
// (r <= 8, <= 16, <= 32, > 32) to account for its block shapes.  The VOLTA and
// AMPERE models below are the paper's constants and adjustments; MI355X is
// this library's fit of the same form for its gfx950 kernels (one
// super-super-row per workgroup, one super-row per wavefront), refitted from
// measured sweeps.
#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "host.hpp"

namespace csrk {

namespace {

int64_t round_half_up(double v) { return static_cast<int64_t>(std::floor(v + 0.5)); }

int case_of(double r) {
    if (r <= 8) return 1;
    if (r <= 16) return 2;
    if (r <= 32) return 3;
    return 4;
}

// MI355X fit of the same logarithmic form, from the autotuner's sweep of
// SRS in {16..128} x SSRS in {2, 4, 8} x lanes per row in {1, 2, 4} over
// eight stencil matrices with rdensity 5 to 26.5, FP64 and FP32 storage,
// timing the forward product followed by its adjoint.  The best SRS falls
// with rdensity; the best SSRS shows no trend (the fit is flat near 2).  One
// super-row per wavefront was best on every matrix, so a workgroup has SSRS
// wavefronts, and SSRS is snapped to a power of two (workgroups of 3 or 6
// wavefronts measured 5-8% slower).
constexpr double kMiSsrsA = 2.294, kMiSsrsB = -0.0357;
constexpr double kMiSrsA = 124.21, kMiSrsB = 32.80;

// Nearest power of two, ties toward the smaller.
int64_t nearest_pow2(int64_t v) {
    if (v <= 1) return 1;
    int64_t lo = 1;
    while (lo * 2 <= v) lo *= 2;
    return (v - lo <= 2 * lo - v) ? lo : 2 * lo;
}

// Nearest size of the sweep's {2^i, 3 * 2^(i-1)} set (1, 2, 3, 4, 6, 8, 12,
// ...), ties toward the smaller, but at least `floor`.  The model is fitted on
// those sizes only; off-set sizes between them measured up to 6% slower on
// stencil matrices (a super-row of 57 or 61 rows against 48 or 64 on the
// 128^3 7-point grid), so the fitted value is snapped back onto the set.
int64_t snap_srs(int64_t v, int64_t floor) {
    int64_t best = 1, up = -1;
    for (int64_t p = 1; p <= (int64_t(1) << 40); p *= 2) {
        for (int64_t c : {p, 3 * p / 2}) {  // ascending, so ties keep the smaller
            if (std::llabs(c - v) < std::llabs(best - v)) best = c;
            if (up < 0 && c >= floor) up = c;
        }
        if (p > 2 * v && p > floor) break;
    }
    return best >= floor ? best : up;
}

int32_t clamp_size(int64_t v, int64_t hi) { return static_cast<int32_t>(std::max<int64_t>(1, std::min(v, hi))); }

}  // namespace

csrk_status tune(int64_t n, int64_t nnz, csrk_model model, csrk_params *out) {
    if (!out || n <= 0 || nnz <= 0) return CSRK_ERR_ARG;
    if (model == CSRK_MODEL_HOST_CPU) {
        // Section 4.2: on CPUs CSR-2 is preferred and the best SRS does not
        // follow the matrix's simple statistics; a geometric mean of the
        // per-matrix optima, 96, is the constant-time choice.  ssrs = 1 makes
        // every super-row a unit of the host kernel's parallel loop.
        *out = csrk_params{2, 96, 1, 1, 4, CSRK_REORDER_BANDK};
        return CSRK_OK;
    }
    const double r = double(nnz) / double(n);
    const double lr = std::log(r);
    const int c = case_of(r);
    int64_t ssrs, srs;
    csrk_params p{};
    p.k = 3;
    p.reorder = CSRK_REORDER_BANDK;
    switch (model) {
    case CSRK_MODEL_VOLTA:
        ssrs = round_half_up(8.900 - 1.25 * lr);
        srs = round_half_up(10.146 - 1.50 * lr);
        if (c == 2) {
            ssrs = round_half_up(double(ssrs) * 1.5);
            srs = ssrs * 2;
        } else if (c == 3) {
            ssrs = ssrs * 4;
            srs = ssrs / 2 - ((ssrs % 2 != 0 && ssrs < 0) ? 1 : 0);
        } else if (c == 4) {
            ssrs = ssrs * 5;
            srs = ssrs / 2 - ((ssrs % 2 != 0 && ssrs < 0) ? 1 : 0);
        }
        break;
    case CSRK_MODEL_AMPERE:
        ssrs = round_half_up(9.175 - 1.32 * lr);
        srs = round_half_up(20.500 - 3.50 * lr);
        if (c == 2) {
            srs = ssrs * 4;
        } else if (c == 3) {
            ssrs = round_half_up(double(ssrs) * 2.5);
            srs = ssrs * 3;
        } else if (c == 4) {
            ssrs = ssrs * 2;
            srs = ssrs * 2;
        }
        break;
    case CSRK_MODEL_MI355X:
        ssrs = nearest_pow2(round_half_up(kMiSsrsA - kMiSsrsB * lr));
        // The fit turns negative past rdensity ~87 (the paper flattens its own
        // fits by hand there); keep a super-row at least half a staging window.
        srs = snap_srs(round_half_up(kMiSrsA - kMiSrsB * lr), static_cast<int64_t>(std::ceil(256.0 / r)));
        break;
    default:
        return CSRK_ERR_ARG;
    }
    p.ssrs = clamp_size(ssrs, model == CSRK_MODEL_MI355X ? 16 : INT32_MAX);
    p.srs = clamp_size(srs, INT32_MAX);
    // Lanes that reduce one row: a row per lane while rows are short, wider
    // groups as rows lengthen (the paper switches to an in-row parallel kernel
    // above 8 nonzeros per row, Section 3; the sweep put the switches near 6
    // and 24).
    p.lanes_per_row = r <= 6 ? 1 : r <= 24 ? 2 : r <= 48 ? 4 : r <= 96 ? 8 : 16;
    p.waves_per_wg = model == CSRK_MODEL_MI355X ? p.ssrs : 4;
    *out = p;
    return CSRK_OK;
}

csrk_status tune_rhs(int64_t n, int64_t nnz, int32_t nrhs, csrk_model model, csrk_params *out) {
    if (nrhs < 1) return CSRK_ERR_ARG;
    const csrk_status s = tune(n, nnz, model, out);
    if (s != CSRK_OK || model != CSRK_MODEL_MI355X || nrhs == 1) return s;
    // Blocks of right-hand sides (the batched autotuner's sweep on 64 3D
    // 7-point matrices with 8 columns, one workgroup per work item: SRS
    // {16, 24, 32, 48, 64} x SSRS {2, 4, 8}): a row moves nrhs times the
    // vector bytes, and the best super-row held half the rows of the
    // one-column choice (32 against 64; 1.24 ms per forward + adjoint step
    // against 1.34 ms), with 4 super-rows (and wavefronts) per workgroup.
    out->srs = static_cast<int32_t>(snap_srs(std::max<int64_t>(1, out->srs / 2), 1));
    out->ssrs = out->waves_per_wg = 4;
    return CSRK_OK;
}

void check_params(const csrk_params &p) {
    if (p.k < 2 || p.k > kMaxK) throw Error{CSRK_ERR_ARG, "k must be in 2..8"};
    if (p.srs < 1 || p.ssrs < 1) throw Error{CSRK_ERR_ARG, "srs and ssrs must be >= 1"};
    const int L = p.lanes_per_row;
    if (L < 1 || L > 64 || (L & (L - 1))) throw Error{CSRK_ERR_ARG, "lanes_per_row must be a power of two in 1..64"};
    if (p.waves_per_wg < 1 || p.waves_per_wg > 16) throw Error{CSRK_ERR_ARG, "waves_per_wg must be in 1..16"};
    if (p.reorder < CSRK_REORDER_BANDK || p.reorder > CSRK_REORDER_NONE) throw Error{CSRK_ERR_ARG, "unknown reorder"};
}

}  // namespace csrk
