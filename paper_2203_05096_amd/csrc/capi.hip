// C ABI of the CSR-k library (include/csrk.h): handles, argument checks,
// status mapping, device upload and kernel dispatch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <initializer_list>
#include <mutex>
#include <cstdlib>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/csrk.h"
#include "device/launch.hpp"
#include "host/host.hpp"

using csrk::Error;

struct csrk_matrix {
    int32_t n = 0;
    int64_t nnz = 0;
    csrk_params params{};
    std::vector<int32_t> perm, row_ptr, col_idx, sr_ptr, ssr_ptr;
    std::vector<std::vector<int32_t>> upper_ptr;  // grouping levels 3 .. k-1 (k >= 4)
    std::vector<int64_t> vmap;
    std::vector<double> vals;
    csrk::Stats in_stats, out_stats;
    int32_t max_sr_nnz = 0, max_ssr_rows = 0;
    csrk::Transposed trans;  // index structure of A'^T for the adjoint
    csrk::UnionIndex uni;    // union pattern A' + A'^T of a nonsymmetric A' (ok == false otherwise)
    // device side
    bool on_device = false;
    csrk_dtype store = CSRK_F64;
    int device = -1;
    int32_t *d_row_ptr = nullptr, *d_col_idx = nullptr, *d_sr_ptr = nullptr, *d_ssr_ptr = nullptr, *d_perm = nullptr;
    int32_t *d_t_row_ptr = nullptr, *d_t_col = nullptr, *d_t_src = nullptr;  // t_row_ptr/t_col only if nonsymmetric
    void *d_vals = nullptr;
    void *d_vals_t = nullptr;  // stored values in A'^T order, for the adjoint
    // rows of A' / A'^T longer than csrk::dev::kLongRow (t_ only if nonsymmetric)
    std::vector<int32_t> long_rows, t_long_rows;
    int32_t *d_long = nullptr, *d_t_long = nullptr;
    csrk::dev::SrRec *d_srec = nullptr;    // super-row records (see csrk::dev::SrRec)
    csrk::dev::SrRec *d_srec_t = nullptr;  // records of the same rows of A'^T (nonsymmetric patterns)
    int32_t srec_stride = 0;
    csrk::dev::XcdSplit split_fwd, split_adj;  // SSR ranges per XCD (set at upload)
    bool values_symmetric = false;  // A' == A'^T exactly: d_vals_t aliases d_vals
    int32_t max_row_any = 0;        // longest row of A' or of A'^T
    // union pattern of a nonsymmetric A' (csrk::union_index), for the one-pass adjoint
    int32_t *d_u_col = nullptr, *d_u_src = nullptr, *d_erow_ptr = nullptr;
    void *d_u_vals = nullptr;
    csrk::dev::SrRec *d_srec_u = nullptr;
    int64_t nu = 0;
};

struct csrk_batch_s {
    std::vector<csrk_handle> handles;
    csrk_dtype store = CSRK_F64;
    int device = -1;
    int32_t nitems = 0, max_n = 0;
    int2 *d_items = nullptr;
    csrk::dev::SrRec *d_brec = nullptr;  // per item, brec_stride super-row records of its SSR
    csrk::dev::SrRec *d_brec_u = nullptr;  // the same slots' union-pattern records (matrices that have one)
    int32_t brec_stride = 1;
    // Descriptor tables on the device (forward, adjoint) and the host copies
    // they were written from; a call re-uploads only when its pointers change.
    csrk::dev::MatDesc *d_descs[2] = {nullptr, nullptr};
    std::vector<csrk::dev::MatDesc> last[2];
    bool last_valid[2] = {false, false};
    csrk::dev::Shape shape;
    int cus = 0;
    int blocks_per_cu = 0;  // 0: one workgroup per work item (batch_grid)
    bool all_sym = true;    // every handle's pattern is symmetric
};

namespace {

thread_local std::string g_detail;

void set_detail(const std::string &s) { g_detail = s; }

template <typename F>
csrk_status guard(F &&f) {
    try {
        g_detail.clear();
        return f();
    } catch (const Error &e) {
        set_detail(e.detail);
        return e.status;
    } catch (const std::bad_alloc &) {
        set_detail("host allocation failed");
        return CSRK_ERR_ALLOC;
    } catch (const std::exception &e) {
        set_detail(e.what());
        return CSRK_ERR_ARG;
    }
}

void hip_check(hipError_t e, const char *what) {
    if (e == hipSuccess) return;
    if (e == hipErrorOutOfMemory) throw Error{CSRK_ERR_ALLOC, std::string(what) + ": " + hipGetErrorString(e)};
    throw Error{CSRK_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e)};
}

size_t dtype_bytes(csrk_dtype d) { return d == CSRK_F64 ? 8 : d == CSRK_F32 ? 4 : 2; }

// Makes the handle's device current for the scope of a call.
struct DeviceScope {
    int prev = -1;
    explicit DeviceScope(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (dev >= 0 && dev != prev) hip_check(hipSetDevice(dev), "hipSetDevice");
    }
    ~DeviceScope() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

void free_device(csrk_matrix *h) {
    if (!h->on_device) return;
    DeviceScope ds(h->device);
    for (void *p : {(void *)h->d_row_ptr, (void *)h->d_col_idx, (void *)h->d_sr_ptr, (void *)h->d_ssr_ptr,
                    (void *)h->d_perm, (void *)h->d_t_row_ptr, (void *)h->d_t_col, (void *)h->d_t_src, h->d_vals,
                    h->d_vals_t == h->d_vals ? nullptr : h->d_vals_t, (void *)h->d_long, (void *)h->d_t_long,
                    (void *)h->d_srec, (void *)h->d_srec_t, (void *)h->d_u_col, (void *)h->d_u_src,
                    (void *)h->d_erow_ptr, h->d_u_vals, (void *)h->d_srec_u})
        if (p) (void)hipFree(p);
    h->d_u_col = h->d_u_src = h->d_erow_ptr = nullptr;
    h->d_u_vals = nullptr;
    h->d_srec_u = nullptr;
    h->nu = 0;
    h->d_row_ptr = h->d_col_idx = h->d_sr_ptr = h->d_ssr_ptr = h->d_perm = nullptr;
    h->d_t_row_ptr = h->d_t_col = h->d_t_src = nullptr;
    h->d_long = h->d_t_long = nullptr;
    h->d_srec = h->d_srec_t = nullptr;
    h->d_vals = h->d_vals_t = nullptr;
    h->on_device = false;
}

template <typename T>
T *upload_array(const std::vector<T> &v, const char *what) {
    T *d = nullptr;
    hip_check(hipMalloc(&d, std::max<size_t>(1, v.size()) * sizeof(T)), what);
    if (!v.empty()) {
        hipError_t e = hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(d);
            hip_check(e, what);
        }
    }
    return d;
}

void finish_host(csrk_matrix *h, const int32_t *row_ptr, const int32_t *col_idx, const double *vals,
                 csrk::Grouping &&gr) {
    csrk::Permuted pm = csrk::permute(h->n, row_ptr, col_idx, vals, gr.perm);
    h->perm = std::move(gr.perm);
    h->sr_ptr = std::move(gr.sr_ptr);
    h->ssr_ptr = std::move(gr.ssr_ptr);
    h->upper_ptr = std::move(gr.upper);
    h->row_ptr = std::move(pm.row_ptr);
    h->col_idx = std::move(pm.col_idx);
    h->vals = std::move(pm.vals);
    h->vmap = std::move(pm.vmap);
    h->in_stats = csrk::row_stats(h->n, row_ptr, col_idx, false);
    h->out_stats = csrk::row_stats(h->n, h->row_ptr.data(), h->col_idx.data(), true);
    h->max_sr_nnz = 0;
    for (size_t s = 0; s + 1 < h->sr_ptr.size(); ++s)
        h->max_sr_nnz = std::max(h->max_sr_nnz, h->row_ptr[h->sr_ptr[s + 1]] - h->row_ptr[h->sr_ptr[s]]);
    h->max_ssr_rows = 0;
    for (size_t t = 0; t + 1 < h->ssr_ptr.size(); ++t)
        h->max_ssr_rows = std::max(h->max_ssr_rows, h->sr_ptr[h->ssr_ptr[t + 1]] - h->sr_ptr[h->ssr_ptr[t]]);
    h->trans = csrk::transpose_index(h->n, h->row_ptr, h->col_idx);
    h->uni = csrk::union_index(h->n, h->row_ptr, h->col_idx, h->sr_ptr, h->trans, csrk::dev::kUnionRows,
                               csrk::dev::kUnionWindow);
    h->max_row_any = 0;
    for (int32_t i = 0; i < h->n; ++i) {
        h->max_row_any = std::max(h->max_row_any, h->row_ptr[size_t(i) + 1] - h->row_ptr[size_t(i)]);
        if (!h->trans.symmetric)
            h->max_row_any =
                std::max(h->max_row_any, h->trans.t_row_ptr[size_t(i) + 1] - h->trans.t_row_ptr[size_t(i)]);
    }
}

// The host keeps an FP64 master copy of the values.  FP32 and BF16 input
// values widen to FP64 exactly, so converting back to the input's own type at
// upload returns the caller's bits.  Returns a pointer to FP64 values (the
// input itself when it already is FP64; NULL for a pattern-only build).
const double *values_as_f64(const void *vals, csrk_dtype in, int64_t nnz, std::vector<double> &buf) {
    if (in != CSRK_F64 && in != CSRK_F32 && in != CSRK_BF16) throw Error{CSRK_ERR_ARG, "unknown input dtype"};
    if (!vals) return nullptr;
    if (in == CSRK_F64) return static_cast<const double *>(vals);
    buf.resize(size_t(nnz));
    if (in == CSRK_F32) {
        const float *f = static_cast<const float *>(vals);
        for (int64_t k = 0; k < nnz; ++k) buf[size_t(k)] = double(f[k]);
    } else {
        const uint16_t *b = static_cast<const uint16_t *>(vals);
        for (int64_t k = 0; k < nnz; ++k) {
            const uint32_t u = uint32_t(b[k]) << 16;
            float f;
            std::memcpy(&f, &u, sizeof(f));
            buf[size_t(k)] = double(f);
        }
    }
    return buf.data();
}

csrk_params resolve_params(int32_t n, int64_t nnz, const csrk_params *p) {
    csrk_params q{};
    if (p) {
        q = *p;
    } else {
        if (n == 0 || nnz == 0) {
            q = csrk_params{3, 1, 1, 1, 4, CSRK_REORDER_BANDK};
        } else if (csrk::tune(n, nnz, CSRK_MODEL_MI355X, &q) != CSRK_OK) {
            throw Error{CSRK_ERR_ARG, "tuning failed"};
        }
    }
    csrk::check_params(q);
    return q;
}

csrk::dev::Arrays arrays_of(const csrk_matrix *h) {
    csrk::dev::Arrays a;
    a.n = h->n;
    a.nnz = h->nnz;
    a.nsr = static_cast<int32_t>(h->sr_ptr.size()) - 1;
    a.nssr = static_cast<int32_t>(h->ssr_ptr.size()) - 1;
    a.row_ptr = h->d_row_ptr;
    a.col_idx = h->d_col_idx;
    a.sr_ptr = h->d_sr_ptr;
    a.ssr_ptr = h->d_ssr_ptr;
    a.perm = h->d_perm;
    const bool sym = h->trans.symmetric;
    a.t_row_ptr = sym ? h->d_row_ptr : h->d_t_row_ptr;
    a.t_col = sym ? h->d_col_idx : h->d_t_col;
    a.t_src = h->d_t_src;
    a.vals_t = h->d_vals_t;
    a.sym = sym;
    a.long_rows = h->d_long;
    a.nlong = static_cast<int32_t>(h->long_rows.size());
    a.t_long_rows = sym ? h->d_long : h->d_t_long;
    a.t_nlong = static_cast<int32_t>(sym ? h->long_rows.size() : h->t_long_rows.size());
    a.split_fwd = h->split_fwd;
    a.split_adj = h->split_adj;
    a.max_row = h->max_row_any;
    a.srec = h->d_srec;
    a.srec_t = sym ? h->d_srec : h->d_srec_t;
    a.srec_stride = h->srec_stride;
    a.u_col = h->d_u_col;
    a.u_src = h->d_u_src;
    a.u_vals = h->d_u_vals;
    a.erow_ptr = h->d_erow_ptr;
    a.srec_u = h->d_srec_u;
    a.nu = h->nu;
    return a;
}

// Work-balanced XCD ranges over the super-super-rows: the cost of a row is
// its nonzeros (0 for rows longer than kLongRow, which run elsewhere) plus 1,
// summed over row_ptr and, when given, a second row pointer array (the
// adjoint's transposed rows).  Range x ends at the first SSR whose prefix cost
// reaches x/8 of the total.
csrk::dev::XcdSplit xcd_split(const csrk_matrix *h, const std::vector<int32_t> &rp,
                              const std::vector<int32_t> *rp2) {
    using csrk::dev::kXcds;
    const int64_t nssr = int64_t(h->ssr_ptr.size()) - 1;
    std::vector<int64_t> prefix(size_t(nssr) + 1, 0);
    auto row_cost = [](const std::vector<int32_t> &p, int32_t i) -> int64_t {
        const int64_t len = int64_t(p[i + 1]) - p[i];
        return len > csrk::dev::kLongRow ? 0 : len;
    };
    for (int64_t t = 0; t < nssr; ++t) {
        int64_t c = 0;
        for (int32_t i = h->sr_ptr[h->ssr_ptr[t]]; i < h->sr_ptr[h->ssr_ptr[t + 1]]; ++i)
            c += 1 + row_cost(rp, i) + (rp2 ? row_cost(*rp2, i) : 0);
        prefix[t + 1] = prefix[t] + c;
    }
    csrk::dev::XcdSplit sp;
    const int64_t total = prefix[nssr];
    sp.b[0] = 0;
    for (int x = 1; x < kXcds; ++x) {
        const int64_t target = (total * x + kXcds - 1) / kXcds;
        const int64_t t = std::lower_bound(prefix.begin(), prefix.end(), target) - prefix.begin();
        sp.b[x] = static_cast<int32_t>(std::max<int64_t>(sp.b[x - 1], std::min<int64_t>(t, nssr)));
    }
    sp.b[kXcds] = static_cast<int32_t>(nssr);
    for (int x = 0; x < kXcds; ++x) sp.width = std::max(sp.width, sp.b[x + 1] - sp.b[x]);
    return sp;
}

// Rows whose length (from a row pointer array) exceeds kLongRow, ascending.
std::vector<int32_t> long_rows_of(const std::vector<int32_t> &rp) {
    std::vector<int32_t> out;
    for (size_t i = 0; i + 1 < rp.size(); ++i)
        if (rp[i + 1] - rp[i] > csrk::dev::kLongRow) out.push_back(static_cast<int32_t>(i));
    return out;
}

void need_device(const csrk_matrix *h) {
    if (!h) throw Error{CSRK_ERR_ARG, "null handle"};
    if (!h->on_device) throw Error{CSRK_ERR_UNSUPPORTED, "handle has no device arrays (call csrk_upload)"};
}

void check_vec(const void *p, const csrk_matrix *h, const char *name) {
    if (h->n > 0 && !p) throw Error{CSRK_ERR_ARG, std::string(name) + " is NULL"};
}

void check_align16(const void *p, const char *name) {
    if (reinterpret_cast<uintptr_t>(p) % 16 != 0) throw Error{CSRK_ERR_ARG, std::string(name) + " must be 16-byte aligned"};
}

const void *values_for(const csrk_matrix *h, const void *vals_dev) {
    const void *v = vals_dev ? vals_dev : h->d_vals;
    if (reinterpret_cast<uintptr_t>(v) % 16 != 0) throw Error{CSRK_ERR_ARG, "vals_dev must be 16-byte aligned"};
    return v;
}

csrk::dev::Shape shape_of(const csrk_matrix *h) {
    csrk::dev::Shape s;
    s.lanes_per_row = h->params.lanes_per_row;
    s.waves = h->params.waves_per_wg;
    return s;
}

}  // namespace

extern "C" {

const char *csrk_status_string(csrk_status s) {
    switch (s) {
    case CSRK_OK:
        return "CSRK_OK";
    case CSRK_ERR_ARG:
        return "CSRK_ERR_ARG: invalid argument";
    case CSRK_ERR_BAD_ROWPTR:
        return "CSRK_ERR_BAD_ROWPTR: malformed row_ptr";
    case CSRK_ERR_COL_RANGE:
        return "CSRK_ERR_COL_RANGE: column index out of range";
    case CSRK_ERR_DUPLICATE:
        return "CSRK_ERR_DUPLICATE: duplicate column in a row";
    case CSRK_ERR_ALLOC:
        return "CSRK_ERR_ALLOC: allocation failed";
    case CSRK_ERR_DEVICE:
        return "CSRK_ERR_DEVICE: HIP device error";
    case CSRK_ERR_UNSUPPORTED:
        return "CSRK_ERR_UNSUPPORTED: operation not supported";
    }
    return "unknown csrk_status";
}

const char *csrk_last_error_detail(void) { return g_detail.c_str(); }

csrk_status csrk_tune(int64_t n, int64_t nnz, csrk_model model, csrk_params *out) {
    return guard([&] {
        csrk_status s = csrk::tune(n, nnz, model, out);
        if (s != CSRK_OK) set_detail("csrk_tune needs n > 0, nnz > 0, a known model and an output pointer");
        return s;
    });
}

csrk_status csrk_spmv_host(csrk_handle h, const double *x, double *y, int32_t nthreads) {
    return guard([&] {
        if (!h || (!x && h->n > 0) || (!y && h->n > 0)) throw Error{CSRK_ERR_ARG, "null handle or vector"};
        csrk::spmv_host(int64_t(h->ssr_ptr.size()) - 1, h->ssr_ptr.data(), h->sr_ptr.data(), h->row_ptr.data(),
                        h->col_idx.data(), h->vals.data(), x, y, nthreads);
        return CSRK_OK;
    });
}

csrk_status csrk_tune_rhs(int64_t n, int64_t nnz, int32_t nrhs, csrk_model model, csrk_params *out) {
    return guard([&] {
        if (nrhs < 1) throw Error{CSRK_ERR_ARG, "nrhs must be >= 1"};
        csrk_status s = csrk::tune_rhs(n, nnz, nrhs, model, out);
        if (s != CSRK_OK) {
            set_detail("csrk_tune_rhs needs n > 0, nnz > 0, a known model and an output pointer");
            return s;
        }
        return CSRK_OK;
    });
}

csrk_status csrk_build_host(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                            const void *vals_in, csrk_dtype in_dtype, const csrk_params *p, csrk_handle *out) {
    return guard([&] {
        if (!out) throw Error{CSRK_ERR_ARG, "out is NULL"};
        *out = nullptr;
        csrk::validate_csr(n, nnz, row_ptr, col_idx);
        std::vector<double> widened;
        const double *vals = values_as_f64(vals_in, in_dtype, nnz, widened);
        csrk_params q = resolve_params(n, nnz, p);
        csrk::Grouping gr;
        if (q.reorder == CSRK_REORDER_BANDK && q.k >= 4) {
            std::vector<int32_t> sizes(size_t(q.k) - 1, q.ssrs);
            sizes[0] = q.srs;
            gr = csrk::bandk_levels(n, row_ptr, col_idx, sizes);
        } else if (q.reorder == CSRK_REORDER_BANDK) {
            gr = q.k == 2 ? csrk::bandk2(n, row_ptr, col_idx, q.srs, q.ssrs)
                          : csrk::bandk(n, row_ptr, col_idx, q.srs, q.ssrs);
        } else if (q.reorder == CSRK_REORDER_RCM) {
            gr = csrk::rcm_chunked(n, row_ptr, col_idx, q.srs, q.ssrs);
            csrk::chunk_upper(gr, q.k, q.ssrs);
        } else {
            std::vector<int32_t> id(n);
            std::iota(id.begin(), id.end(), 0);
            gr = csrk::chunked(std::move(id), q.srs, q.ssrs);
            csrk::chunk_upper(gr, q.k, q.ssrs);
        }
        csrk::balance(gr, row_ptr, csrk::sr_budget(n, nnz, q.srs), q.ssrs);
        auto h = new csrk_matrix();
        try {
            h->n = n;
            h->nnz = nnz;
            h->params = q;
            finish_host(h, row_ptr, col_idx, vals, std::move(gr));
        } catch (...) {
            delete h;
            throw;
        }
        *out = h;
        return CSRK_OK;
    });
}

csrk_status csrk_build_from_groups(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                                   const void *vals_in, csrk_dtype in_dtype, const int32_t *perm, int32_t nsr,
                                   const int32_t *sr_sizes, int32_t nssr, const int32_t *ssr_sizes,
                                   const csrk_params *p, csrk_handle *out) {
    return guard([&] {
        if (!out) throw Error{CSRK_ERR_ARG, "out is NULL"};
        *out = nullptr;
        csrk::validate_csr(n, nnz, row_ptr, col_idx);
        std::vector<double> widened;
        const double *vals = values_as_f64(vals_in, in_dtype, nnz, widened);
        if (n > 0 && !perm) throw Error{CSRK_ERR_ARG, "perm is NULL"};
        csrk_params q = resolve_params(n, nnz, p);
        if (q.k > 3) throw Error{CSRK_ERR_ARG, "csrk_build_from_groups takes two grouping levels: k must be 2 or 3"};
        csrk::Grouping gr = csrk::from_sizes(std::vector<int32_t>(perm, perm + n), sr_sizes, nsr, ssr_sizes, nssr);
        auto h = new csrk_matrix();
        try {
            h->n = n;
            h->nnz = nnz;
            h->params = q;
            finish_host(h, row_ptr, col_idx, vals, std::move(gr));
        } catch (...) {
            delete h;
            throw;
        }
        *out = h;
        return CSRK_OK;
    });
}

csrk_status csrk_upload(csrk_handle h, csrk_dtype store) {
    return guard([&] {
        if (!h) throw Error{CSRK_ERR_ARG, "null handle"};
        if (store != CSRK_F64 && store != CSRK_F32 && store != CSRK_BF16) throw Error{CSRK_ERR_ARG, "unknown dtype"};
        int count = 0;
        if (hipGetDeviceCount(&count) != hipSuccess || count == 0) throw Error{CSRK_ERR_DEVICE, "no HIP device"};
        free_device(h);
        int dev = 0;
        hip_check(hipGetDevice(&dev), "hipGetDevice");
        h->device = dev;
        h->store = store;
        try {
            h->d_row_ptr = upload_array(h->row_ptr, "row_ptr");
            h->d_col_idx = upload_array(h->col_idx, "col_idx");
            h->d_sr_ptr = upload_array(h->sr_ptr, "sr_ptr");
            h->d_ssr_ptr = upload_array(h->ssr_ptr, "ssr_ptr");
            h->d_perm = upload_array(h->perm, "perm");
            h->d_t_src = upload_array(h->trans.t_src, "transposed map");
            if (!h->trans.symmetric) {
                h->d_t_row_ptr = upload_array(h->trans.t_row_ptr, "transposed row_ptr");
                h->d_t_col = upload_array(h->trans.t_col, "transposed col_idx");
            }
            h->long_rows = long_rows_of(h->row_ptr);
            h->t_long_rows = h->trans.symmetric ? std::vector<int32_t>() : long_rows_of(h->trans.t_row_ptr);
            {
                // one record per (SSR, slot): the slot-th super-row's rows and entries
                const size_t nssr = h->ssr_ptr.size() - 1;
                int32_t stride = 1;
                for (size_t t = 0; t < nssr; ++t) stride = std::max(stride, h->ssr_ptr[t + 1] - h->ssr_ptr[t]);
                std::vector<csrk::dev::SrRec> rec(nssr * size_t(stride), csrk::dev::SrRec{0, 0, 0, 0});
                for (size_t t = 0; t < nssr; ++t)
                    for (int32_t s = h->ssr_ptr[t]; s < h->ssr_ptr[t + 1]; ++s) {
                        const int32_t r0 = h->sr_ptr[size_t(s)], r1 = h->sr_ptr[size_t(s) + 1];
                        rec[t * size_t(stride) + size_t(s - h->ssr_ptr[t])] =
                            csrk::dev::SrRec{r0, r1, h->row_ptr[size_t(r0)], h->row_ptr[size_t(r1)]};
                    }
                h->srec_stride = stride;
                h->d_srec = upload_array(rec, "super-row records");
                if (!h->trans.symmetric) {
                    // the same rows of A'^T: their entries in the transposed structure
                    for (auto &r : rec)
                        if (r.r0 < r.r1) {
                            r.e0 = h->trans.t_row_ptr[size_t(r.r0)];
                            r.e1 = h->trans.t_row_ptr[size_t(r.r1)];
                        }
                    h->d_srec_t = upload_array(rec, "transposed super-row records");
                    // the union pattern, when every super-row fits one staging window
                    const csrk::UnionIndex &un = h->uni;
                    if (un.ok) {
                        for (size_t t = 0; t < nssr; ++t)
                            for (int32_t s = h->ssr_ptr[t]; s < h->ssr_ptr[t + 1]; ++s) {
                                auto &r = rec[t * size_t(stride) + size_t(s - h->ssr_ptr[t])];
                                r.e0 = un.sr_begin[size_t(s)];
                                r.e1 = un.sr_end[size_t(s)];
                            }
                        h->nu = static_cast<int64_t>(un.u_col.size());
                        h->d_srec_u = upload_array(rec, "union super-row records");
                        h->d_u_col = upload_array(un.u_col, "union columns");
                        h->d_u_src = upload_array(un.u_src, "union sources");
                        h->d_erow_ptr = upload_array(un.erow_ptr, "union extras per row");
                    }
                }
            }
            if (!h->long_rows.empty()) h->d_long = upload_array(h->long_rows, "long rows");
            if (!h->t_long_rows.empty()) h->d_t_long = upload_array(h->t_long_rows, "transposed long rows");
            h->split_fwd = xcd_split(h, h->row_ptr, nullptr);
            h->split_adj = h->trans.symmetric ? h->split_fwd : xcd_split(h, h->row_ptr, &h->trans.t_row_ptr);
            // A symmetric matrix (pattern and values) is its own transpose: the
            // adjoint then reads the values the forward reads, instead of a copy.
            // (compared bit for bit: a -0.0 mirrored by a +0.0 keeps the copy)
            h->values_symmetric = h->trans.symmetric;
            for (int64_t k = 0; h->values_symmetric && k < h->nnz; ++k)
                h->values_symmetric = std::memcmp(&h->vals[size_t(k)], &h->vals[size_t(h->trans.t_src[size_t(k)])],
                                                  sizeof(double)) == 0;
            hip_check(hipMalloc(&h->d_vals, std::max<size_t>(1, size_t(h->nnz)) * dtype_bytes(store)), "vals");
            if (h->values_symmetric)
                h->d_vals_t = h->d_vals;
            else
                hip_check(hipMalloc(&h->d_vals_t, std::max<size_t>(1, size_t(h->nnz)) * dtype_bytes(store)), "vals_t");
            if (h->d_u_col)
                hip_check(hipMalloc(&h->d_u_vals, std::max<size_t>(1, size_t(h->nu)) * dtype_bytes(store)), "u_vals");
            h->on_device = true;
            if (h->nnz > 0) {
                double *tmp = upload_array(h->vals, "vals (staging)");
                hipError_t e = csrk::dev::convert_values(tmp, h->d_vals, h->nnz, store, nullptr);
                if (e == hipSuccess && !h->values_symmetric)
                    e = csrk::dev::transpose_values(arrays_of(h), store, h->d_vals, h->d_vals_t, nullptr);
                if (e == hipSuccess && h->d_u_vals)
                    e = csrk::dev::gather_values(h->d_u_src, h->nu, store, h->d_vals, h->d_u_vals, nullptr);
                hipError_t e2 = hipDeviceSynchronize();
                (void)hipFree(tmp);
                hip_check(e, "value conversion");
                hip_check(e2, "value conversion");
            }
        } catch (...) {
            h->on_device = true;
            free_device(h);
            throw;
        }
        return CSRK_OK;
    });
}

csrk_status csrk_build(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx, const void *vals,
                       csrk_dtype in_dtype, csrk_dtype store, const csrk_params *p, csrk_handle *out) {
    csrk_status s = csrk_build_host(n, nnz, row_ptr, col_idx, vals, in_dtype, p, out);
    if (s != CSRK_OK) return s;
    s = csrk_upload(*out, store);
    if (s != CSRK_OK) {
        std::string keep = g_detail;
        csrk_destroy(*out);
        *out = nullptr;
        g_detail = keep;
    }
    return s;
}

csrk_status csrk_set_launch(csrk_handle h, int32_t lanes_per_row, int32_t waves_per_wg) {
    return guard([&] {
        if (!h) throw Error{CSRK_ERR_ARG, "null handle"};
        csrk_params q = h->params;
        q.lanes_per_row = lanes_per_row;
        q.waves_per_wg = waves_per_wg;
        csrk::check_params(q);
        h->params = q;
        return CSRK_OK;
    });
}

csrk_status csrk_get_info(csrk_handle h, csrk_info *out) {
    return guard([&] {
        if (!h || !out) throw Error{CSRK_ERR_ARG, "null argument"};
        csrk_info i{};
        i.n = h->n;
        i.nnz = h->nnz;
        i.nsr = static_cast<int32_t>(h->sr_ptr.size()) - 1;
        i.nssr = static_cast<int32_t>(h->ssr_ptr.size()) - 1;
        i.rdensity = h->out_stats.rdensity;
        i.row_variance = h->out_stats.row_variance;
        i.max_row = h->out_stats.max_row;
        i.bandwidth_input = h->in_stats.bandwidth;
        i.bandwidth = h->out_stats.bandwidth;
        i.symmetry = h->out_stats.symmetry;
        i.max_sr_nnz = h->max_sr_nnz;
        i.max_ssr_rows = h->max_ssr_rows;
        i.on_device = h->on_device ? 1 : 0;
        i.store = h->store;
        i.long_rows = static_cast<int32_t>(long_rows_of(h->row_ptr).size());
        i.values_symmetric = h->on_device && h->values_symmetric ? 1 : 0;
        i.adjoint_union = h->on_device && h->d_srec_u ? 1 : 0;
        i.params = h->params;
        *out = i;
        return CSRK_OK;
    });
}

csrk_status csrk_copy_structure(csrk_handle h, int32_t *perm, int32_t *row_ptr, int32_t *col_idx, double *vals,
                                int64_t *vmap, int32_t *sr_ptr, int32_t *ssr_ptr) {
    return guard([&] {
        if (!h) throw Error{CSRK_ERR_ARG, "null handle"};
        auto cp = [](auto *dst, const auto &v) {
            if (dst && !v.empty()) std::memcpy(dst, v.data(), v.size() * sizeof(v[0]));
        };
        cp(perm, h->perm);
        cp(row_ptr, h->row_ptr);
        cp(col_idx, h->col_idx);
        cp(vals, h->vals);
        cp(vmap, h->vmap);
        cp(sr_ptr, h->sr_ptr);
        cp(ssr_ptr, h->ssr_ptr);
        return CSRK_OK;
    });
}

csrk_status csrk_level_ptr(csrk_handle h, int32_t level, int32_t *count, int32_t *out) {
    return guard([&] {
        if (!h || !count) throw Error{CSRK_ERR_ARG, "null handle or count"};
        const int32_t top = std::max(2, h->params.k - 1);
        if (level < 1 || level > top) throw Error{CSRK_ERR_ARG, "level out of range (1 .. max(2, k - 1))"};
        const std::vector<int32_t> &v =
            level == 1 ? h->sr_ptr : level == 2 ? h->ssr_ptr : h->upper_ptr[size_t(level) - 3];
        *count = static_cast<int32_t>(v.size()) - 1;
        if (out) std::memcpy(out, v.data(), v.size() * sizeof(int32_t));
        return CSRK_OK;
    });
}

csrk_status csrk_copy_union(csrk_handle h, int64_t *nu, int32_t *u_col, int32_t *u_src, int32_t *erow_ptr,
                            int32_t *sr_begin, int32_t *sr_end) {
    return guard([&] {
        if (!h || !nu) throw Error{CSRK_ERR_ARG, "null handle or nu"};
        const csrk::UnionIndex &u = h->uni;
        *nu = u.ok ? static_cast<int64_t>(u.u_col.size()) : 0;
        if (!u.ok) return CSRK_OK;
        auto cp = [](int32_t *dst, const std::vector<int32_t> &v) {
            if (dst && !v.empty()) std::memcpy(dst, v.data(), v.size() * sizeof(int32_t));
        };
        cp(u_col, u.u_col);
        cp(u_src, u.u_src);
        cp(erow_ptr, u.erow_ptr);
        cp(sr_begin, u.sr_begin);
        cp(sr_end, u.sr_end);
        return CSRK_OK;
    });
}

csrk_status csrk_device_vals(csrk_handle h, void **vals_dev) {
    return guard([&] {
        need_device(h);
        if (!vals_dev) throw Error{CSRK_ERR_ARG, "null output"};
        *vals_dev = h->d_vals;
        return CSRK_OK;
    });
}

csrk_status csrk_copy_device_vals(csrk_handle h, void *dst_dev, void *stream) {
    return guard([&] {
        need_device(h);
        if (!dst_dev && h->nnz > 0) throw Error{CSRK_ERR_ARG, "dst_dev is NULL"};
        if (h->nnz == 0) return CSRK_OK;
        DeviceScope ds(h->device);
        hip_check(hipMemcpyAsync(dst_dev, h->d_vals, size_t(h->nnz) * dtype_bytes(h->store), hipMemcpyDeviceToDevice,
                                 static_cast<hipStream_t>(stream)),
                  "csrk_copy_device_vals");
        return CSRK_OK;
    });
}

csrk_status csrk_spmv(csrk_handle h, const void *vals_dev, const void *x_dev, void *y_dev, int32_t nrhs,
                      void *stream) {
    return guard([&] {
        need_device(h);
        if (nrhs < 1) throw Error{CSRK_ERR_ARG, "nrhs must be >= 1"};
        check_vec(x_dev, h, "x");
        check_vec(y_dev, h, "y");
        if (h->n > 0 && x_dev == y_dev) throw Error{CSRK_ERR_ARG, "y must not alias x"};
        const void *v = values_for(h, vals_dev);
        DeviceScope ds(h->device);
        hip_check(csrk::dev::spmv(arrays_of(h), h->store, v, x_dev, y_dev, nrhs, shape_of(h),
                                  static_cast<hipStream_t>(stream)),
                  "csrk_spmv launch");
        return CSRK_OK;
    });
}

namespace {

// Work memory of one CG solve: r and p (FP64), q (the product's output:
// FP32 with FP32/BF16 storage), p_lo (FP32 copy of p feeding FP32/BF16
// storage), one FP64 partial sum per workgroup of the largest reduction grid,
// and the scalars.  Each array starts on a 256-byte boundary.
struct CgWork {
    double *r = nullptr, *p = nullptr;
    void *q = nullptr;
    float *p_lo = nullptr;
    double *part = nullptr, *s = nullptr;
};

size_t round256(size_t b) { return (std::max<size_t>(b, 16) + 255) / 256 * 256; }

// Bytes of CgWork for this handle, and the pointers inside base.
size_t cg_work_layout(const csrk_matrix *h, unsigned char *base, CgWork *w) {
    const size_t n = size_t(h->n);
    const bool lo = h->store != CSRK_F64;
    const int nparts = std::max(csrk::dev::kCgGrid, csrk::dev::spmv_grid(arrays_of(h)));
    const size_t sizes[6] = {n * 8, n * 8, n * (lo ? 4 : 8), lo ? n * 4 : 0, size_t(nparts) * 8, 8 * 8};
    size_t off[6], total = 0;
    for (int i = 0; i < 6; ++i) {
        off[i] = total;
        total += sizes[i] ? round256(sizes[i]) : 0;
    }
    if (base && w) {
        w->r = reinterpret_cast<double *>(base + off[0]);
        w->p = reinterpret_cast<double *>(base + off[1]);
        w->q = base + off[2];
        w->p_lo = lo ? reinterpret_cast<float *>(base + off[3]) : nullptr;
        w->part = reinterpret_cast<double *>(base + off[4]);
        w->s = reinterpret_cast<double *>(base + off[5]);
    }
    return total;
}

// Checks shared by the CG entry points.
void cg_check_args(csrk_handle h, const double *b_dev, double *x_dev, double rtol, int32_t max_iter,
                   int32_t check_every) {
    need_device(h);
    if (!b_dev || !x_dev || !(rtol > 0) || max_iter < 0 || check_every < 1)
        throw Error{CSRK_ERR_ARG, "need b, x, rtol > 0, max_iter >= 0, check_every >= 1"};
    check_vec(b_dev, h, "b");
    check_vec(x_dev, h, "x");
}

// The CG iteration on work memory w (the caller's device is current).  Every
// work array is written before it is read (r by the residual, p by its first
// update, q by the product, each partial sum by its workgroup, each scalar by
// the reduction that produces it), so w needs no clearing.
void cg_run(csrk_handle h, const double *b_dev, double *x_dev, double rtol, int32_t max_iter, int32_t check_every,
            hipStream_t st, const CgWork &w, int32_t *iters_out, double *rel_resid_out) {
    const int64_t n = h->n;
    const bool lo = h->store != CSRK_F64;  // product vectors are FP32
    const csrk::dev::Arrays a = arrays_of(h);
    const csrk::dev::Shape shp = shape_of(h);
    double *r = w.r, *p = w.p, *part = w.part, *s = w.s;
    void *q = w.q;
    float *p_lo = w.p_lo;
    auto spmv = [&](const void *in) {
        hip_check(csrk::dev::spmv(a, h->store, h->d_vals, in, q, 1, shp, st), "cg product");
    };
    // r = b - A x0, p = r, rr = r . r, bb = b . b
    if (lo) hip_check(csrk::dev::cg_round(x_dev, p_lo, n, st), "cg round");
    spmv(lo ? static_cast<const void *>(p_lo) : static_cast<const void *>(x_dev));
    hip_check(csrk::dev::cg_residual(b_dev, q, lo, r, n, part, s, st), "cg residual");
    hip_check(csrk::dev::cg_norm2(b_dev, n, part, s, st), "cg norm");
    hip_check(csrk::dev::cg_set_p(r, p, p_lo, s, n, false, st), "cg p");
    double host_s[6] = {0, 0, 0, 0, 0, 0};
    auto read_scalars = [&]() {
        hip_check(hipMemcpyAsync(host_s, s, sizeof(host_s), hipMemcpyDeviceToHost, st), "cg read");
        hip_check(hipStreamSynchronize(st), "cg sync");
    };
    read_scalars();
    const double bnorm = std::sqrt(host_s[5]);
    const double target = rtol * (bnorm > 0 ? bnorm : 1.0);
    int32_t it = 0;
    bool done = std::sqrt(host_s[0]) <= target;
    // Per iteration: q = A p with p . q summed per workgroup of the product
    // (no separate pass over p and q), alpha; r -= alpha q with r . r, beta;
    // then x += alpha p and p = r + beta p in one pass over p.
    while (!done && it < max_iter) {
        hip_check(csrk::dev::spmv_dot(a, h->store, h->d_vals,
                                      lo ? static_cast<const void *>(p_lo) : static_cast<const void *>(p), q, p,
                                      part, shp, st),
                  "cg product");
        hip_check(csrk::dev::cg_alpha_parts(part, csrk::dev::spmv_grid(a), s, st), "cg alpha");
        hip_check(csrk::dev::cg_update_r(r, q, lo, n, part, s, st), "cg residual update");
        hip_check(csrk::dev::cg_update_xp(x_dev, p, p_lo, r, s, n, st), "cg x and p update");
        ++it;
        if (it % check_every == 0 || it == max_iter) {
            read_scalars();
            if (!(host_s[1] > 0) || !std::isfinite(host_s[0]))
                throw Error{CSRK_ERR_UNSUPPORTED,
                            "CG breakdown (p'Ap <= 0 or a non-finite residual): the matrix is not symmetric "
                            "positive definite in the stored precision"};
            done = std::sqrt(host_s[0]) <= target;
        }
    }
    if (iters_out) *iters_out = it;
    if (rel_resid_out) *rel_resid_out = std::sqrt(host_s[0]) / (bnorm > 0 ? bnorm : 1.0);
    hip_check(hipStreamSynchronize(st), "cg sync");
}

// Device work memory of one csrk_cg call, freed on every exit path.
struct CgAlloc {
    void *ptr = nullptr;
    ~CgAlloc() {
        if (ptr) (void)hipFree(ptr);
    }
};

// Work memory of csrk_cg_noalloc: one array per device, held until the
// process ends.  In host code `scratch` only names the symbol; its device
// address comes from hipGetSymbolAddress, once per device, with that device
// current.
constexpr size_t kCgScratchBytes = size_t(CSRK_CG_NOALLOC_BYTES);
__device__ __align__(256) unsigned char scratch[kCgScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_dev[kMaxDevices] = {};

unsigned char *scratch_on(int device) {
    if (device < 0 || device >= kMaxDevices) throw Error{CSRK_ERR_DEVICE, "device index out of range"};
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[device]) {
        void *ptr = nullptr;
        hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "csrk_cg_noalloc scratch address");
        if (!ptr) throw Error{CSRK_ERR_DEVICE, "csrk_cg_noalloc: no device address for the scratch array"};
        g_scratch_dev[device] = static_cast<unsigned char *>(ptr);
    }
    return g_scratch_dev[device];
}

}  // namespace

csrk_status csrk_cg(csrk_handle h, const double *b_dev, double *x_dev, double rtol, int32_t max_iter,
                    int32_t check_every, void *stream, int32_t *iters_out, double *rel_resid_out) {
    return guard([&] {
        cg_check_args(h, b_dev, x_dev, rtol, max_iter, check_every);
        DeviceScope ds(h->device);
        const size_t bytes = cg_work_layout(h, nullptr, nullptr);
        CgAlloc mem;
        hip_check(hipMalloc(&mem.ptr, bytes), "cg work vectors");
        CgWork w;
        cg_work_layout(h, static_cast<unsigned char *>(mem.ptr), &w);
        cg_run(h, b_dev, x_dev, rtol, max_iter, check_every, static_cast<hipStream_t>(stream), w, iters_out,
               rel_resid_out);
        return CSRK_OK;
    });
}

csrk_status csrk_cg_noalloc_bytes(csrk_handle h, int64_t *bytes_out) {
    return guard([&] {
        if (!h || !bytes_out) throw Error{CSRK_ERR_ARG, "null argument"};
        need_device(h);
        *bytes_out = static_cast<int64_t>(cg_work_layout(h, nullptr, nullptr));
        return CSRK_OK;
    });
}

csrk_status csrk_cg_noalloc(csrk_handle h, const double *b_dev, double *x_dev, double rtol, int32_t max_iter,
                            int32_t check_every, void *stream, int32_t *iters_out, double *rel_resid_out) {
    return guard([&] {
        cg_check_args(h, b_dev, x_dev, rtol, max_iter, check_every);
        const size_t bytes = cg_work_layout(h, nullptr, nullptr);
        if (bytes > kCgScratchBytes)
            throw Error{CSRK_ERR_ARG, "csrk_cg_noalloc: the solve needs " + std::to_string(bytes) +
                                          " bytes of work memory, more than its fixed " +
                                          std::to_string(kCgScratchBytes) + "-byte array; use csrk_cg"};
        DeviceScope ds(h->device);
        CgWork w;
        cg_work_layout(h, scratch_on(h->device), &w);
        cg_run(h, b_dev, x_dev, rtol, max_iter, check_every, static_cast<hipStream_t>(stream), w, iters_out,
               rel_resid_out);
        return CSRK_OK;
    });
}

csrk_status csrk_spmv_plain(csrk_handle h, const void *vals_dev, const void *x_dev, void *y_dev, int32_t nrhs,
                            void *stream) {
    return guard([&] {
        need_device(h);
        if (nrhs < 1) throw Error{CSRK_ERR_ARG, "nrhs must be >= 1"};
        check_vec(x_dev, h, "x");
        check_vec(y_dev, h, "y");
        if (h->n > 0 && x_dev == y_dev) throw Error{CSRK_ERR_ARG, "y must not alias x"};
        const void *v = values_for(h, vals_dev);
        DeviceScope ds(h->device);
        hip_check(csrk::dev::spmv_plain(arrays_of(h), h->store, v, x_dev, y_dev, nrhs, shape_of(h),
                                        static_cast<hipStream_t>(stream)),
                  "csrk_spmv_plain launch");
        return CSRK_OK;
    });
}

csrk_status csrk_spmv_adjoint(csrk_handle h, const void *vals_dev, const void *x_dev, const void *g_dev,
                              void *grad_x_dev, void *grad_vals_dev, int32_t nrhs, void *stream) {
    return guard([&] {
        need_device(h);
        if (nrhs < 1) throw Error{CSRK_ERR_ARG, "nrhs must be >= 1"};
        check_vec(g_dev, h, "g");
        if (grad_vals_dev) check_vec(x_dev, h, "x");
        if (!grad_x_dev && !grad_vals_dev) return CSRK_OK;
        if (grad_x_dev && h->n > 0 && (grad_x_dev == g_dev || grad_x_dev == x_dev))
            throw Error{CSRK_ERR_ARG, "grad_x must not alias x or g"};
        if (grad_vals_dev) check_align16(grad_vals_dev, "grad_vals");
        if (vals_dev) check_align16(vals_dev, "vals_dev");
        DeviceScope ds(h->device);
        hip_check(csrk::dev::adjoint(arrays_of(h), h->store, vals_dev, x_dev, g_dev, grad_x_dev, grad_vals_dev, nrhs,
                                     shape_of(h), static_cast<hipStream_t>(stream)),
                  "csrk_spmv_adjoint launch");
        return CSRK_OK;
    });
}

csrk_status csrk_permute(csrk_handle h, int32_t direction, const void *in_dev, void *out_dev, int32_t nrhs,
                         int32_t elem_bytes, void *stream) {
    return guard([&] {
        need_device(h);
        if (direction != 0 && direction != 1) throw Error{CSRK_ERR_ARG, "direction must be 0 or 1"};
        if (elem_bytes != 4 && elem_bytes != 8) throw Error{CSRK_ERR_ARG, "elem_bytes must be 4 or 8"};
        if (nrhs < 1) throw Error{CSRK_ERR_ARG, "nrhs must be >= 1"};
        check_vec(in_dev, h, "in");
        check_vec(out_dev, h, "out");
        if (h->n > 0 && in_dev == out_dev) throw Error{CSRK_ERR_ARG, "in and out must not alias"};
        DeviceScope ds(h->device);
        hip_check(csrk::dev::permute(arrays_of(h), direction, in_dev, out_dev, nrhs, elem_bytes,
                                     static_cast<hipStream_t>(stream)),
                  "csrk_permute launch");
        return CSRK_OK;
    });
}

csrk_status csrk_destroy(csrk_handle h) {
    return guard([&] {
        if (!h) return CSRK_OK;
        free_device(h);
        delete h;
        return CSRK_OK;
    });
}

csrk_status csrk_batch_create(const csrk_handle *handles, int32_t count, csrk_batch *out) {
    return guard([&] {
        if (!out || !handles || count < 1) throw Error{CSRK_ERR_ARG, "need count >= 1 handles and an output"};
        *out = nullptr;
        for (int32_t b = 0; b < count; ++b) {
            need_device(handles[b]);
            if (handles[b]->store != handles[0]->store) throw Error{CSRK_ERR_ARG, "all handles need one storage type"};
            if (handles[b]->device != handles[0]->device) throw Error{CSRK_ERR_ARG, "all handles need one device"};
        }
        auto bt = new csrk_batch_s();
        try {
            bt->handles.assign(handles, handles + count);
            bt->store = handles[0]->store;
            bt->device = handles[0]->device;
            DeviceScope ds(bt->device);
            std::vector<int2> items;
            for (int32_t b = 0; b < count; ++b) {
                const int32_t nssr = static_cast<int32_t>(handles[b]->ssr_ptr.size()) - 1;
                for (int32_t t = 0; t < nssr; ++t) items.push_back(make_int2(b, t));
                bt->max_n = std::max(bt->max_n, handles[b]->n);
                bt->all_sym = bt->all_sym && handles[b]->trans.symmetric;
            }
            if (items.size() > size_t(INT32_MAX)) throw Error{CSRK_ERR_ARG, "work list too long"};
            bt->nitems = static_cast<int32_t>(items.size());
            bt->d_items = upload_array(items, "batch work list");
            // super-row records per item (the same records each handle keeps)
            for (int32_t b = 0; b < count; ++b) bt->brec_stride = std::max(bt->brec_stride, handles[b]->srec_stride);
            std::vector<csrk::dev::SrRec> brec(items.size() * size_t(bt->brec_stride), csrk::dev::SrRec{0, 0, 0, 0});
            for (size_t it = 0; it < items.size(); ++it) {
                const csrk_matrix *h = handles[items[it].x];
                const int32_t t = items[it].y;
                for (int32_t s = h->ssr_ptr[size_t(t)]; s < h->ssr_ptr[size_t(t) + 1]; ++s) {
                    const int32_t r0 = h->sr_ptr[size_t(s)], r1 = h->sr_ptr[size_t(s) + 1];
                    brec[it * size_t(bt->brec_stride) + size_t(s - h->ssr_ptr[size_t(t)])] =
                        csrk::dev::SrRec{r0, r1, h->row_ptr[size_t(r0)], h->row_ptr[size_t(r1)]};
                }
            }
            bt->d_brec = upload_array(brec, "batch super-row records");
            // the union-pattern ranges of the same super-rows (nonsymmetric matrices that have a union index)
            for (size_t it = 0; it < items.size(); ++it) {
                const csrk_matrix *h = handles[items[it].x];
                if (!h->d_srec_u) continue;
                const int32_t t = items[it].y;
                for (int32_t s = h->ssr_ptr[size_t(t)]; s < h->ssr_ptr[size_t(t) + 1]; ++s) {
                    auto &r = brec[it * size_t(bt->brec_stride) + size_t(s - h->ssr_ptr[size_t(t)])];
                    r.e0 = h->uni.sr_begin[size_t(s)];
                    r.e1 = h->uni.sr_end[size_t(s)];
                }
            }
            bt->d_brec_u = upload_array(brec, "batch union super-row records");
            for (int k = 0; k < 2; ++k)
                hip_check(hipMalloc(&bt->d_descs[k], sizeof(csrk::dev::MatDesc) * size_t(count)), "batch descriptors");
            // Batch-wide kernel shape: the first handle's lanes/waves, which
            // the batch tuner makes uniform.
            bt->shape = shape_of(handles[0]);
            int cus = 0;
            hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, bt->device), "CU count");
            bt->cus = cus;
        } catch (...) {
            if (bt->d_items) (void)hipFree(bt->d_items);
            if (bt->d_brec) (void)hipFree(bt->d_brec);
            if (bt->d_brec_u) (void)hipFree(bt->d_brec_u);
            for (auto *p : bt->d_descs)
                if (p) (void)hipFree(p);
            delete bt;
            throw;
        }
        *out = bt;
        return CSRK_OK;
    });
}

namespace {

csrk::dev::MatDesc *upload_descs(csrk_batch b, int which, const void *const *vals, const void *const *x, void *const *y, const void *const *g,
                  void *const *gx, void *const *gv, hipStream_t st) {
    const size_t count = b->handles.size();
    std::vector<csrk::dev::MatDesc> d(count);
    for (size_t i = 0; i < count; ++i) {
        const csrk_matrix *h = b->handles[i];
        csrk::dev::MatDesc &m = d[i];
        std::memset(&m, 0, sizeof(m));
        m.ssr_ptr = h->d_ssr_ptr;
        m.sr_ptr = h->d_sr_ptr;
        m.row_ptr = h->d_row_ptr;
        m.col_idx = h->d_col_idx;
        const csrk::dev::Arrays a = arrays_of(h);
        m.t_row_ptr = a.t_row_ptr;
        m.t_col = a.t_col;
        m.t_src = a.t_src;
        m.vals = values_for(h, vals ? vals[i] : nullptr);
        m.x = x ? x[i] : nullptr;
        m.y = y ? y[i] : nullptr;
        m.g = g ? g[i] : nullptr;
        m.gx = gx ? gx[i] : nullptr;
        m.gv = gv ? gv[i] : nullptr;
        m.nnz = h->nnz;
        m.n = h->n;
        m.nssr = static_cast<int32_t>(h->ssr_ptr.size()) - 1;
        m.sym = h->trans.symmetric ? 1 : 0;
        if (which == 1 && h->d_srec_u) {
            m.uni = 1;
            m.u_col = a.u_col;
            m.u_src = a.u_src;
            m.erow_ptr = a.erow_ptr;
            m.u_vals = a.u_vals;
            m.nu = a.nu;
        }
        if (which == 1) {
            // adjoint: caller values (CSR-k order, reached through t_src) when any
            // are given, otherwise the handles' transposed copies
            const bool any = vals && std::any_of(vals, vals + count, [](const void *p) { return p != nullptr; });
            m.vals = any ? values_for(h, vals[i]) : h->d_vals_t;
        }
    }
    if (b->last_valid[which] && std::memcmp(d.data(), b->last[which].data(), count * sizeof(d[0])) == 0)
        return b->d_descs[which];
    // Pageable source: the runtime has consumed it when the call returns.  The
    // copy is ordered after earlier kernels of the same stream that read the table.
    hip_check(hipMemcpyAsync(b->d_descs[which], d.data(), count * sizeof(d[0]), hipMemcpyHostToDevice, st),
              "batch descriptor upload");
    b->last[which] = std::move(d);
    b->last_valid[which] = true;
    return b->d_descs[which];
}

// True when every non-null pointer of every array is 16-byte aligned.
bool all_aligned16(std::initializer_list<const void *const *> arrays, size_t count) {
    for (const void *const *a : arrays) {
        if (!a) continue;
        for (size_t i = 0; i < count; ++i)
            if (a[i] && reinterpret_cast<uintptr_t>(a[i]) % 16) return false;
    }
    return true;
}

// Grid of a batched launch.  By default one workgroup per (matrix, SSR) work
// item: workgroups are dispatched in order and each XCD takes a contiguous
// range of items, so the workgroups resident on an XCD at any time work on
// neighbouring super-super-rows and share their x (and g) rows in that XCD's
// L2.  On the 64-matrix, 8-right-hand-side set this measured 15% faster in
// both directions than 16 workgroups per CU each walking a contiguous range of
// items (there, the resident workgroups of an XCD were spread over its whole
// range and the L2 hit rate fell to about a third).  With blocks_per_cu > 0
// (autotuner), the grid is at least that many workgroups per CU, each taking
// a contiguous range of items.
int batch_grid(csrk_batch b, int nrhs, bool adj, bool ind, bool vec, bool both) {
    if (b->blocks_per_cu == 0) return std::max(1, b->nitems);
    const int per_cu = std::max(b->blocks_per_cu, csrk::dev::batch_occupancy(b->store, nrhs, b->shape, adj, ind, vec,
                                                                              b->all_sym, both));
    const int64_t g = int64_t(b->cus) * per_cu;
    return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(g, b->nitems)));
}

}  // namespace

csrk_status csrk_batch_spmv(csrk_batch b, const void *const *vals, const void *const *x, void *const *y, int32_t nrhs,
                            void *stream) {
    return guard([&] {
        if (!b || !x || !y) throw Error{CSRK_ERR_ARG, "null argument"};
        if (nrhs < 1) throw Error{CSRK_ERR_ARG, "nrhs must be >= 1"};
        for (size_t i = 0; i < b->handles.size(); ++i) {
            check_vec(x[i], b->handles[i], "x");
            check_vec(y[i], b->handles[i], "y");
        }
        DeviceScope ds(b->device);
        hipStream_t st = static_cast<hipStream_t>(stream);
        csrk::dev::MatDesc *descs = upload_descs(b, 0, vals, x, y, nullptr, nullptr, nullptr, st);
        const bool vec = all_aligned16({x, reinterpret_cast<const void *const *>(y)}, b->handles.size());
        hip_check(csrk::dev::batch_forward(descs, b->d_items, b->d_brec, b->brec_stride, b->nitems, b->store, nrhs,
                                           b->shape,
                                           batch_grid(b, nrhs, false, false, vec, false), vec, st),
                  "csrk_batch_spmv launch");
        return CSRK_OK;
    });
}

csrk_status csrk_batch_spmv_adjoint(csrk_batch b, const void *const *vals, const void *const *x, const void *const *g,
                                    void *const *grad_x, void *const *grad_vals, int32_t nrhs, void *stream) {
    return guard([&] {
        if (!b || !g) throw Error{CSRK_ERR_ARG, "null argument"};
        if (nrhs < 1) throw Error{CSRK_ERR_ARG, "nrhs must be >= 1"};
        if (!grad_x && !grad_vals) return CSRK_OK;
        for (size_t i = 0; i < b->handles.size(); ++i) {
            check_vec(g[i], b->handles[i], "g");
            if (grad_vals) check_vec(x ? x[i] : nullptr, b->handles[i], "x");
            if (grad_vals && grad_vals[i]) check_align16(grad_vals[i], "grad_vals");
        }
        DeviceScope ds(b->device);
        hipStream_t st = static_cast<hipStream_t>(stream);
        csrk::dev::MatDesc *descs = upload_descs(b, 1, vals, x, nullptr, g, grad_x, grad_vals, st);
        const bool ind = vals && std::any_of(vals, vals + b->handles.size(), [](const void *p) { return p != nullptr; });
        const bool vec = all_aligned16({x, g, reinterpret_cast<const void *const *>(grad_x)}, b->handles.size());
        const bool both = grad_x && grad_vals;
        hip_check(csrk::dev::batch_adjoint(descs, b->d_items, b->d_brec, b->d_brec_u, b->brec_stride, b->nitems,
                                           b->store, nrhs,
                                           b->shape,
                                           batch_grid(b, nrhs, true, ind, vec, both), ind, vec, b->all_sym, both, st),
                  "csrk_batch_spmv_adjoint launch");
        return CSRK_OK;
    });
}

csrk_status csrk_probe_read(const void *buf_dev, int64_t bytes, double *part_dev, void *stream) {
    return guard([&] {
        if (bytes < 0 || bytes % 16 || (bytes > 0 && (!buf_dev || !part_dev)))
            throw Error{CSRK_ERR_ARG, "need bytes >= 0, a multiple of 16, and non-null buffers"};
        check_align16(buf_dev, "buf_dev");
        hip_check(csrk::dev::probe_read(buf_dev, bytes, part_dev, static_cast<hipStream_t>(stream)), "csrk_probe_read");
        return CSRK_OK;
    });
}

csrk_status csrk_probe_copy(const void *src_dev, void *dst_dev, int64_t bytes, void *stream) {
    return guard([&] {
        if (bytes < 0 || bytes % 16 || (bytes > 0 && (!src_dev || !dst_dev)))
            throw Error{CSRK_ERR_ARG, "need bytes >= 0, a multiple of 16, and non-null buffers"};
        check_align16(src_dev, "src_dev");
        check_align16(dst_dev, "dst_dev");
        hip_check(csrk::dev::probe_copy(src_dev, dst_dev, bytes, static_cast<hipStream_t>(stream)), "csrk_probe_copy");
        return CSRK_OK;
    });
}

csrk_status csrk_batch_set_launch(csrk_batch b, int32_t blocks_per_cu, int32_t waves_per_wg) {
    return guard([&] {
        if (!b) throw Error{CSRK_ERR_ARG, "null batch"};
        if (blocks_per_cu < 0 || blocks_per_cu > 256) throw Error{CSRK_ERR_ARG, "blocks_per_cu must be in 0..256"};
        if (waves_per_wg < 0 || waves_per_wg > 16) throw Error{CSRK_ERR_ARG, "waves_per_wg must be in 0..16"};
        b->blocks_per_cu = blocks_per_cu;
        if (waves_per_wg > 0) b->shape.waves = waves_per_wg;
        return CSRK_OK;
    });
}

csrk_status csrk_batch_destroy(csrk_batch b) {
    return guard([&] {
        if (!b) return CSRK_OK;
        DeviceScope ds(b->device);
        if (b->d_items) (void)hipFree(b->d_items);
        if (b->d_brec) (void)hipFree(b->d_brec);
        if (b->d_brec_u) (void)hipFree(b->d_brec_u);
        for (auto *p : b->d_descs)
            if (p) (void)hipFree(p);
        delete b;
        return CSRK_OK;
    });
}

}  // extern "C"
