// C-ABI of libffc_hip: argument checking, the compile step + upload, workspace handling
// and kernel dispatch.  Declarations and conventions: include/ffc_hip.h.
#include <hip/hip_runtime.h>

#include <dlfcn.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <initializer_list>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ffc_hip.h"
#include "kernels.h"
#include "assembly.h"
#include "mlp.h"
#include "reference_tensor.h"

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(FFC_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                         \
    do {                                            \
        hipError_t _e = (expr);                     \
        if (_e != hipSuccess) return hip_fail(_e, what); \
    } while (0)

// A usable device is a gfx950 (MI355X); anything else is refused loudly.
int check_device(int* device_out) {
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count <= 0) return fail(FFC_E_DEVICE, "no HIP device available");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(FFC_E_DEVICE, std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950");
    *device_out = dev;
    return FFC_OK;
}

template <typename T>
int upload(const std::vector<T>& host, T** dev) {
    *dev = nullptr;
    if (host.empty()) return FFC_OK;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(dev), host.size() * sizeof(T));
    if (e != hipSuccess) return fail(FFC_E_NOMEM, "hipMalloc failed for form tables");
    HIP_TRY(hipMemcpy(*dev, host.data(), host.size() * sizeof(T), hipMemcpyHostToDevice), "hipMemcpy");
    return FFC_OK;
}

bool valid_tile(int t) { return t == 16 || t == 32 || t == 64; }

// Element tensors with at least this many entries use the persistent FP64 kernel on 16-cell
// tiles by default; from kPersistentMidEntries on, the 12-wave persistent kernel on tiles of
// 16, 32 or 64 cells (below it, even a 64-cell tile carries too little output to pay for the
// per-tile pipeline; measured on MI355X: the tile kernels win at 36 entries and below).
constexpr int kPersistentMinEntries = 576;
constexpr int kPersistentMidEntries = 100;
// The persistent split-BF16 kernel (FP32 output: half the bytes per entry; it reads the
// affine maps of a geometry pass) by default from 144 entries, or from 100 for forms with
// coefficients (measured on MI355X at ~10^6 cells: 64-cell persistent tiles 5-19% faster
// than the tile kernels there, 3-11% slower for the 100-entry Laplacian and mass matrices
// on tetrahedra, whose geometry-pass traffic is large against their output).
constexpr int kBf16PersistentMinEntries = 144;
constexpr int kBf16PersistentMinEntriesCoeff = 100;
bool valid_waves(int w) { return w == 1 || w == 2 || w == 4 || w == 8 || w == 12 || w == 16; }

int check_desc(const ffc_form_desc* d, ffc::FormSpec* spec) {
    if (!d) return fail(FFC_E_INVALID, "desc is NULL");
    spec->kind = d->kind;
    spec->dim = d->dim;
    spec->degree = d->degree;
    spec->lambda = d->lambda;
    spec->mu = d->mu;
    std::string why;
    if (!ffc::supported(*spec, &why)) return fail(FFC_E_UNSUPPORTED, why);
    if (d->precision < FFC_FP64 || d->precision > FFC_SPLIT_BF16_6)
        return fail(FFC_E_UNSUPPORTED, "unknown precision");
    if (d->kernel != FFC_KERNEL_AUTO && d->kernel != FFC_KERNEL_TENSOR && d->kernel != FFC_KERNEL_QUADRATURE)
        return fail(FFC_E_UNSUPPORTED, "unknown kernel");
    if (d->kernel == FFC_KERNEL_QUADRATURE && d->precision != FFC_FP64)
        return fail(FFC_E_UNSUPPORTED, "the quadrature kernel is FP64 only");
    if (d->kernel == FFC_KERNEL_QUADRATURE &&
        (d->kind == FFC_PIOLA_MASS || d->kind == FFC_CURVED_LAPLACE || d->kind == FFC_NEDELEC_MASS))
        return fail(FFC_E_UNSUPPORTED, "the quadrature kernel evaluates Lagrange forms on affine cells only");
    if (d->kind == FFC_CURVED_LAPLACE && d->precision != FFC_FP64)
        return fail(FFC_E_UNSUPPORTED, "the curvilinear Laplacian is FP64 only");
    if (d->tile_cells != 0 && !valid_tile(d->tile_cells)) return fail(FFC_E_INVALID, "tile_cells must be 0, 16, 32 or 64");
    if (d->waves != 0 && !valid_waves(d->waves)) return fail(FFC_E_INVALID, "waves must be 0, 1, 2, 4, 8, 12 or 16");
    if (d->geometry < 0 || d->geometry > FFC_GEOMETRY_FUSED) return fail(FFC_E_INVALID, "geometry must be 0, 1 or 2");
    if (d->symmetry < -1 || d->symmetry > 0) return fail(FFC_E_INVALID, "symmetry must be 0 or -1");
    if (d->persistent < -1 || d->persistent > 1) return fail(FFC_E_INVALID, "persistent must be -1, 0 or 1");
    if (d->tile_window != 0 && d->tile_window != -1 && (d->tile_window < 16 || d->tile_window % 16 != 0))
        return fail(FFC_E_INVALID, "tile_window must be 0, -1 or a positive multiple of 16");
    return FFC_OK;
}

constexpr int kAutoBuckets = 41;  // cell counts 2^0 .. 2^40

int auto_bucket(int64_t cells) {
    const double l = cells > 0 ? std::log2(static_cast<double>(cells)) : 0.0;
    return static_cast<int>(std::min<double>(kAutoBuckets - 1, std::max(0.0, std::floor(l + 0.5))));
}

// ------------------------------------------------------------------ selector file ----
// The learned kernel choice (the automatic tensor-vs-quadrature decision of Sec. 4.4): a
// multilayer perceptron trained on timings of every candidate launch predicts
// log(t_candidate / t_default) from seven features of the form and the cell count; the
// lowest candidate is taken if it beats the default by more than the file's decision margin.
// The text file holds: "ffc_selector 2", the sizes, the feature means and deviations, the
// target offset, the margin (a fraction; version 1 files have none: plain argmin), the flat
// FP32 parameters (W1 [n_in][h], b1, W2 [h][h], b2, W3 [h][n_out], b3) and one line per
// candidate launch.
struct SelectorNet {
    int n_in = 0, h = 0, n_out = 0;
    std::vector<double> mu, sd;
    double tmu = 0.0, margin = 0.0;
    std::vector<float> params;
    struct Cand {
        int kernel, tile_cells, waves, persistent, tile_window, geometry;
    };
    std::vector<Cand> cands;

    bool load(const std::string& path, std::string* err) {
        FILE* fp = std::fopen(path.c_str(), "r");
        if (!fp) {
            *err = "cannot open " + path;
            return false;
        }
        auto word = [&](const char* want) {
            char buf[64] = {0};
            return std::fscanf(fp, "%63s", buf) == 1 && std::strcmp(buf, want) == 0;
        };
        int version = 0;
        bool ok = word("ffc_selector") && std::fscanf(fp, "%d", &version) == 1 && (version == 1 || version == 2) &&
                  word("n_in") &&
                  std::fscanf(fp, "%d", &n_in) == 1 && word("n_hidden") && std::fscanf(fp, "%d", &h) == 1 &&
                  word("n_out") && std::fscanf(fp, "%d", &n_out) == 1 && n_in == 7 && h > 0 && h <= 4096 &&
                  n_out > 0 && n_out <= 64;
        if (ok) {
            mu.resize(n_in);
            sd.resize(n_in);
            ok = word("mu");
            for (int i = 0; ok && i < n_in; ++i) ok = std::fscanf(fp, "%lf", &mu[i]) == 1;
            ok = ok && word("sd");
            for (int i = 0; ok && i < n_in; ++i) ok = std::fscanf(fp, "%lf", &sd[i]) == 1 && sd[i] > 0.0;
            ok = ok && word("tmu") && std::fscanf(fp, "%lf", &tmu) == 1;
            if (version == 2)
                ok = ok && word("margin") && std::fscanf(fp, "%lf", &margin) == 1 && margin >= 0.0 && margin < 1.0;
        }
        long long np = 0;
        if (ok) ok = word("params") && std::fscanf(fp, "%lld", &np) == 1 &&
                     np == static_cast<long long>(n_in) * h + h + static_cast<long long>(h) * h + h +
                               static_cast<long long>(h) * n_out + n_out;
        if (ok) {
            params.resize(static_cast<size_t>(np));
            for (long long i = 0; ok && i < np; ++i) ok = std::fscanf(fp, "%f", &params[i]) == 1;
        }
        int nc = 0;
        ok = ok && word("candidates") && std::fscanf(fp, "%d", &nc) == 1 && nc == n_out;
        for (int i = 0; ok && i < nc; ++i) {
            Cand c{};
            ok = std::fscanf(fp, "%d %d %d %d %d %d", &c.kernel, &c.tile_cells, &c.waves, &c.persistent,
                             &c.tile_window, &c.geometry) == 6 &&
                 (c.kernel == FFC_KERNEL_TENSOR || c.kernel == FFC_KERNEL_QUADRATURE);
            cands.push_back(c);
        }
        std::fclose(fp);
        if (!ok) *err = "malformed selector file " + path;
        return ok;
    }

    // predicted log(t_c / t_default) of every candidate for one feature vector
    std::vector<double> predict(const double* x_raw) const {
        std::vector<double> x(n_in), h1(h), h2(h), y(n_out);
        for (int i = 0; i < n_in; ++i) x[i] = (x_raw[i] - mu[i]) / sd[i];
        const float* W1 = params.data();
        const float* b1 = W1 + n_in * h;
        const float* W2 = b1 + h;
        const float* b2 = W2 + h * h;
        const float* W3 = b2 + h;
        const float* b3 = W3 + h * n_out;
        for (int j = 0; j < h; ++j) {
            double a = b1[j];
            for (int i = 0; i < n_in; ++i) a += x[i] * W1[i * h + j];
            h1[j] = a > 0.0 ? a : 0.0;
        }
        for (int j = 0; j < h; ++j) {
            double a = b2[j];
            for (int i = 0; i < h; ++i) a += h1[i] * W2[i * h + j];
            h2[j] = a > 0.0 ? a : 0.0;
        }
        for (int j = 0; j < n_out; ++j) {
            double a = b3[j];
            for (int i = 0; i < h; ++i) a += h2[i] * W3[i * n_out + j];
            y[j] = a + tmu;
        }
        return y;
    }
};

// The selector file: $FFC_SELECTOR if set ("none" or empty: no file), else
// data/selector_mi355x_fp64.txt in the directory of this library.
std::string selector_path() {
    if (const char* e = std::getenv("FFC_SELECTOR")) return std::strcmp(e, "none") == 0 ? std::string() : e;
    Dl_info info;
    if (dladdr(reinterpret_cast<void*>(&auto_bucket), &info) == 0 || !info.dli_fname) return std::string();
    std::string lib = info.dli_fname;
    const size_t slash = lib.find_last_of('/');
    return (slash == std::string::npos ? std::string(".") : lib.substr(0, slash)) + "/data/selector_mi355x_fp64.txt";
}

}  // namespace

struct ffc_form {
    ffc_form_desc desc{};
    ffc::ReferenceTensor rt;
    int n_tiles = 0, kpad = 0, n_seg = 0, gpiece[6] = {0, 0, 0, 0, 0, 0};
    int64_t mfma_k = 0;
    int tile_cells = 64, waves = 4;
    hipStream_t stream = nullptr;
    int device = 0;
    int tile_window = -1;
    int32_t* d_koff = nullptr;
    uint32_t* d_apack = nullptr;
    int32_t* d_entry = nullptr;
    double* d_b = nullptr;
    uint16_t* d_bb = nullptr;
    uint8_t* d_nz = nullptr;
    double* d_pts = nullptr;
    double* d_wts = nullptr;
    double* d_phi = nullptr;
    double* d_dphi = nullptr;
    int quad_npts = 0, quad_cpb = 1;
    double* d_amap = nullptr;
    int64_t amap_cap = 0;
    // persistent FP64 contraction
    int pwaves = 0, pkmax = 0, pgrid = 0, n_zero = 0;
    int pmt = 1;  // persistent FP64 kernel: cell tiles of 16 * pmt cells
    bool bpersistent = false;  // split modes: persistent BF16 contraction (pwaves, pkmax, pgrid set)
    int ptile = 16;            // its cell tile
    bool fused = false;  // ffc_tabulate_tensor computes the affine map inside the tile kernel
    // FP64: tabulations take the 16-cell tile kernel although a persistent schedule exists
    // (which the operator action and batches keep using)
    bool tab_tile = false;
    int sym_n = 0;       // FP64 symmetric tiles: element dofs
    int n_alpha_form = 0;  // |alpha| and nnz of A^0 as the form defines them (before the fold)
    int64_t nnz_form = 0;
    int32_t* d_woff = nullptr;
    double* d_wave_b = nullptr;
    uint32_t* d_wave_word = nullptr;
    uint32_t* d_wave_mask = nullptr;
    int32_t* d_zero = nullptr;
    double* d_geo_grad = nullptr;  // curvilinear cells: geometry basis gradients at the points
    // FFC_KERNEL_AUTO: the forms of the launches the selector picks (subs[0] = the library
    // default tensor launch) and, per cell-count bucket round(log2 cells), the sub-form used
    // and the selector's candidate index
    bool is_auto = false, auto_from_selector = false;
    std::vector<std::unique_ptr<ffc_form>> subs;
    int8_t bucket_sub[kAutoBuckets] = {};
    int32_t bucket_cand[kAutoBuckets] = {};

    ~ffc_form() {
        for (void* p : {static_cast<void*>(d_koff), static_cast<void*>(d_apack), static_cast<void*>(d_entry),
                        static_cast<void*>(d_b),
                        static_cast<void*>(d_bb), static_cast<void*>(d_nz), static_cast<void*>(d_pts),
                        static_cast<void*>(d_wts), static_cast<void*>(d_phi), static_cast<void*>(d_dphi),
                        static_cast<void*>(d_amap), static_cast<void*>(d_woff),
                        static_cast<void*>(d_wave_b), static_cast<void*>(d_wave_word), static_cast<void*>(d_wave_mask),
                        static_cast<void*>(d_zero), static_cast<void*>(d_geo_grad)})
            if (p) (void)hipFree(p);
    }
};

extern "C" {

const char* ffc_last_error(void) { return g_last_error.c_str(); }

const char* ffc_version(void) { return "ffc_hip 0.1 (gfx950)"; }

int ffc_compile_reference_tensor(const ffc_form_desc* desc, int64_t* n_I, int64_t* n_alpha, double* A0) {
    ffc::FormSpec spec;
    int rc = check_desc(desc, &spec);
    if (rc) return rc;
    if (!n_I || !n_alpha) return fail(FFC_E_INVALID, "n_I / n_alpha is NULL");
    ffc::ReferenceTensor rt;
    std::string err;
    if (!ffc::build_reference_tensor(spec, &rt, &err)) return fail(FFC_E_UNSUPPORTED, err);
    *n_I = rt.n_I;
    *n_alpha = rt.n_alpha;
    if (A0) std::memcpy(A0, rt.A0.data(), rt.A0.size() * sizeof(double));
    return FFC_OK;
}

namespace {
// The form a call on `cells` cells runs on: an FFC_KERNEL_AUTO form delegates to the launch
// its selector picked for that cell count; other forms are their own launch.
const ffc_form* resolve(const ffc_form* f, int64_t cells) {
    return f && f->is_auto ? f->subs[f->bucket_sub[auto_bucket(cells)]].get() : f;
}
// the library default tensor launch of an AUTO form (entry points other than tabulation)
const ffc_form* resolve_default(const ffc_form* f) { return f && f->is_auto ? f->subs[0].get() : f; }

int create_auto(const ffc_form_desc* desc, const ffc::FormSpec& spec, ffc_form** out) {
    std::unique_ptr<ffc_form> f(new ffc_form());
    f->desc = *desc;
    f->is_auto = true;
    ffc_form_desc d0 = *desc;
    d0.kernel = FFC_KERNEL_TENSOR;
    ffc_form* sub = nullptr;
    int rc = ffc_form_create(&d0, &sub);
    if (rc) return rc;
    f->subs.emplace_back(sub);
    f->device = sub->device;
    f->stream = sub->stream;
    // the selector was trained on FP64 Lagrange forms on affine cells: it decides there only
    const bool lagrange = spec.kind >= FFC_MASS && spec.kind <= FFC_NS_CONVECTION;
    if (desc->precision == FFC_FP64 && lagrange) {
        const std::string path = selector_path();
        SelectorNet net;
        std::string err;
        if (!path.empty() && net.load(path, &err)) {
            f->auto_from_selector = true;
            std::map<int, int> sub_of_cand{{0, 0}};
            const double lI = std::log2(static_cast<double>(sub->rt.n_I));
            const double la = std::log2(static_cast<double>(sub->n_alpha_form) + 1.0);
            for (int b = 0; b < kAutoBuckets; ++b) {
                // features: form rank, degree, log2 |i|, log2(|alpha| + 1), dimension, log2 cells,
                // log2(cells |i|)
                const double x[7] = {2.0, static_cast<double>(desc->degree), lI, la, static_cast<double>(desc->dim),
                                     static_cast<double>(b), b + lI};
                const std::vector<double> y = net.predict(x);
                int best = static_cast<int>(std::min_element(y.begin(), y.end()) - y.begin());
                if (!(y[best] < y[0] - std::log1p(net.margin))) best = 0;  // within the margin: the default
                auto it = sub_of_cand.find(best);
                if (it == sub_of_cand.end()) {
                    const SelectorNet::Cand& c = net.cands[best];
                    ffc_form_desc dc = *desc;
                    dc.kernel = c.kernel;
                    dc.tile_cells = c.tile_cells;
                    dc.waves = c.waves;
                    dc.persistent = c.persistent;
                    dc.tile_window = c.tile_window;
                    dc.geometry = c.geometry;
                    ffc_form* sc = nullptr;
                    if ((rc = ffc_form_create(&dc, &sc))) return rc;
                    f->subs.emplace_back(sc);
                    it = sub_of_cand.emplace(best, static_cast<int>(f->subs.size()) - 1).first;
                }
                f->bucket_sub[b] = static_cast<int8_t>(it->second);
                f->bucket_cand[b] = best;
            }
        } else if (std::getenv("FFC_SELECTOR") && !path.empty()) {
            return fail(FFC_E_INVALID, "FFC_SELECTOR: " + err);  // a file was named and cannot be used
        }
    }
    *out = f.release();
    return FFC_OK;
}
}  // namespace

int ffc_form_create(const ffc_form_desc* desc, ffc_form** out) {
    if (!out) return fail(FFC_E_INVALID, "form output pointer is NULL");
    *out = nullptr;
    ffc::FormSpec spec;
    int rc = check_desc(desc, &spec);
    if (rc) return rc;
    int dev = 0;
    rc = check_device(&dev);
    if (rc) return rc;
    if (desc->kernel == FFC_KERNEL_AUTO) return create_auto(desc, spec, out);
    std::unique_ptr<ffc_form> f(new ffc_form());
    f->desc = *desc;
    f->device = dev;
    f->stream = static_cast<hipStream_t>(desc->stream);
    f->tile_cells = desc->tile_cells;
    f->waves = desc->waves;
    std::string err;
    if (!ffc::build_reference_tensor(spec, &f->rt, &err)) return fail(FFC_E_UNSUPPORTED, err);
    f->n_alpha_form = f->rt.n_alpha;
    f->nnz_form = f->rt.nnz;
    // tensor kernels contract symmetric geometry tensors over unordered index pairs
    if (desc->kernel == FFC_KERNEL_TENSOR) {
        f->rt = ffc::fold_symmetric_g(f->rt);
        if (spec.kind != FFC_CURVED_LAPLACE && f->rt.n_alpha != ffc::folded_n_alpha(spec.kind, spec.dim))
            return fail(FFC_E_UNSUPPORTED, "internal: G entry count does not match the kernels");
        if (spec.kind == FFC_CURVED_LAPLACE && (rc = upload(f->rt.geo_grad, &f->d_geo_grad))) return rc;
    }
    const ffc::ReferenceTensor& rt = f->rt;
    if (desc->kernel == FFC_KERNEL_QUADRATURE) {
        ffc::QuadTables qt = ffc::make_quad_tables(spec);
        f->quad_npts = qt.npts;
        f->quad_cpb = ffc::quad_cells_per_block(spec.dim, spec.kind, qt.ns, qt.npts);
        if ((rc = upload(qt.pts, &f->d_pts)) || (rc = upload(qt.wts, &f->d_wts)) || (rc = upload(qt.phi, &f->d_phi)) ||
            (rc = upload(qt.dphi, &f->d_dphi)))
            return rc;
    } else if (desc->precision == FFC_FP64) {
        // default grouping: greedy clustering over all rows for large element tensors (the
        // persistent kernel), consecutive rows for small ones (64-cell tiles) -- and for
        // mid-size ones (from kPersistentMidEntries) clustering too where it moves the 12-wave
        // schedule into a smaller register-step bucket (elasticity P1 on tetrahedra: 8 instead
        // of 16 steps per wave, 0.331 -> 0.253 ms at ~10^6 cells; with the bucket unchanged,
        // fewer steps alone measured -2% to +13%)
        f->tile_window = desc->tile_window ? desc->tile_window : (rt.n_I >= kPersistentMinEntries ? -1 : 16);
        // symmetric forms: tiles over the entries i1 <= i2, where that takes fewer MFMA steps
        auto tiles_for = [&](int window, int* sym_n) {
            ffc::TilesF64 tt = ffc::make_tiles_f64(rt, window, false);
            *sym_n = 0;
            if (desc->symmetry == 0 && spec.kind != FFC_NS_CONVECTION) {
                ffc::TilesF64 ts = ffc::make_tiles_f64(rt, window, true);
                if (ts.koff.back() < tt.koff.back()) {
                    tt = std::move(ts);
                    *sym_n = rt.n;
                }
            }
            return tt;
        };
        ffc::TilesF64 t = tiles_for(f->tile_window, &f->sym_n);
        if (desc->tile_window == 0 && f->tile_window == 16 && rt.n_I >= kPersistentMidEntries) {
            int sym_c = 0;
            ffc::TilesF64 tc = tiles_for(-1, &sym_c);
            auto bucket = [](int steps) { return steps <= 8 ? 8 : steps <= 16 ? 16 : 24; };
            if (bucket(ffc::make_wave_schedule(tc, 12 - ffc::kIoWaves).max_steps) <
                bucket(ffc::make_wave_schedule(t, 12 - ffc::kIoWaves).max_steps)) {
                t = std::move(tc);
                f->sym_n = sym_c;
                f->tile_window = -1;
            }
        }
        f->n_tiles = t.n_tiles;
        f->mfma_k = t.koff.back();
        if ((rc = upload(t.koff, &f->d_koff)) || (rc = upload(t.apack, &f->d_apack)) ||
            (rc = upload(t.entry, &f->d_entry)) || (rc = upload(t.b, &f->d_b)))
            return rc;
        // persistent workgroups of 12 waves (6 compute, ~168 registers per lane: the kernel then
        // also computes the affine maps) or 16 waves (10 compute, 128 registers, affine maps from
        // a geometry pass), with up to 24 register-resident k steps per compute wave; cell tiles
        // of 16 cells, or (12 waves, tile_cells = 32 or 64) 32 or 64 cells with up to 16 steps;
        // the output rows of a tile must be stageable in LDS and in the I/O registers
        const bool want_persistent = spec.kind != FFC_CURVED_LAPLACE &&
            (desc->persistent == 1 || (desc->persistent == 0 && rt.n_I >= kPersistentMidEntries));
        // launch shapes to try, in order: (waves per workgroup, 16-cell blocks per cell tile)
        std::vector<std::pair<int, int>> shapes;
        auto waves_ok = [&](int w) { return desc->waves == 0 || desc->waves == w; };
        const int req_mt = desc->tile_cells == 16 ? 1 : desc->tile_cells == 32 ? 2 : desc->tile_cells == 64 ? 4 : 0;
        ffc::WaveSchedule ws12;  // the 12-wave schedule (6 compute waves), if have12
        bool have12 = false;
        if (want_persistent && desc->persistent == 1 && req_mt > 0) {
            // as requested; 32- and 64-cell tiles take 12-wave workgroups
            for (int w : {16, 12})
                if (waves_ok(w) && (req_mt == 1 || w == 12)) shapes.push_back({w, req_mt});
        } else if (want_persistent && (desc->persistent == 1 || rt.n_I >= kPersistentMinEntries)) {
            // large tensors: 16-cell tiles.  Forms with coefficients: 12 waves first (the
            // kernel computes the affine maps: one launch; the convection form 10% faster than
            // on 16 waves).  Without coefficients 16 waves first: those forms tabulate on
            // per-tile workgroups by default (below), and the schedule serves the operator
            // action, measured faster on 16 waves (elasticity P2: 0.77 vs 0.88 ms per action)
            if (desc->tile_cells == 0 || req_mt == 1) {
                const bool twelve_first = desc->persistent == 0 && rt.n_coeff > 0;
                for (int w : twelve_first ? std::initializer_list<int>{12, 16} : std::initializer_list<int>{16, 12})
                    if (waves_ok(w)) shapes.push_back({w, 1});
            }
        } else if (want_persistent && desc->tile_cells == 0 && waves_ok(12)) {
            // mid-size tensors: 12 waves, on the largest cell tile whose staged rows and
            // schedule fit -- except 16-cell tiles once those carry 48 KiB of output and a
            // wave takes at most 8 steps (measured on MI355X, 100 to 400 entries: 64-cell
            // tiles 20-35% faster than the tile kernels at 100 and 144 entries, 32-cell tiles
            // at 225; at 400 entries 16-cell tiles with 8 steps, 32-cell tiles with 16)
            ws12 = ffc::make_wave_schedule(t, 12 - ffc::kIoWaves);
            have12 = true;
            std::vector<int> fit;
            for (int m : {4, 2, 1})
                if (ws12.max_steps <= (m == 1 ? 24 : 16) &&
                    ffc::persistent_fits(spec.dim, spec.kind, rt.n_I, rt.n_alpha, m, true, nullptr, nullptr, nullptr))
                    fit.push_back(m);
            if (!fit.empty()) {
                int m = fit.front();
                if (fit.back() == 1 && 16 * 8 * static_cast<int64_t>(rt.n_I) >= 48 * 1024 && ws12.max_steps <= 8)
                    m = 1;
                shapes.push_back({12, m});
            }
        }
        if (!shapes.empty()) {
            ffc::WaveSchedule ws;
            for (const auto& [w, mt] : shapes) {
                if (!ffc::persistent_fits(spec.dim, spec.kind, rt.n_I, rt.n_alpha, mt, w == 12, nullptr, nullptr,
                                          nullptr))
                    continue;
                ffc::WaveSchedule cand =
                    w == 12 && have12 ? ws12 : ffc::make_wave_schedule(t, w - ffc::kIoWaves);
                if (cand.max_steps <= (mt == 1 ? 24 : 16)) {
                    ws = std::move(cand);
                    ws.waves = w;
                    f->pmt = mt;
                    break;
                }
            }
            if (ws.waves > 0) {
                f->pwaves = ws.waves;
                f->pkmax = ws.max_steps <= 8 ? 8 : ws.max_steps <= 16 ? 16 : 24;
                f->n_zero = static_cast<int>(ws.zero_entries.size());
                // each compute wave's register contents, expanded per step and lane so that
                // the kernel loads them with independent, coalesced loads
                const int nw = ws.waves - ffc::kIoWaves, km = f->pkmax;
                std::vector<double> wb(static_cast<size_t>(nw) * km * 64, 0.0);
                std::vector<uint32_t> wword(static_cast<size_t>(nw) * km * 64, 0u), wmask(nw, 0u);
                for (int w = 0; w < nw; ++w)
                    for (int s = 0; s < ws.woff[w + 1] - ws.woff[w]; ++s) {
                        const int ks = ws.step_kstep[ws.woff[w] + s], te = ws.step_end[ws.woff[w] + s];
                        if (te >= 0) wmask[w] |= 1u << s;
                        for (int l = 0; l < 64; ++l) {
                            const int lk = l / 16, lr = l % 16;
                            const size_t i = (static_cast<size_t>(w) * km + s) * 64 + l;
                            wb[i] = t.b[(static_cast<size_t>(ks) * 4 + lk) * 16 + lr];
                            uint32_t word = (t.apack[ks] >> (8 * lk)) & 0xffu;
                            const int e = te >= 0 ? t.entry[te * 16 + lr] : -1;
                            if (e >= 0) {
                                word |= static_cast<uint32_t>(e + 1) << 8;
                                // symmetric forms: the transposed entry too (off the diagonal)
                                const int e2 = f->sym_n ? (e % f->sym_n) * f->sym_n + e / f->sym_n : e;
                                if (e2 != e) word |= static_cast<uint32_t>(e2 + 1) << 20;
                            }
                            wword[i] = word;
                        }
                    }
                if ((rc = upload(ws.woff, &f->d_woff)) || (rc = upload(wb, &f->d_wave_b)) ||
                    (rc = upload(wword, &f->d_wave_word)) || (rc = upload(wmask, &f->d_wave_mask)) ||
                    (rc = upload(ws.zero_entries, &f->d_zero)))
                    return rc;
                // one workgroup per CU: 1024 threads at ~128 registers per lane, or 768 at
                // ~168, fill the register file
                hipDeviceProp_t prop;
                HIP_TRY(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
                f->pgrid = prop.multiProcessorCount;
            }
        }
    } else {
        ffc::TilesBF16 t = ffc::make_tiles_bf16(rt, desc->precision == FFC_SPLIT_BF16_3 ? 3 : 6);
        f->n_tiles = t.n_tiles;
        f->kpad = t.kpad;
        f->n_seg = t.n_seg;
        std::copy(t.gpiece, t.gpiece + 6, f->gpiece);
        f->mfma_k = static_cast<int64_t>(t.kpad) * t.n_tiles;
        if ((rc = upload(t.b, &f->d_bb)) || (rc = upload(t.nonzero, &f->d_nz))) return rc;
        // persistent split-BF16 kernel when the form fits it (B fragments of at most 16
        // steps per wave in registers, a staged tile in the I/O lanes' registers)
        // (cell tiles: the largest that fits among 64, 32, 16 cells -- except 3 products on
        // tensors of 256 entries and more, which take 32 and 16 (measured on MI355X: 64-cell
        // tiles 4% faster than 32 for x6 on the weighted Laplacian P3, 7% slower for x3, and
        // faster for both below 256 entries); 64 there on request)
        const bool bwant = desc->persistent == 1 ||
                           (desc->persistent == 0 && (rt.n_I >= kBf16PersistentMinEntries ||
                                                      (rt.n_I >= kBf16PersistentMinEntriesCoeff && rt.n_coeff > 0)));
        if (desc->kernel == FFC_KERNEL_TENSOR && bwant && (desc->waves == 0 || desc->waves == 16)) {
            for (int ct : {64, 32, 16}) {
                const bool skip64 = ct == 64 && t.n_seg != 6 && rt.n_I >= 256;
                if (desc->tile_cells != ct && (desc->tile_cells != 0 || skip64)) continue;
                if (!ffc::plan_bf16_persistent(spec.dim, spec.kind, ct, rt.n_I, t.n_tiles, t.kpad, t.n_seg).staged)
                    continue;
                hipDeviceProp_t prop;
                HIP_TRY(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
                f->bpersistent = true;
                f->ptile = ct;
                f->pwaves = 16;
                f->pkmax = ffc::bf16_persistent_steps(t.n_tiles, t.kpad);
                f->pgrid = prop.multiProcessorCount;
                break;
            }
        }
    }
    if (desc->kernel == FFC_KERNEL_TENSOR) {
        // geometry workspace (chunks of 2^21 cells), unless every tabulation is fused
        // (curvilinear cells: G itself, n_alpha rows, in chunks of the same byte size)
        const int rows = spec.kind == FFC_CURVED_LAPLACE ? rt.n_alpha : 1 + spec.dim * spec.dim;
        f->amap_cap = spec.kind == FFC_CURVED_LAPLACE ? ((int64_t(1) << 21) * (1 + spec.dim * spec.dim) / rows + 63) / 64 * 64
                                                     : int64_t(1) << 21;
        const size_t bytes = static_cast<size_t>(f->amap_cap) * rows * sizeof(double);
        // default launch shape when the persistent kernel does not apply
        const bool bf = desc->precision != FFC_FP64;
        auto plan = [&](int ct) {
            return ffc::plan_lds(spec.dim, spec.kind, ct, rt.n_I, rt.n_alpha, f->kpad, bf, ffc::kLdsBudget);
        };
        int dw = 0;  // default waves
        // Tensors of 400 entries and more without coefficients: with non-temporal stores for
        // the staged rows, 16-cell tiles of one workgroup each after a geometry pass measured
        // faster than the persistent kernel on MI355X (elasticity P2 on tetrahedra, 750k
        // cells: step 1.02-1.03 vs 1.06 ms; Laplacian P3 on tetrahedra 0.569 vs 0.667 ms,
        // elasticity P3 on triangles 0.520 vs 0.578, mass P3 0.610 vs 0.639 at ~10^6 cells;
        // not at 225 entries, nor for the forms with coefficients), so tabulation takes them;
        // the persistent schedule stays for the operator action and batches
        if (!bf && f->pwaves > 0 && desc->persistent == 0 && desc->tile_cells == 0 && desc->waves == 0 &&
            rt.n_coeff == 0 && rt.n_I >= 400 && plan(16).staged)
            f->tab_tile = true;
        if (f->tab_tile) {
            f->tile_cells = 16, dw = 16;
        } else if (f->tile_cells == 0) {
            if (!bf && rt.n_I < kPersistentMinEntries) {
                // small FP64 tensors (measured on MI355X): 64-cell tiles staged in at most
                // 40 KiB of LDS (several workgroups per CU); else 32-cell tiles staged in at
                // most 80 KiB (two per CU); else 64-cell tiles written directly (consecutive
                // output rows per MFMA tile keep those writes in whole 128-byte runs).  Tiny
                // tensors take one- or two-wave workgroups: a tile's latency chain (coordinate
                // load, geometry, MFMA, staged write) is then overlapped by more resident
                // workgroups -- 32-cell tiles of one wave up to 16 entries (P1 forms 1.3-1.9x
                // faster than 64-cell tiles of 4 waves), 64-cell tiles of two waves up to 36
                // (1.2x)
                const ffc::LdsPlan p64 = plan(64), p32 = plan(32);
                const bool tiny = spec.kind != FFC_CURVED_LAPLACE;
                if (!tiny && rt.n_I <= 36 && p32.staged) {
                    // curvilinear cells, small tensors (G per cell from the quadrature points):
                    // 32-cell tiles of four waves (P1 functions in 3D 0.215 -> 0.168 ms, P2 in 2D
                    // 0.118 -> 0.108 ms at 7.5e5 cells)
                    f->tile_cells = 32, dw = 4;
                } else if (tiny && rt.n_coeff > 0 && rt.n_I > 9 && rt.n_I <= 36 && p32.staged) {
                    // forms with coefficients (longer G build per cell): 32-cell tiles of two
                    // waves (weighted Laplacian P1 on tetrahedra 0.114 -> 0.103 ms, P2 on
                    // triangles 0.113 -> 0.104 at ~10^6 cells)
                    f->tile_cells = 32, dw = 2;
                } else if (tiny && rt.n_I <= 16 && p32.staged) {
                    f->tile_cells = 32, dw = 1;
                } else if (tiny && rt.n_I <= 36 && p64.staged && p64.total <= 40 * 1024) {
                    f->tile_cells = 64, dw = 2;
                } else if (p64.staged && p64.total <= 40 * 1024) {
                    f->tile_cells = 64, dw = 4;
                } else if (p32.staged && p32.total <= 80 * 1024) {
                    f->tile_cells = 32, dw = 8;
                } else {
                    f->tile_cells = 64, dw = 4;
                }
            } else {
                // large FP64 tensors without the persistent kernel, and the split modes: the
                // largest stageable tile among 64 / 32 / 16 cells
                f->tile_cells = 64;
                for (int ct : {64, 32, 16}) {
                    const ffc::LdsPlan p = plan(ct);
                    if (p.staged && p.total <= (ct == 16 ? ffc::kLdsBudget : ffc::kLdsBudget / 2 + 8192)) {
                        f->tile_cells = ct;
                        break;
                    }
                }
                // split modes, 64-cell tiles of small tensors: few waves per workgroup, so more
                // workgroups stay resident and overlap each tile's latency chain (measured on
                // MI355X at ~10^6 cells, x6 and x3: against 8 waves, 1 wave 2.7x faster for 9
                // entries, 2 waves 1.6-2.1x for 16-36, 4 waves 1.1-1.5x for 100 entries and for
                // forms with coefficients, whose G build is longer)
                if (bf && f->tile_cells == 64 && rt.n_I <= 100)
                    dw = rt.n_coeff > 0 || rt.n_I > 36 ? 4 : rt.n_I > 9 ? 2 : 1;
            }
        }
        if (f->waves == 0) f->waves = dw ? dw : f->tile_cells == 16 ? 16 : bf ? 8 : 4;
        if (!bf && f->sym_n && f->pwaves == 0 && !plan(f->tile_cells).staged) {
            // direct stores: the transposed entries of a tile's columns would be scattered
            // writes, so this launch shape computes every entry
            for (void* p : {static_cast<void*>(f->d_koff), static_cast<void*>(f->d_apack),
                            static_cast<void*>(f->d_entry), static_cast<void*>(f->d_b)})
                if (p) (void)hipFree(p);
            f->d_koff = nullptr, f->d_apack = nullptr, f->d_entry = nullptr, f->d_b = nullptr;
            const ffc::TilesF64 t = ffc::make_tiles_f64(rt, f->tile_window, false);
            f->sym_n = 0;
            f->n_tiles = t.n_tiles;
            f->mfma_k = t.koff.back();
            if ((rc = upload(t.koff, &f->d_koff)) || (rc = upload(t.apack, &f->d_apack)) ||
                (rc = upload(t.entry, &f->d_entry)) || (rc = upload(t.b, &f->d_b)))
                return rc;
        }
        const size_t lds = ffc::contract_lds_bytes(spec.dim, spec.kind, f->tile_cells, rt.n_I, rt.n_alpha, f->kpad, bf);
        if (lds > ffc::kLdsBudget) return fail(FFC_E_UNSUPPORTED, "tile does not fit the 160 KiB LDS of a CU");
        // fused: the contraction computes the affine map itself -- the per-tile kernels in LDS
        // per tile, the persistent FP64 kernel one tile ahead (the split-BF16 persistent kernel
        // keeps the pass).  By default not for FP64 tile launches of 16-cell tiles (large
        // tensors the persistent kernel does not take): measured on MI355X, the pass is 17-20%
        // faster there (Laplacian P4 on tetrahedra, 2^18 and 2^19 cells)
        const bool pass_default =
            !bf && f->tile_cells == 16 && (f->tab_tile || (f->pwaves == 0 && rt.n_I >= kPersistentMinEntries));
        f->fused = desc->geometry == FFC_GEOMETRY_FUSED ||
                   (desc->geometry == 0 && !pass_default && !f->bpersistent && (f->pwaves == 0 || f->pwaves == 12));
        if (f->bpersistent || f->pwaves == 16) f->fused = false;
        // the workspace serves the geometry pass, and the persistent operator action
        const bool need_workspace = !f->fused || f->pwaves > 0;
        if (need_workspace && hipMalloc(reinterpret_cast<void**>(&f->d_amap), bytes) != hipSuccess)
            return fail(FFC_E_NOMEM, "hipMalloc failed for the geometry workspace");
    }
    *out = f.release();
    return FFC_OK;
}

int ffc_form_get_info(const ffc_form* form, ffc_form_info* info) {
    if (!form || !info) return fail(FFC_E_INVALID, "NULL argument");
    const ffc_form* f = resolve_default(form);
    const auto& rt = f->rt;
    const int d = f->desc.dim;
    info->n_dofs = rt.n;
    info->n_entries = rt.n_I;
    info->n_alpha = f->n_alpha_form;
    info->nnz_a0 = f->nnz_form;
    info->g_entries = rt.n_alpha;
    info->n_coords = f->desc.kind == FFC_CURVED_LAPLACE ? f->rt.n_geo * d : (d + 1) * d;
    info->n_coeffs = rt.n_coeff;
    info->out_bytes = (f->desc.kernel == FFC_KERNEL_TENSOR && f->desc.precision != FFC_FP64) ? 4 : 8;
    info->mfma_k_per_tile = f->mfma_k;
    info->n_tiles = f->n_tiles;
    info->quad_points = f->quad_npts;
    info->persistent_waves = f->tab_tile ? 0 : f->pwaves;
    info->persistent_kmax = f->pkmax;
    info->tile_cells = f->bpersistent ? f->ptile : (f->pwaves && !f->tab_tile) ? 16 * f->pmt : f->tile_cells;
    info->waves = f->waves;
    info->fused_geometry = f->fused ? 1 : 0;
    info->symmetric = f->sym_n ? 1 : 0;
    info->auto_launches = form->is_auto ? static_cast<int64_t>(form->subs.size()) : 0;
    return FFC_OK;
}

int ffc_form_select(const ffc_form* f, int64_t cells, int32_t* candidate, int32_t* from_selector) {
    if (!f || !candidate) return fail(FFC_E_INVALID, "NULL argument");
    if (!f->is_auto) return fail(FFC_E_INVALID, "not an FFC_KERNEL_AUTO form");
    if (cells < 0) return fail(FFC_E_INVALID, "cells < 0");
    *candidate = f->bucket_cand[auto_bucket(cells)];
    if (from_selector) *from_selector = f->auto_from_selector ? 1 : 0;
    return FFC_OK;
}

void ffc_form_destroy(ffc_form* f) { delete f; }

int ffc_compute_geometry(int32_t dim, int64_t cells, const double* coords, double* affine_map, void* stream) {
    if (dim != 2 && dim != 3) return fail(FFC_E_UNSUPPORTED, "dim must be 2 or 3");
    if (cells < 0) return fail(FFC_E_INVALID, "cells < 0");
    if (cells == 0) return FFC_OK;
    if (!coords || !affine_map) return fail(FFC_E_INVALID, "NULL device pointer");
    int dev;
    int rc = check_device(&dev);
    if (rc) return rc;
    hipError_t e = ffc::launch_geometry(dim, cells, coords, cells, affine_map, cells, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "geometry kernel launch");
    return FFC_OK;
}

int ffc_check_cells(int32_t dim, int64_t cells, const double* coords, double tol, int64_t* count, int64_t* first,
                    void* stream) {
    if (count) *count = 0;
    if (first) *first = -1;
    if (dim != 2 && dim != 3) return fail(FFC_E_UNSUPPORTED, "dim must be 2 or 3");
    if (cells < 0) return fail(FFC_E_INVALID, "cells < 0");
    if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(FFC_E_INVALID, "tol must be finite and >= 0");
    if (cells == 0) return FFC_OK;
    if (!coords) return fail(FFC_E_INVALID, "coords is NULL");
    int dev;
    int rc = check_device(&dev);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    unsigned long long* d_out = nullptr;
    if (hipMalloc(reinterpret_cast<void**>(&d_out), 2 * sizeof(unsigned long long)) != hipSuccess)
        return fail(FFC_E_NOMEM, "hipMalloc failed for the validation counters");
    unsigned long long h_out[2] = {0ull, ~0ull};
    hipError_t e = ffc::launch_degenerate_cells(dim, cells, coords, tol, d_out, s);
    if (e == hipSuccess) e = hipMemcpyAsync(h_out, d_out, sizeof(h_out), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(d_out);
    if (e != hipSuccess) return hip_fail(e, "degenerate-cell check");
    if (count) *count = static_cast<int64_t>(h_out[0]);
    if (first) *first = h_out[0] ? static_cast<int64_t>(h_out[1]) : -1;
    if (h_out[0]) {
        char msg[160];
        std::snprintf(msg, sizeof(msg), "%llu degenerate cell(s) (|det J| <= tol * h^d), the first at index %llu",
                      h_out[0], h_out[1]);
        return fail(FFC_E_DEGENERATE, msg);
    }
    return FFC_OK;
}

namespace {
// contraction of cells [0, n) whose affine map sits at amap with row stride astride
ffc::ContractArgs contract_args(const ffc_form* f, int64_t n, const double* amap, int64_t astride,
                                const double* coeffs, int64_t cstride, void* out) {
    const auto& rt = f->rt;
    ffc::ContractArgs a{};
    a.cells = n;
    a.amap = amap;
    a.astride = astride;
    a.coeffs = coeffs;
    a.cstride = cstride;
    a.out = out;
    a.n_I = rt.n_I;
    a.n_alpha = rt.n_alpha;
    a.n_tiles = f->n_tiles;
    a.lambda = f->desc.lambda;
    a.mu = f->desc.mu;
    a.koff = f->d_koff;
    a.apack = f->d_apack;
    a.entry = f->d_entry;
    a.b = f->d_b;
    a.bb = f->d_bb;
    a.nonzero = f->d_nz;
    a.kpad = f->kpad;
    a.n_seg = f->n_seg;
    a.sym_n = f->sym_n;
    a.geo_grad = f->d_geo_grad;
    a.n_pts = rt.n_pts;
    std::copy(f->gpiece, f->gpiece + 6, a.gpiece);
    return a;
}

int contract_chunk(const ffc_form* f, int64_t n, const double* amap, int64_t astride, const double* coeffs,
                   int64_t cstride, void* out) {
    const bool bf16 = f->desc.precision != FFC_FP64;
    ffc::ContractArgs a = contract_args(f, n, amap, astride, coeffs, cstride, out);
    hipError_t e = hipErrorInvalidValue;
    if (f->bpersistent) {
        e = ffc::launch_contract_bf16_persistent(f->desc.dim, f->desc.kind, f->ptile, f->pgrid, a, f->stream);
    } else if (f->pwaves > 0 && !f->tab_tile) {
        ffc::PersistArgs p{f->d_woff, f->d_wave_b, f->d_wave_word, f->d_wave_mask, f->d_zero, f->n_zero};
        e = ffc::launch_contract_persistent(f->desc.dim, f->desc.kind, f->pkmax, f->pwaves, f->pmt, f->pgrid, a, p,
                                            f->stream);
    }
    if (e == hipErrorInvalidValue)
        e = ffc::launch_contract(f->desc.dim, f->desc.kind, bf16, f->tile_cells, f->waves, a, f->stream);
    if (e != hipSuccess) return hip_fail(e, "contraction kernel launch");
    return FFC_OK;
}
}  // namespace

int ffc_tabulate_tensor_affine(const ffc_form* form, int64_t cells, const double* affine_map, const double* coeffs,
                               void* out) {
    if (!form) return fail(FFC_E_INVALID, "form is NULL");
    const ffc_form* f = resolve_default(form);
    if (f->desc.kernel != FFC_KERNEL_TENSOR) return fail(FFC_E_INVALID, "not a tensor-kernel form");
    if (f->desc.kind == FFC_CURVED_LAPLACE) return fail(FFC_E_UNSUPPORTED, "curvilinear cells have no affine map");
    if (cells < 0) return fail(FFC_E_INVALID, "cells < 0");
    if (cells == 0) return FFC_OK;
    if (!affine_map || !out) return fail(FFC_E_INVALID, "affine_map / out is NULL");
    if (f->rt.n_coeff > 0 && !coeffs) return fail(FFC_E_INVALID, "this form needs coefficients (coeffs is NULL)");
    return contract_chunk(f, cells, affine_map, cells, coeffs, cells, out);
}

namespace {
// launch shape of the operator action's tile kernel: the largest cell tile whose element
// tensors and local vectors fit the LDS (64-cell tiles only while several workgroups stay
// resident per CU)
bool apply_tile_shape(const ffc_form* f, int* tile_cells, int* waves) {
    const auto& rt = f->rt;
    // tiny tensors: 32-cell tiles of one wave up to 9 entries, of two up to 36, so more
    // workgroups stay resident (measured on MI355X at ~10^6 cells against 64-cell tiles of 4
    // waves: Laplacian P1 on triangles 1.8x, P1 on tetrahedra and mass P1 1.5x, Laplacian P2 on
    // triangles 1.3x, elasticity P1 on triangles 1.2x faster)
    if (rt.n_I <= 36 &&
        ffc::plan_lds(f->desc.dim, f->desc.kind, 32, rt.n_I, rt.n_alpha, 0, false, ffc::kLdsBudget).staged &&
        ffc::apply_lds_bytes(f->desc.dim, f->desc.kind, 32, rt.n_I, rt.n_alpha, rt.n) <= 48 * 1024) {
        *tile_cells = 32;
        *waves = rt.n_I <= 9 ? 1 : 2;
        return true;
    }
    for (int ct : {64, 32, 16}) {
        const size_t lds = ffc::apply_lds_bytes(f->desc.dim, f->desc.kind, ct, rt.n_I, rt.n_alpha, rt.n);
        const ffc::LdsPlan p =
            ffc::plan_lds(f->desc.dim, f->desc.kind, ct, rt.n_I, rt.n_alpha, 0, false, ffc::kLdsBudget);
        if (!p.staged || lds > (ct == 64 ? 48 * 1024 : ffc::kLdsBudget)) continue;
        *tile_cells = ct;
        *waves = ct == 64 ? 4 : ct == 32 ? 8 : 16;
        return true;
    }
    return false;
}
}  // namespace

int ffc_apply_tensor(const ffc_form* form, int64_t cells, const double* coords, const double* coeffs, const double* x,
                     double* y) {
    if (!form) return fail(FFC_E_INVALID, "form is NULL");
    const ffc_form* f = resolve_default(form);
    if (f->desc.kernel != FFC_KERNEL_TENSOR || f->desc.precision != FFC_FP64 || f->desc.kind == FFC_CURVED_LAPLACE)
        return fail(FFC_E_UNSUPPORTED, "the operator action needs an FP64 tensor-kernel form on affine cells");
    if (cells < 0) return fail(FFC_E_INVALID, "cells < 0");
    if (cells == 0) return FFC_OK;
    if (!coords || !x || !y) return fail(FFC_E_INVALID, "coords / x / y is NULL");
    const auto& rt = f->rt;
    if (rt.n_coeff > 0 && !coeffs) return fail(FFC_E_INVALID, "this form needs coefficients (coeffs is NULL)");
    const int d = f->desc.dim, kind = f->desc.kind, n = rt.n;
    if (f->pwaves > 0 && f->pmt == 1) {
        hipError_t e = hipSuccess;
        for (int64_t c0 = 0; c0 < cells; c0 += f->amap_cap) {
            const int64_t m = std::min(f->amap_cap, cells - c0);
            e = ffc::launch_geometry(d, m, coords + c0, cells, f->d_amap, f->amap_cap, f->stream);
            if (e != hipSuccess) return hip_fail(e, "geometry kernel launch");
            ffc::ContractArgs a =
                contract_args(f, m, f->d_amap, f->amap_cap, coeffs ? coeffs + c0 : nullptr, cells, y + c0 * n);
            a.xloc = x + c0 * n;
            a.n_dof = n;
            ffc::PersistArgs p{f->d_woff, f->d_wave_b, f->d_wave_word, f->d_wave_mask, f->d_zero, f->n_zero};
            e = ffc::launch_apply_persistent(d, kind, f->pkmax, f->pwaves, f->pgrid, a, p, f->stream);
            if (e == hipErrorInvalidValue) break;  // the form does not fit it: tile kernel below
            if (e != hipSuccess) return hip_fail(e, "operator action kernel launch");
        }
        if (e == hipSuccess) return FFC_OK;
    }
    int ct = 0, w = 0;
    // a launch shape the form was created with (tile_cells and waves both given) when the
    // action's tile fits it, else the action's own choice
    const int dct = f->desc.tile_cells, dw = f->desc.waves;
    if (dct && dw >= 1 && dw <= 16 &&
        ffc::plan_lds(d, kind, dct, rt.n_I, rt.n_alpha, 0, false, ffc::kLdsBudget).staged &&
        ffc::apply_lds_bytes(d, kind, dct, rt.n_I, rt.n_alpha, n) <= ffc::kLdsBudget) {
        ct = dct, w = dw;
    } else if (!apply_tile_shape(f, &ct, &w)) {
        return fail(FFC_E_UNSUPPORTED, "the element tensors of a 16-cell tile do not fit the LDS of a CU");
    }
    ffc::ContractArgs a = contract_args(f, cells, nullptr, 0, coeffs, cells, y);
    a.coords = coords;
    a.xloc = x;
    a.n_dof = n;
    hipError_t e = ffc::launch_apply(d, kind, ct, w, a, f->stream);
    if (e != hipSuccess) return hip_fail(e, "operator action kernel launch");
    return FFC_OK;
}

int ffc_tabulate_tensor(const ffc_form* form, int64_t cells, const double* coords, const double* coeffs, void* out) {
    if (!form) return fail(FFC_E_INVALID, "form is NULL");
    const ffc_form* f = resolve(form, cells);
    if (cells < 0) return fail(FFC_E_INVALID, "cells < 0");
    if (cells == 0) return FFC_OK;
    if (!coords || !out) return fail(FFC_E_INVALID, "coords / out is NULL");
    const auto& rt = f->rt;
    if (rt.n_coeff > 0 && !coeffs) return fail(FFC_E_INVALID, "this form needs coefficients (coeffs is NULL)");
    const int d = f->desc.dim;
    const int kind = f->desc.kind;
    if (f->desc.kernel == FFC_KERNEL_QUADRATURE) {
        ffc::QuadArgs a{};
        a.cells = cells;
        a.coords = coords;
        a.cstride = cells;
        a.coeffs = coeffs;
        a.kstride = cells;
        a.out = static_cast<double*>(out);
        a.ns = rt.ns;
        a.n = rt.n;
        a.n_I = rt.n_I;
        a.npts = f->quad_npts;
        a.pts = f->d_pts;
        a.wts = f->d_wts;
        a.phi = f->d_phi;
        a.dphi = f->d_dphi;
        a.lambda = f->desc.lambda;
        a.mu = f->desc.mu;
        a.cells_per_block = f->quad_cpb;
        hipError_t e = ffc::launch_quadrature(d, kind, a, f->stream);
        if (e != hipSuccess) return hip_fail(e, "quadrature kernel launch");
        return FFC_OK;
    }
    const bool bf16 = f->desc.precision != FFC_FP64;
    const size_t obytes = bf16 ? 4 : 8;
    if (f->fused) {
        // one launch: the contraction computes the affine maps from the coordinates
        ffc::ContractArgs a = contract_args(f, cells, nullptr, 0, coeffs, cells, out);
        a.coords = coords;
        hipError_t e = hipErrorInvalidValue;
        if (f->pwaves > 0 && !bf16 && !f->tab_tile) {
            ffc::PersistArgs p{f->d_woff, f->d_wave_b, f->d_wave_word, f->d_wave_mask, f->d_zero, f->n_zero};
            e = ffc::launch_contract_persistent(d, kind, f->pkmax, f->pwaves, f->pmt, f->pgrid, a, p, f->stream);
        }
        if (e == hipErrorInvalidValue) e = ffc::launch_contract(d, kind, bf16, f->tile_cells, f->waves, a, f->stream);
        if (e != hipSuccess) return hip_fail(e, "contraction kernel launch");
        return FFC_OK;
    }
    for (int64_t c0 = 0; c0 < cells; c0 += f->amap_cap) {
        const int64_t n = std::min(f->amap_cap, cells - c0);
        hipError_t e = kind == FFC_CURVED_LAPLACE
                           ? ffc::launch_curved_geometry(d, n, coords + c0, cells, rt.n_pts, f->d_geo_grad, f->d_amap,
                                                         f->amap_cap, f->stream)
                           : ffc::launch_geometry(d, n, coords + c0, cells, f->d_amap, f->amap_cap, f->stream);
        if (e != hipSuccess) return hip_fail(e, "geometry kernel launch");
        int rc = contract_chunk(f, n, f->d_amap, f->amap_cap, coeffs ? coeffs + c0 : nullptr, cells,
                                static_cast<char*>(out) + static_cast<size_t>(c0) * rt.n_I * obytes);
        if (rc) return rc;
    }
    return FFC_OK;
}

// ------------------------------------------------------------------ batches ----

// One launch of a batch: a tile launch over a group of items, or the persistent launch of
// one form's items.  Each launch has its own device copy of its items' descriptors.
struct BatchLaunch {
    bool persistent = false;
    int dim = 0, kind = 0, kmax = 0;  // persistent launches (FP64 or split BF16 per the batch)
    std::vector<ffc::BatchItem> items;
    ffc::BatchItem* d_items = nullptr;
    int32_t* d_unit_item = nullptr;  // tile launches: [units] item of each tile
    int64_t units = 0;               // tiles
    int waves = 16, mt = 1, grid = 0;  // waves per workgroup; tile launches: tile size 16*mt
    size_t lds = 0;
};

struct ffc_batch {
    std::vector<BatchLaunch> launches;
    struct Geo {
        int dim;
        int64_t cells;
        const double* coords;
        double* amap;
    };
    std::vector<Geo> geometry;  // geometry passes of the persistent items
    double* d_amap = nullptr;
    int64_t total_cells = 0, total_units = 0;
    int nseg = 0;
    hipStream_t stream = nullptr;
    ~ffc_batch() {
        for (auto& l : launches) {
            if (l.d_unit_item) (void)hipFree(l.d_unit_item);
            if (l.d_items) (void)hipFree(l.d_items);
        }
        if (d_amap) (void)hipFree(d_amap);
    }
};

namespace {
// Tile launches are grouped by workgroup size, tile size and the number of workgroups per
// CU that an item's LDS plan allows (1 .. 4), so that each kernel has the register count of
// its own tile and no item runs at a lower occupancy than its own plan gives.
int lds_class(size_t bytes) {
    return static_cast<int>(std::min<size_t>(4, (160 * 1024) / std::max<size_t>(bytes, 1)));
}
}  // namespace

int ffc_batch_create(int32_t n, const ffc_form* const* forms, const int64_t* cells, const double* const* coords,
                     const double* const* coeffs, void* const* outs, void* stream, ffc_batch** out) {
    if (!out) return fail(FFC_E_INVALID, "batch output pointer is NULL");
    *out = nullptr;
    if (n <= 0 || !forms || !cells || !coords || !outs) return fail(FFC_E_INVALID, "empty batch or NULL array");
    int dev;
    int rc = check_device(&dev);
    if (rc) return rc;
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
    std::unique_ptr<ffc_batch> b(new ffc_batch());
    b->stream = static_cast<hipStream_t>(stream);
    bool bf16 = false;
    std::map<const ffc_form*, std::vector<ffc::BatchItem>> pgroups;  // persistent launches, per form
    std::map<int, std::vector<ffc::BatchItem>> tgroups;              // tile launches
    int64_t amap_doubles = 0;
    for (int i = 0; i < n; ++i) {
        const ffc_form* f = resolve_default(forms[i]);
        if (!f) return fail(FFC_E_INVALID, "NULL form in batch");
        if (f->desc.kernel != FFC_KERNEL_TENSOR) return fail(FFC_E_UNSUPPORTED, "batches use the tensor kernel only");
        if (f->desc.kind == FFC_PIOLA_MASS || f->desc.kind == FFC_CURVED_LAPLACE || f->desc.kind == FFC_NEDELEC_MASS)
            return fail(FFC_E_UNSUPPORTED, "batches take Lagrange forms on affine cells only");
        const bool bf = f->desc.precision != FFC_FP64;
        if (i == 0) {
            bf16 = bf;
            b->nseg = bf ? f->n_seg : 0;
        }
        if (bf != bf16 || (bf && f->n_seg != b->nseg))
            return fail(FFC_E_INVALID, "all forms of a batch must share one precision");
        if (cells[i] < 0) return fail(FFC_E_INVALID, "cells < 0");
        if (cells[i] > 0 && (!coords[i] || !outs[i])) return fail(FFC_E_INVALID, "NULL coords / out in batch");
        if (cells[i] > 0 && f->rt.n_coeff > 0 && (!coeffs || !coeffs[i]))
            return fail(FFC_E_INVALID, "batch item needs coefficients");
        b->total_cells += cells[i];
        if (cells[i] == 0) continue;
        const int d = f->desc.dim;
        ffc::BatchItem it{};
        it.cells = cells[i];
        it.coords = coords[i];
        it.coeffs = coeffs ? coeffs[i] : nullptr;
        it.out = outs[i];
        it.dim = d;
        it.kind = f->desc.kind;
        it.n_I = f->rt.n_I;
        it.n_alpha = f->rt.n_alpha;
        it.n_tiles = f->n_tiles;
        it.kpad = f->kpad;
        it.n_seg = f->n_seg;
        it.n_coeff = f->rt.n_coeff;
        it.sym_n = f->sym_n;
        it.koff = f->d_koff;
        it.apack = f->d_apack;
        it.entry = f->d_entry;
        it.b = f->d_b;
        it.bb = f->d_bb;
        it.nonzero = f->d_nz;
        std::copy(f->gpiece, f->gpiece + 6, it.gpiece);
        const bool aligned = (reinterpret_cast<uintptr_t>(outs[i]) & 15u) == 0;
        if (bf && f->bpersistent && aligned) {
            const ffc::LdsPlan pb =
                ffc::plan_bf16_persistent(d, f->desc.kind, f->ptile, f->rt.n_I, f->n_tiles, f->kpad, f->n_seg);
            it.kmax = f->pkmax;
            it.mt = f->ptile / 16;
            it.stage_bytes = pb.stage_bytes;
            it.head_bytes = pb.head_bytes;
            amap_doubles += cells[i] * (1 + d * d);
            pgroups[f].push_back(it);
        } else if (size_t pst = 0, phd = 0;
                   !bf && (f->pwaves == 12 || f->pwaves == 16) && aligned &&
                   ffc::persistent_fits(d, f->desc.kind, f->rt.n_I, f->rt.n_alpha, f->pmt, f->pwaves == 12, &pst, &phd,
                                        nullptr)) {
            // 12-wave schedules: the persistent launch computes each tile's affine map from the
            // coordinates; 16-wave schedules read the maps of a geometry pass
            it.kmax = f->pkmax;
            it.p = ffc::PersistArgs{f->d_woff, f->d_wave_b, f->d_wave_word, f->d_wave_mask, f->d_zero, f->n_zero};
            it.stage_bytes = pst;
            it.head_bytes = phd;
            it.waves = f->pwaves;
            it.mt = f->pmt;
            if (f->pwaves == 16) amap_doubles += cells[i] * (1 + d * d);
            pgroups[f].push_back(it);
        } else {
            const int ct = f->tile_cells;
            it.mt = ct / 16;
            const ffc::LdsPlan pl = ffc::plan_lds(d, f->desc.kind, ct, f->rt.n_I, f->rt.n_alpha, f->kpad, bf,
                                                  ffc::kLdsBudget);
            it.staged = pl.staged && aligned;
            it.stage_bytes = it.staged ? pl.stage_bytes : 0;
            it.head_bytes = pl.head_bytes;
            const size_t lds = it.stage_bytes + pl.head_bytes + pl.g_bytes;
            tgroups[(f->waves << 8) | (it.mt << 4) | lds_class(lds)].push_back(it);
        }
    }
    // geometry workspace of the persistent items
    if (amap_doubles > 0 &&
        hipMalloc(reinterpret_cast<void**>(&b->d_amap), static_cast<size_t>(amap_doubles) * sizeof(double)) != hipSuccess)
        return fail(FFC_E_NOMEM, "hipMalloc failed for the batch geometry workspace");
    int64_t amap_off = 0;
    for (auto& kv : pgroups) {
        BatchLaunch L;
        L.persistent = true;
        L.items = kv.second;
        L.dim = L.items[0].dim;
        L.kind = L.items[0].kind;
        L.kmax = L.items[0].kmax;
        L.mt = L.items[0].mt;
        const int ct = 16 * L.mt;
        if (bf16) {
            L.lds = ffc::plan_bf16_persistent(L.dim, L.kind, ct, L.items[0].n_I, L.items[0].n_tiles, L.items[0].kpad,
                                              L.items[0].n_seg).total;
        } else {
            size_t total = 0;
            ffc::persistent_fits(L.dim, L.kind, L.items[0].n_I, L.items[0].n_alpha, L.mt, L.items[0].waves == 12,
                                 nullptr, nullptr, &total);
            L.lds = total;
        }
        L.waves = bf16 ? 16 : L.items[0].waves;
        for (auto& it : L.items) {
            it.unit_begin = L.units;
            L.units += (it.cells + ct - 1) / ct;
            if (bf16 || L.waves == 16) {  // affine maps from a geometry pass
                it.amap = b->d_amap + amap_off;
                b->geometry.push_back({it.dim, it.cells, it.coords, b->d_amap + amap_off});
                amap_off += it.cells * (1 + it.dim * it.dim);
            }
        }
        // one workgroup per CU (768 or 1024 threads: the register file holds one)
        L.grid = static_cast<int>(std::min<int64_t>(prop.multiProcessorCount, L.units));
        b->launches.push_back(std::move(L));
    }
    for (auto& kv : tgroups) {
        BatchLaunch L;
        L.waves = kv.first >> 8;
        L.mt = (kv.first >> 4) & 15;
        L.items = kv.second;
        std::vector<int32_t> unit_item;
        for (size_t i = 0; i < L.items.size(); ++i) {
            ffc::BatchItem& it = L.items[i];
            const int ct = 16 * it.mt;
            const ffc::LdsPlan pl = ffc::plan_lds(it.dim, it.kind, ct, it.n_I, it.n_alpha, it.kpad, bf16,
                                                  ffc::kLdsBudget);
            L.lds = std::max(L.lds, it.stage_bytes + it.head_bytes + pl.g_bytes);
            it.unit_begin = static_cast<int64_t>(unit_item.size());
            unit_item.insert(unit_item.end(), static_cast<size_t>((it.cells + ct - 1) / ct), static_cast<int32_t>(i));
        }
        if (L.lds > ffc::kLdsBudget) return fail(FFC_E_UNSUPPORTED, "batch tile does not fit LDS");
        L.units = static_cast<int64_t>(unit_item.size());
        if (L.units > INT32_MAX) return fail(FFC_E_UNSUPPORTED, "too many tiles in one batch launch");
        if ((rc = upload(unit_item, &L.d_unit_item))) return rc;
        b->launches.push_back(std::move(L));
    }
    for (auto& L : b->launches) {
        b->total_units += L.units;
        if ((rc = upload(L.items, &L.d_items))) return rc;
    }
    *out = b.release();
    return FFC_OK;
}

int ffc_batch_run(ffc_batch* b) {
    if (!b) return fail(FFC_E_INVALID, "batch is NULL");
    for (const auto& g : b->geometry) {
        hipError_t e = ffc::launch_geometry(g.dim, g.cells, g.coords, g.cells, g.amap, g.cells, b->stream);
        if (e != hipSuccess) return hip_fail(e, "batch geometry launch");
    }
    for (const auto& L : b->launches) {
        hipError_t e = L.persistent
                           ? ffc::launch_batch_persistent(L.dim, L.kind, L.kmax, b->nseg, L.mt, L.waves, L.d_items,
                                                          static_cast<int>(L.items.size()), L.units, L.grid, L.lds,
                                                          b->stream)
                           : ffc::launch_batch_tiles(L.d_items, L.d_unit_item, L.units, L.waves, L.mt, b->nseg,
                                                     L.lds, b->stream);
        if (e != hipSuccess) return hip_fail(e, "batch kernel launch");
    }
    return FFC_OK;
}

int ffc_batch_info(const ffc_batch* b, int64_t* total_cells, int64_t* work_units, int32_t* launches) {
    if (!b) return fail(FFC_E_INVALID, "batch is NULL");
    if (total_cells) *total_cells = b->total_cells;
    if (work_units) *work_units = b->total_units;
    if (launches) *launches = static_cast<int32_t>(b->geometry.size() + b->launches.size());
    return FFC_OK;
}

void ffc_batch_destroy(ffc_batch* b) { delete b; }

// ------------------------------------------------------------------- assembly ----

struct ffc_assembly {
    int64_t cells = 0, n_global = 0, nnz = 0;
    int n = 0, max_row = 0;
    std::vector<int64_t> row_ptr;
    std::vector<int32_t> col;
    uint16_t* d_pos = nullptr;      // [cells][n][n] index of each element-tensor entry within its CSR row
    int64_t* d_row_ptr = nullptr;   // [n_global + 1]
    int64_t* d_slot_ptr = nullptr;  // [n_global + 1]
    int32_t* d_slots = nullptr;     // [cells * n] element-tensor rows per matrix row
    int32_t* d_dofmap = nullptr;    // [cells][n] (operator action: gather of the local vectors)
    hipStream_t stream = nullptr;
    ~ffc_assembly() {
        for (void* p : {static_cast<void*>(d_pos), static_cast<void*>(d_row_ptr), static_cast<void*>(d_slot_ptr),
                        static_cast<void*>(d_slots), static_cast<void*>(d_dofmap)})
            if (p) (void)hipFree(p);
    }
};

int ffc_assembly_create(int64_t cells, int32_t n_local, const int32_t* dofmap, int64_t n_global, void* stream,
                        ffc_assembly** out) {
    if (!out) return fail(FFC_E_INVALID, "assembly output pointer is NULL");
    *out = nullptr;
    if (cells < 0 || n_local <= 0 || n_global <= 0 || n_global > INT32_MAX)
        return fail(FFC_E_INVALID, "bad assembly sizes");
    if (n_local > 64) return fail(FFC_E_UNSUPPORTED, "at most 64 dofs per cell");
    if (cells * n_local > INT32_MAX) return fail(FFC_E_UNSUPPORTED, "cells * n_local must be below 2^31");
    if (cells > 0 && !dofmap) return fail(FFC_E_INVALID, "dofmap is NULL");
    for (int64_t k = 0; k < cells * n_local; ++k)
        if (dofmap[k] < 0 || dofmap[k] >= n_global) return fail(FFC_E_INVALID, "dofmap entry out of [0, n_global)");
    int dev;
    int rc = check_device(&dev);
    if (rc) return rc;
    std::unique_ptr<ffc_assembly> a(new ffc_assembly());
    a->cells = cells;
    a->n = n_local;
    a->n_global = n_global;
    a->stream = static_cast<hipStream_t>(stream);
    std::vector<int64_t> slot_ptr;
    std::vector<int32_t> slots;
    if (!ffc::csr_pattern(cells, n_local, dofmap, n_global, &a->row_ptr, &a->col, &slot_ptr, &slots))
        return fail(FFC_E_UNSUPPORTED, "assembled pattern has 2^31 entries or more");
    a->nnz = a->row_ptr.back();
    for (int64_t r = 0; r < n_global; ++r)
        a->max_row = std::max<int>(a->max_row, static_cast<int>(a->row_ptr[r + 1] - a->row_ptr[r]));
    if (a->max_row > 1024) return fail(FFC_E_UNSUPPORTED, "a matrix row longer than 1024 entries");
    if (cells > 0) {
        int32_t* d_col = nullptr;
        std::vector<int32_t> dm(dofmap, dofmap + cells * n_local);
        const size_t entries = static_cast<size_t>(cells) * n_local * n_local;
        if ((rc = upload(dm, &a->d_dofmap)) || (rc = upload(a->row_ptr, &a->d_row_ptr)) ||
            (rc = upload(a->col, &d_col)) || (rc = upload(slot_ptr, &a->d_slot_ptr)) ||
            (rc = upload(slots, &a->d_slots))) {
            (void)hipFree(d_col);
            return rc;
        }
        hipError_t e = hipMalloc(reinterpret_cast<void**>(&a->d_pos), entries * sizeof(uint16_t));
        if (e == hipSuccess)
            e = ffc::scatter_positions(cells, n_local, a->d_dofmap, a->d_row_ptr, d_col, a->d_pos, a->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(a->stream);
        (void)hipFree(d_col);
        if (e != hipSuccess) return hip_fail(e, "assembly symbolic phase");
    }
    *out = a.release();
    return FFC_OK;
}

int ffc_assembly_info(const ffc_assembly* a, int64_t* n_rows, int64_t* nnz) {
    if (!a) return fail(FFC_E_INVALID, "assembly is NULL");
    if (n_rows) *n_rows = a->n_global;
    if (nnz) *nnz = a->nnz;
    return FFC_OK;
}

int ffc_assembly_pattern(const ffc_assembly* a, int64_t* row_ptr, int32_t* col_idx) {
    if (!a || !row_ptr || (a->nnz > 0 && !col_idx)) return fail(FFC_E_INVALID, "NULL argument");
    std::copy(a->row_ptr.begin(), a->row_ptr.end(), row_ptr);
    std::copy(a->col.begin(), a->col.end(), col_idx);
    return FFC_OK;
}

int ffc_assemble(ffc_assembly* a, const void* element_tensors, int32_t tensor_bytes, double* values,
                 int32_t accumulate) {
    if (!a) return fail(FFC_E_INVALID, "assembly is NULL");
    if (tensor_bytes != 8 && tensor_bytes != 4) return fail(FFC_E_INVALID, "tensor_bytes must be 8 or 4");
    if (a->nnz > 0 && !values) return fail(FFC_E_INVALID, "values is NULL");
    if (a->cells > 0 && !element_tensors) return fail(FFC_E_INVALID, "element_tensors is NULL");
    if (a->cells == 0) return FFC_OK;  // every row is empty
    hipError_t e = ffc::gather_rows(a->n_global, a->n, a->d_slot_ptr, a->d_slots, element_tensors, tensor_bytes,
                                    a->d_pos, a->d_row_ptr, values, accumulate ? 1 : 0, a->max_row, a->stream);
    return e == hipSuccess ? FFC_OK : hip_fail(e, "assembly launch");
}

namespace {
int operator_apply_impl(const ffc_assembly* a, const ffc_form* f, const double* coords, const double* coeffs,
                        const double* x, double* y, double* work) {
    const int64_t m = a->cells * a->n;
    double* xl = work;
    double* yl = work + m;
    hipError_t e = ffc::gather_local(m, a->d_dofmap, x, xl, f->stream);
    if (e != hipSuccess) return hip_fail(e, "gather launch");
    if (a->cells > 0) {
        const int rc = ffc_apply_tensor(f, a->cells, coords, coeffs, xl, yl);
        if (rc) return rc;
    }
    e = ffc::sum_slots(a->n_global, a->d_slot_ptr, a->d_slots, yl, y, f->stream);
    return e == hipSuccess ? FFC_OK : hip_fail(e, "sum launch");
}

int check_operator_args(const ffc_assembly* a, const ffc_form*& f, const double* coords, const double* x,
                        const double* y) {
    f = resolve_default(f);
    if (!a || !f) return fail(FFC_E_INVALID, "assembly / form is NULL");
    if (f->rt.n != a->n) return fail(FFC_E_INVALID, "the form's element dofs differ from the dofmap's");
    if (!x || !y) return fail(FFC_E_INVALID, "x / y is NULL");
    if (a->cells > 0 && !coords) return fail(FFC_E_INVALID, "coords is NULL");
    return FFC_OK;
}

// Scratch of the allocation-free operator: one array per device, in the library's code
// object, loaded with it and kept until the process ends.  In host code `scratch` only
// names the symbol; its device address comes from hipGetSymbolAddress, once per device.
constexpr int64_t kNoallocScratchDoubles = int64_t(1) << 24;  // 128 MiB
static __device__ __align__(256) double scratch[kNoallocScratchDoubles];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_ptr[kMaxDevices] = {};

int scratch_on_current_device(int expected_device, double** out) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    if (dev != expected_device) return fail(FFC_E_INVALID, "call with the form's device current");
    if (dev < 0 || dev >= kMaxDevices) return fail(FFC_E_UNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (!p) return fail(FFC_E_DEVICE, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return FFC_OK;
}
}  // namespace

int ffc_operator_apply(const ffc_assembly* a, const ffc_form* f, const double* coords, const double* coeffs,
                       const double* x, double* y, double* work) {
    int rc = check_operator_args(a, f, coords, x, y);
    if (rc) return rc;
    if (a->cells > 0 && !work) return fail(FFC_E_INVALID, "work is NULL");
    return operator_apply_impl(a, f, coords, coeffs, x, y, work);
}

int ffc_operator_apply_noalloc(const ffc_assembly* a, const ffc_form* f, const double* coords, const double* coeffs,
                               const double* x, double* y) {
    int rc = check_operator_args(a, f, coords, x, y);
    if (rc) return rc;
    if (2 * a->cells * a->n > kNoallocScratchDoubles)
        return fail(FFC_E_UNSUPPORTED, "2 * cells * n_local exceeds the 2^24 doubles of the allocation-free scratch");
    double* work = nullptr;
    if ((rc = scratch_on_current_device(f->device, &work))) return rc;
    return operator_apply_impl(a, f, coords, coeffs, x, y, work);
}

void ffc_assembly_destroy(ffc_assembly* a) { delete a; }

// ------------------------------------------------------------- selector network ----

int64_t ffc_mlp_param_count(int32_t n_in, int32_t n_hidden, int32_t n_out) {
    if (n_in <= 0 || n_hidden <= 0 || n_out <= 0) return fail(FFC_E_INVALID, "MLP sizes must be positive");
    return ffc::mlp_param_count(n_in, n_hidden, n_out);
}

int ffc_mlp_forward(int32_t n_in, int32_t n_hidden, int32_t n_out, int64_t batch, const float* params,
                    const float* x, float* act, float* y, void* stream) {
    if (n_in <= 0 || n_hidden <= 0 || n_out <= 0 || batch < 0) return fail(FFC_E_INVALID, "bad MLP sizes");
    if (batch == 0) return FFC_OK;
    if (!params || !x || !act || !y) return fail(FFC_E_INVALID, "NULL MLP buffer");
    hipError_t e = ffc::mlp_forward(n_in, n_hidden, n_out, batch, params, x, act, y, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? FFC_OK : hip_fail(e, "MLP forward launch");
}

int ffc_mlp_backward(int32_t n_in, int32_t n_hidden, int32_t n_out, int64_t batch, const float* params,
                     const float* x, const float* act, const float* dy, float* grad, float* work, void* stream) {
    if (n_in <= 0 || n_hidden <= 0 || n_out <= 0 || batch <= 0) return fail(FFC_E_INVALID, "bad MLP sizes");
    if (!params || !x || !act || !dy || !grad || !work) return fail(FFC_E_INVALID, "NULL MLP buffer");
    hipError_t e = ffc::mlp_backward(n_in, n_hidden, n_out, batch, params, x, act, dy, grad, work,
                                     static_cast<hipStream_t>(stream));
    return e == hipSuccess ? FFC_OK : hip_fail(e, "MLP backward launch");
}

int ffc_mlp_mse(int64_t n, const float* y, const float* target, const float* mask, float* dy, float* loss,
                void* stream) {
    if (n <= 0 || !y || !target || !mask || !dy || !loss) return fail(FFC_E_INVALID, "bad MSE arguments");
    hipError_t e = ffc::mlp_mse(n, y, target, mask, dy, loss, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? FFC_OK : hip_fail(e, "MSE launch");
}

int ffc_adam_step(int64_t n, float* params, const float* grad, float* m, float* v, float lr, float beta1,
                  float beta2, float eps, float weight_decay, int32_t step, void* stream) {
    if (n <= 0 || !params || !grad || !m || !v || step < 1 || !(weight_decay >= 0.f))
        return fail(FFC_E_INVALID, "bad Adam arguments");
    hipError_t e = ffc::adam_step(n, params, grad, m, v, lr, beta1, beta2, eps, weight_decay, step,
                                  static_cast<hipStream_t>(stream));
    return e == hipSuccess ? FFC_OK : hip_fail(e, "Adam launch");
}

}  // extern "C"
