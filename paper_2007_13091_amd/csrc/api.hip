// C ABI of the UGKWP library (declared in include/ugkwp.h): argument checks, workspace
// carving, uploads and the per-step launch sequence on the caller's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "device_common.hpp"
#include "launch.hpp"
#include "mesh_prep.hpp"
#include "ugkwp.h"

using ugkwp::Dev;
using ugkwp::DevBC;
using ugkwp::HostMesh;
using ugkwp::Scalars;

namespace {
// Measurement support: hip events bracket each group of kernel launches of a step on the
// library's stream; elapsed times are summed when read.
struct EventProf : ugkwp::Prof {
    hipStream_t s = nullptr;
    bool on = false;
    uint32_t mask = 0xFFFFFFFFu;  // slots recorded while on
    std::vector<hipEvent_t> pool;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[ugkwp::kNumSlots];
    hipEvent_t open[ugkwp::kNumSlots] = {};
    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    void begin(int slot) override {
        if (!on || !((mask >> slot) & 1u)) return;
        hipEvent_t e = get();
        if (e) (void)hipEventRecord(e, s);
        open[slot] = e;
    }
    void end(int slot) override {
        if (!on || !open[slot]) return;
        hipEvent_t e = get();
        if (!e) return;
        (void)hipEventRecord(e, s);
        pending[slot].emplace_back(open[slot], e);
        open[slot] = nullptr;
    }
    // sums (ms) and counts per slot; recycles the events
    void drain(double *ms, int64_t *cnt, int n) {
        for (int k = 0; k < ugkwp::kNumSlots; ++k) {
            double acc = 0.0;
            for (auto &pr : pending[k]) {
                float t = 0.f;
                if (hipEventElapsedTime(&t, pr.first, pr.second) == hipSuccess) acc += t;
                pool.push_back(pr.first);
                pool.push_back(pr.second);
            }
            if (k < n) {
                if (ms) ms[k] = acc;
                if (cnt) cnt[k] = (int64_t)pending[k].size();
            }
            pending[k].clear();
        }
    }
    ~EventProf() override {
        for (auto &v : pending)
            for (auto &pr : v) {
                (void)hipEventDestroy(pr.first);
                (void)hipEventDestroy(pr.second);
            }
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};
const char *kSlotNames[ugkwp::kNumSlots] = {"prim_dt", "cell_prep",    "scan_sample", "flux",    "sample",
                                             "stream",  "stream_wall",  "count",       "scan_buckets", "scatter",
                                             "gather",  "finalize"};
}  // namespace

// Workspace of ugkwp_init_mesh_static, for callers that cannot allocate device memory: one
// array per GPU in the library's own device memory, reserved when the code object is loaded
// on that GPU and held until the process ends.  Host code never passes its name to a kernel
// or a copy: the array's device address comes from hipGetSymbolAddress, once per device.
constexpr size_t kStaticWorkspaceBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticWorkspaceBytes];

namespace {
constexpr int kMaxStaticDevices = 64;
std::mutex g_static_mu;
void *g_static_ptr[kMaxStaticDevices] = {};   // device address of `scratch` on each GPU
bool g_static_busy[kMaxStaticDevices] = {};   // a live context uses that GPU's array
}  // namespace

struct ugkwp_ctx {
    int static_dev = -1;  // >= 0: the context lives in that GPU's static workspace
    EventProf prof;
    HostMesh H;
    ugkwp_params p{};                          // instance 0 (shared settings: precision)
    std::vector<ugkwp_params> ps;              // per instance
    std::vector<ugkwp::InstRange> ranges;      // per instance
    hipStream_t stream = nullptr;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    Dev D{};
    int buf = 0;
    ugkwp::LaunchCfg cfg;
    bool have_state = false;
    bool poisoned = false;
    // graph replay: one captured step per starting particle buffer (and per launch sequence)
    bool graph_on = false;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    hipGraphExec_t gexec_wave[2] = {nullptr, nullptr};
    // steps ahead that are wave-only for every instance while no particle exists: they take the
    // shorter launch sequence (the particle kernels would find nothing to do)
    long long wave_only_empty = 0;
    std::string err;
    void drop_graphs() {
        for (auto *gs : {gexec, gexec_wave})
            for (int b = 0; b < 2; ++b)
                if (gs[b]) {
                    (void)hipGraphExecDestroy(gs[b]);
                    gs[b] = nullptr;
                }
    }
    ~ugkwp_ctx() { drop_graphs(); }
};

namespace {

thread_local std::string g_err;

struct Carver {
    char *base;
    size_t off = 0;
    template <typename T>
    T *take(size_t n) {
        off = (off + 255) & ~size_t(255);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += n * sizeof(T);
        return p;
    }
};

// Every cell an axis-aligned box, and each interior face (periodic ones aside) a whole face of
// both its cells: the cell across local face lf (2d low and 2d+1 high side of axis d) then has
// this cell's bounds on the other two axes and, along d, this cell's high bound as its low one
// (or the reverse) and a far bound of its own.  Checked bit for bit on the bounds themselves,
// so that a box built that way during tracking equals the one stored.
static bool conforming_boxes(const HostMesh &H) {
    const size_t nc = (size_t)H.nc;
    for (size_t c = 0; c < nc; ++c)
        if (H.ctype[c] != 8) return false;
    auto same = [](double a, double b) { return std::memcmp(&a, &b, sizeof(double)) == 0; };
    for (size_t c = 0; c < nc; ++c)
        for (int lf = 0; lf < 6; ++lf) {
            const int32_t nb = H.nb[6 * c + lf];
            if (nb < 0 || H.nblf[6 * c + lf] >= ugkwp::kPeriodicEntry) continue;
            const int d = lf >> 1;
            const double *a = &H.box[6 * c], *b = &H.box[6 * (size_t)nb];
            for (int k = 0; k < 3; ++k)
                if (k != d && !(same(a[k], b[k]) && same(a[3 + k], b[3 + k]))) return false;
            if (!((lf & 1) ? same(b[d], a[3 + d]) : same(b[3 + d], a[d]))) return false;
        }
    return true;
}

// Lay the workspace out; with base == nullptr only the size is computed.
size_t carve(const HostMesh &H, int n_inst, long long cap, int prec, bool recon, int K, bool shakhov, Dev &D,
             char *base) {
    Carver C{base};
    D.ip = C.take<ugkwp::InstP>((size_t)n_inst);
    D.is = C.take<ugkwp::InstS>((size_t)n_inst);
    D.cinst = n_inst > 1 ? C.take<int32_t>((size_t)H.nc) : nullptr;
    const size_t nc = (size_t)H.nc, nf = (size_t)H.nf, nbc = H.bcs.size() ? H.bcs.size() : 1;
    D.vol = C.take<double>(nc);
    D.dS = C.take<double>(3 * nc);
    D.orig = C.take<double>(3 * nc);
    D.edge = C.take<double>(9 * nc);
    D.nfc = C.take<uint8_t>(nc);
    D.ctype = C.take<uint8_t>(nc);
    D.box = C.take<double>(6 * nc);
    D.plane = C.take<double4>(6 * nc);
    D.box32 = prec == 1 ? C.take<float>(6 * nc) : nullptr;
    D.plane32 = prec == 1 ? C.take<float4>(6 * nc) : nullptr;
    const bool cb = conforming_boxes(H);
    D.nfar = cb ? C.take<double>(6 * nc) : nullptr;
    D.nfar32 = cb && prec == 1 ? C.take<float>(6 * nc) : nullptr;
    D.nbl = C.take<int2>(6 * nc);
    D.cface = C.take<int32_t>(6 * nc);
    D.fown = C.take<int32_t>(nf);
    D.fnb = C.take<int32_t>(nf);
    D.fn = C.take<double>(3 * nf);
    D.farea = C.take<double>(nf);
    D.bc = C.take<DevBC>(nbc);
    D.xc = recon ? C.take<double>(3 * nc) : nullptr;
    D.lfx = recon ? C.take<double>(18 * nc) : nullptr;
    D.fx = recon ? C.take<double>(3 * nf) : nullptr;
    D.Wh = recon ? C.take<double>(5 * nc) : nullptr;
    D.gW = recon ? C.take<double>(15 * nc) : nullptr;
    D.gH = recon ? C.take<double>(15 * nc) : nullptr;
    D.qh = shakhov ? C.take<double>(3 * nc) : nullptr;
    const size_t nff = (size_t)H.nff;
    D.ffi = C.take<int4>(nff);
    D.ffg = C.take<double>(10 * nff);
    D.bflf = C.take<uint8_t>(H.bf_lf.size());
    D.ninj = C.take<long long>(nff);
    D.injoff = C.take<long long>(nff + 1);
    D.W = C.take<double>(5 * nc);
    D.P = C.take<double>(5 * nc);
    D.nleft = C.take<int32_t>(nc);
    D.tau = C.take<double>(nc);
    D.ec = C.take<double>(nc);
    D.rhoh = C.take<double>(nc);
    D.Phi = C.take<double>(5 * nf);
    D.S = C.take<double>(5 * nc);
    D.nsam = C.take<long long>(nc);
    D.samoff = C.take<long long>(nc + 1);
    D.scan64 = C.take<long long>((size_t)ugkwp::scan_partials_needed((long long)(nc > nff ? nc : nff)));
    D.off = C.take<int32_t>(2 * nc + 1);
    D.scan32 = C.take<int32_t>((size_t)ugkwp::scan_partials_needed(2 * (long long)nc));
    D.spart = C.take<unsigned long long>(128);
    D.cnt64 = C.take<unsigned long long>(2 * nc);
    D.rank = C.take<int32_t>((size_t)(cap + ugkwp::kWallSlack));
    D.wallq = C.take<unsigned int>(ugkwp::kWallSeg);
    D.segoff[0] = C.take<int32_t>(nc + 1);
    D.segoff[1] = C.take<int32_t>(nc + 1);
    D.key = C.take<int32_t>((size_t)cap);
    D.perm = C.take<int32_t>((size_t)cap);
    D.big = C.take<int32_t>(nc);
    for (int b = 0; b < 2; ++b) {
        ugkwp::Particles &P = D.pa[b];
        P.rec = nullptr;
        P.rec32 = nullptr;
        P.m32 = nullptr;
        P.e64 = nullptr;
        P.e32 = nullptr;
        if (prec == 1) {
            P.rec32 = C.take<ugkwp::PRec32>((size_t)cap);
            P.m32 = C.take<float>((size_t)cap);
            if (K > 0) P.e32 = C.take<float>((size_t)cap);
        } else {
            P.rec = C.take<ugkwp::PRec>((size_t)cap);
            if (K > 0) P.e64 = C.take<double>((size_t)cap);
        }
        P.cell = C.take<int32_t>((size_t)cap);
    }
    D.sc = C.take<Scalars>(1);
    D.avgA = C.take<double>(5 * nc);
    D.avgpart = C.take<double>(2 * (size_t)n_inst * ugkwp::kAvgBlocks);
    return (C.off + 255) & ~size_t(255);
}

// the Prandtl number of an instance's collision model: 0 (the default) and 1 are the BGK model
double prandtl_of(const ugkwp_params &p) { return p.prandtl == 0.0 ? 1.0 : p.prandtl; }

// internal degrees of freedom of gamma = (K + 5)/(K + 3), or -1 if gamma is not of that form
int internal_dof(double gamma) {
    if (!(gamma > 1.0)) return -1;
    const double K = 2.0 / (gamma - 1.0) - 3.0;
    const long Ki = std::lround(K);
    if (!(std::fabs(K - (double)Ki) < 1e-9) || Ki < 0 || Ki > ugkwp::kMaxK) return -1;
    return (int)Ki;
}

int32_t check_params(const ugkwp_params &p, int64_t nc, long long &cap, std::string &err) {
    if (internal_dof(p.gamma) < 0) {
        err = "params: gamma must be (K + 5)/(K + 3) for an integer 0 <= K <= 8 (5/3 monatomic, 7/5 diatomic)";
        return UGKWP_E_ARG;
    }
    if (!(p.mu_ref > 0.0) || !std::isfinite(p.omega) || !(p.cfl > 0.0 && p.cfl <= 1.0) || !(p.c2 >= 0.0)) {
        err = "params: need mu_ref > 0, finite omega, 0 < cfl <= 1, c2 >= 0";
        return UGKWP_E_ARG;
    }
    if (p.n_ref < 1 || p.n_ref > (1 << 20) || p.n_min < 0 || p.n_min > (1 << 20) || p.max_crossings < 1) {
        err = "params: need 1 <= n_ref <= 2^20, 0 <= n_min <= 2^20, max_crossings >= 1";
        return UGKWP_E_ARG;
    }
    if (p.recon < 0 || p.recon > 2 || (p.recon == 2 && !(p.venkat_k > 0.0)) ||
        (p.precision != 0 && p.precision != 1)) {
        err = "params: recon is 0, 1 or 2 (2 needs venkat_k > 0); precision is 0 (FP64) or 1 (FP32 form)";
        return UGKWP_E_ARG;
    }
    if (p.gks_steps < 0) {
        err = "params: gks_steps must be >= 0";
        return UGKWP_E_ARG;
    }
    if (p.sampling < 0 || p.sampling > 3 || (p.sampling == 2 && p.recon == 0)) {
        err = "params: sampling is 0 (the pairs of Sec. 2.4(b)), 1 (energy-exact pairs), 2 (first-order g_p of "
              "Sec. 2.3, which needs recon 1 or 2 for the cell gradients) or 3 (independent draws from the "
              "equilibrium of the collision model)";
        return UGKWP_E_ARG;
    }
    const double pr = prandtl_of(p);
    if (!(pr > 0.0 && pr < 2.0)) {
        err = "params: prandtl must be 0 or 1 (the BGK model) or lie in (0, 2) (the Shakhov model)";
        return UGKWP_E_ARG;
    }
    if (pr != 1.0 && (internal_dof(p.gamma) != 0 || p.sampling < 2)) {
        err = "params: the Shakhov model (prandtl != 1) is built for a monatomic gas (gamma 5/3) and draws its "
              "hydro particles one by one (sampling 2 or 3)";
        return UGKWP_E_ARG;
    }
    long long c = p.capacity;
    if (c == 0) {
        long long per = (long long)(p.n_ref > p.n_min ? p.n_ref : p.n_min);
        c = 2 * per * (long long)nc + 65536;
    }
    if (c < 1 || c > 2147483647LL - 1024) {
        err = "params: capacity must fit in a 32-bit particle index";
        return UGKWP_E_ARG;
    }
    cap = c;
    return UGKWP_OK;
}

// Validate and prepare every instance, concatenate them, and total the capacity.
int32_t prepare_batch(const ugkwp_mesh *m, int32_t n_inst, const ugkwp_params *p, HostMesh &H,
                      std::vector<ugkwp::InstRange> &ranges, long long &cap, std::string &err) {
    if (n_inst < 1 || n_inst > 65536) {
        err = "batch: need 1 <= n_inst <= 65536";
        return UGKWP_E_ARG;
    }
    std::vector<HostMesh> parts((size_t)n_inst);
    cap = 0;
    for (int32_t k = 0; k < n_inst; ++k) {
        int32_t st = ugkwp::prepare_mesh(m[k], parts[k], err);
        long long ck = 0;
        if (st == UGKWP_OK) st = check_params(p[k], parts[k].nc, ck, err);
        if (st == UGKWP_OK && parts[k].nper > 0 && p[k].recon != 0) {
            // the least-squares gradients would need the partner's centre shifted
            err = "params: periodic faces need recon = 0 (first order)";
            st = UGKWP_E_ARG;
        }
        if (st == UGKWP_OK && p[k].precision != p[0].precision) {
            err = "params: every instance of a batch must use the same precision";
            st = UGKWP_E_ARG;
        }
        if (st == UGKWP_OK && internal_dof(p[k].gamma) != internal_dof(p[0].gamma)) {
            err = "params: every instance of a batch must have the same gamma (internal degrees of freedom)";
            st = UGKWP_E_ARG;
        }
        if (st != UGKWP_OK) {
            if (n_inst > 1) err = "instance " + std::to_string(k) + ": " + err;
            return st;
        }
        cap += ck;
    }
    if (cap > 2147483647LL - 1024) {
        err = "batch: total capacity must fit in a 32-bit particle index";
        return UGKWP_E_ARG;
    }
    if (n_inst == 1) {
        H = std::move(parts[0]);
        ranges.assign(1, ugkwp::InstRange{0, H.nc, 0, H.nff, 0});
        return UGKWP_OK;
    }
    return ugkwp::concat_meshes(parts, H, ranges, err);
}

int32_t fail(ugkwp_ctx *ctx, int32_t code, const std::string &msg) {
    if (ctx)
        ctx->err = msg;
    else
        g_err = msg;
    return code;
}

#define HIPCHK(ctx, call)                                                                        \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess) return fail((ctx), UGKWP_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <typename T>
hipError_t up(T *dst, const std::vector<T> &src, hipStream_t s) {
    if (src.empty()) return hipSuccess;
    return hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s);
}

// [n][k] row-major host array -> [k][n] column-major
std::vector<double> soa(const std::vector<double> &a, size_t n, size_t k) {
    std::vector<double> o(n * k);
    for (size_t i = 0; i < n; ++i)
        for (size_t j = 0; j < k; ++j) o[j * n + i] = a[i * k + j];
    return o;
}

int32_t device_error_code(uint32_t e) {
    if (e & ugkwp::kErrNonPhys) return UGKWP_E_NONPHYS;
    if (e & ugkwp::kErrLost) return UGKWP_E_LOST;
    if (e & (ugkwp::kErrCapacity | ugkwp::kErrCellCount)) return UGKWP_E_CAPACITY;
    return UGKWP_OK;
}

std::string device_error_text(uint32_t e) {
    std::string s = "device error:";
    if (e & ugkwp::kErrNonPhys) s += " non-physical cell state (rho <= 0 or T <= 0);";
    if (e & ugkwp::kErrLost) s += " a particle exceeded max_crossings;";
    if (e & ugkwp::kErrCapacity) s += " particle capacity exceeded;";
    if (e & ugkwp::kErrCellCount) s += " more than 2^20 particles sampled in one cell;";
    return s;
}

int32_t read_scalars(ugkwp_ctx *ctx, Scalars &s) {
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    HIPCHK(ctx, hipMemcpy(&s, ctx->D.sc, sizeof(Scalars), hipMemcpyDeviceToHost));
    if (s.err) {
        ctx->poisoned = true;
        return fail(ctx, device_error_code(s.err), device_error_text(s.err));
    }
    return UGKWP_OK;
}

}  // namespace

extern "C" {

int32_t ugkwp_workspace_bytes(const ugkwp_mesh *m, int32_t n_inst, const ugkwp_params *p, size_t *bytes) {
    if (!m || !p || !bytes) return fail(nullptr, UGKWP_E_ARG, "null argument");
    HostMesh H;
    std::vector<ugkwp::InstRange> ranges;
    std::string err;
    long long cap = 0;
    int32_t st = prepare_batch(m, n_inst, p, H, ranges, cap, err);
    if (st != UGKWP_OK) return fail(nullptr, st, err);
    Dev D{};
    bool recon = false, shakhov = false;
    for (int32_t k = 0; k < n_inst; ++k) {
        recon = recon || p[k].recon != 0;
        shakhov = shakhov || prandtl_of(p[k]) != 1.0;
    }
    *bytes = carve(H, n_inst, cap, p[0].precision, recon, internal_dof(p[0].gamma), shakhov, D, nullptr);
    return UGKWP_OK;
}

int32_t ugkwp_init_mesh(ugkwp_ctx **out, const ugkwp_mesh *m, int32_t n_inst, const ugkwp_params *p,
                        void *dev_workspace, size_t ws_bytes, void *hip_stream) {
    if (!out || !m || !p || !dev_workspace) return fail(nullptr, UGKWP_E_ARG, "null argument");
    *out = nullptr;
    if (((uintptr_t)dev_workspace & 255) != 0) return fail(nullptr, UGKWP_E_ARG, "workspace must be 256-byte aligned");
    ugkwp_ctx *ctx = new ugkwp_ctx();
    std::string err;
    long long cap = 0;
    int32_t st = prepare_batch(m, n_inst, p, ctx->H, ctx->ranges, cap, err);
    if (st != UGKWP_OK) {
        delete ctx;
        return fail(nullptr, st, err);
    }
    ctx->p = p[0];
    ctx->ps.assign(p, p + n_inst);
    ctx->stream = (hipStream_t)hip_stream;
    ctx->prof.s = ctx->stream;
    ctx->ws = (char *)dev_workspace;
    ctx->ws_bytes = ws_bytes;
    Dev &D = ctx->D;
    bool recon_any = false, recon_all = true, shakhov = false;
    for (int32_t k = 0; k < n_inst; ++k) {
        recon_any = recon_any || p[k].recon != 0;
        recon_all = recon_all && p[k].recon != 0;
        shakhov = shakhov || prandtl_of(p[k]) != 1.0;
    }
    const int K = internal_dof(p[0].gamma);
    size_t need = carve(ctx->H, n_inst, cap, p[0].precision, recon_any, K, shakhov, D, ctx->ws);
    if (ws_bytes < need) {
        delete ctx;
        return fail(nullptr, UGKWP_E_ARG, "workspace too small: need " + std::to_string(need) + " bytes");
    }
    const HostMesh &H = ctx->H;
    D.avg_from = -1;
    D.nc = H.nc;
    D.nf = H.nf;
    D.nbc = (int32_t)H.bcs.size();
    D.nff = H.nff;
    D.n_inst = n_inst;
    D.recon_any = recon_any ? 1 : 0;
    D.recon_all = recon_all ? 1 : 0;
    D.gp_any = 0;
    D.sh_any = 0;
    for (int k = 0; k < n_inst; ++k) {
        D.gp_any = D.gp_any || p[k].sampling >= 2;
        D.sh_any = D.sh_any || prandtl_of(p[k]) != 1.0;
    }
    D.any_diffuse = 0;
    for (const auto &bc : ctx->H.bcs) D.any_diffuse |= bc.type == 1 ? 1 : 0;
    D.all_box = D.nfar != nullptr ? 1 : 0;
    {
        // sparsely filled cells (the tetrahedral runs, ~50 particles each) give a block of the
        // bucket count many distinct keys: smaller blocks and a higher occupancy pay there;
        // dense cells keep the larger blocks (fewer global atomics per key)
        double per_cell = 0.0;
        for (int k = 0; k < n_inst; ++k)
            per_cell += (double)(ctx->ranges[k].cell1 - ctx->ranges[k].cell0) * std::max(p[k].n_ref, p[k].n_min);
        D.count_ch = per_cell < 128.0 * (double)H.nc ? 4 : 8;
    }
    D.cap = cap;
    D.prec = p[0].precision;
    D.K = K;
    std::vector<ugkwp::InstP> ip((size_t)n_inst);
    std::vector<int32_t> cinst;
    if (n_inst > 1) cinst.resize((size_t)H.nc);
    for (int32_t k = 0; k < n_inst; ++k) {
        const ugkwp::InstRange &r = ctx->ranges[k];
        ugkwp::InstP &q = ip[k];
        std::memset(&q, 0, sizeof(q));
        q.mu_ref = p[k].mu_ref;
        q.omega = p[k].omega;
        q.cfl = p[k].cfl;
        q.c2 = p[k].c2;
        q.n_ref = p[k].n_ref;
        q.n_min = p[k].n_min;
        q.max_cross = p[k].max_crossings;
        q.recon = p[k].recon;
        q.venkat_k = p[k].venkat_k;
        q.seed = p[k].seed;
        q.sampling = p[k].sampling;
        q.gks_steps = p[k].gks_steps;
        q.pr = prandtl_of(p[k]);
        q.cell0 = r.cell0;
        q.cell1 = r.cell1;
        q.ff0 = r.ff0;
        q.ff1 = r.ff1;
        q.bf0 = r.bf0;
        for (int32_t c = r.cell0; c < r.cell1 && n_inst > 1; ++c) cinst[c] = k;
    }

    hipStream_t s = ctx->stream;
    const size_t nc = (size_t)H.nc, nf = (size_t)H.nf;
    std::vector<double> dS = soa(H.dS, nc, 3), org = soa(H.orig, nc, 3), edg = soa(H.edge, nc, 9), fn = soa(H.fn, nf, 3);
    std::vector<int2> nbl(6 * nc);
    for (size_t i = 0; i < 6 * nc; ++i) nbl[i] = make_int2(H.nb[i], H.nblf[i]);
    std::vector<DevBC> bcs(H.bcs.size() ? H.bcs.size() : 1);
    std::memset(bcs.data(), 0, bcs.size() * sizeof(DevBC));
    for (size_t b = 0; b < H.bcs.size(); ++b) {
        bcs[b].type = H.bcs[b].type;
        bcs[b].Tw = H.bcs[b].T_w;
        for (int d = 0; d < 3; ++d) bcs[b].Uw[d] = H.bcs[b].U_w[d];
        for (int k = 0; k < 5; ++k) bcs[b].Winf[k] = H.bcs[b].W_inf[k];
        for (int d = 0; d < 3; ++d) bcs[b].shift[d] = H.bcs[b].shift[d];
    }
    std::vector<int4> ffi((size_t)H.nff);
    for (int32_t j = 0; j < H.nff; ++j) ffi[j] = make_int4(H.ff_cell[j], H.ff_lf[j] | (H.ff_tri[j] << 8), H.ff_bf[j], H.ff_bc[j]);
    auto cleanup_fail = [&](const std::string &msg) {
        delete ctx;
        return fail(nullptr, UGKWP_E_DEVICE, msg);
    };
    hipError_t e = hipSuccess;
    e = e ? e : up((double *)D.vol, H.vol, s);
    e = e ? e : up((double *)D.dS, dS, s);
    e = e ? e : up((double *)D.orig, org, s);
    e = e ? e : up((double *)D.box, H.box, s);
    std::vector<float> box32, plane32;
    if (D.prec == 1) {
        box32.assign(H.box.begin(), H.box.end());
        plane32.assign(H.plane.begin(), H.plane.end());
        e = e ? e : up((float *)D.box32, box32, s);
        e = e ? e : hipMemcpyAsync((void *)D.plane32, plane32.data(), plane32.size() * sizeof(float), hipMemcpyHostToDevice, s);
    }
    e = e ? e : up((double *)D.edge, edg, s);
    e = e ? e : up((uint8_t *)D.nfc, H.nfc, s);
    e = e ? e : up((uint8_t *)D.ctype, H.ctype, s);
    e = e ? e : hipMemcpyAsync((void *)D.plane, H.plane.data(), H.plane.size() * sizeof(double), hipMemcpyHostToDevice, s);
    e = e ? e : up((int2 *)D.nbl, nbl, s);
    std::vector<double> far;  // (host copies live until the synchronisation below)
    std::vector<float> far32;
    if (D.all_box) {
        far.assign(6 * nc, 0.0);
        for (size_t i = 0; i < 6 * nc; ++i) {
            const int32_t nb = H.nb[i];
            if (nb < 0 || H.nblf[i] >= ugkwp::kPeriodicEntry) continue;
            const int lf = (int)(i % 6), d = lf >> 1;
            far[i] = H.box[6 * (size_t)nb + ((lf & 1) ? 3 + d : d)];
        }
        e = e ? e : up((double *)D.nfar, far, s);
        if (D.prec == 1) {
            far32.assign(far.begin(), far.end());
            e = e ? e : up((float *)D.nfar32, far32, s);
        }
    }
    e = e ? e : up((int32_t *)D.cface, H.cface, s);
    e = e ? e : up((int32_t *)D.fown, H.fown, s);
    e = e ? e : up((int32_t *)D.fnb, H.fnb, s);
    e = e ? e : up((double *)D.fn, fn, s);
    e = e ? e : up((double *)D.farea, H.farea, s);
    e = e ? e : up((DevBC *)D.bc, bcs, s);
    e = e ? e : up((int4 *)D.ffi, ffi, s);
    e = e ? e : up((double *)D.ffg, H.ff_geo, s);
    e = e ? e : up((uint8_t *)D.bflf, H.bf_lf, s);
    e = e ? e : up((ugkwp::InstP *)D.ip, ip, s);
    std::vector<double> xcs, fxs;
    if (recon_any) {
        xcs = soa(H.xc, nc, 3);
        fxs = soa(H.fx, nf, 3);
        e = e ? e : up((double *)D.xc, xcs, s);
        e = e ? e : up((double *)D.lfx, H.lfx, s);
        e = e ? e : up((double *)D.fx, fxs, s);
    }
    if (n_inst > 1) e = e ? e : up((int32_t *)D.cinst, cinst, s);
    e = e ? e : hipStreamSynchronize(s);
    if (e != hipSuccess) return cleanup_fail(std::string("upload: ") + hipGetErrorString(e));
    *out = ctx;
    return UGKWP_OK;
}

int32_t ugkwp_init_state(ugkwp_ctx *ctx, const double *W0) {
    if (!ctx || !W0) return fail(ctx, UGKWP_E_ARG, "null argument");
    const size_t nc = (size_t)ctx->H.nc;
    for (size_t c = 0; c < nc; ++c) {
        const double *w = W0 + 5 * c;
        double rho = w[0];
        double T = (2.0 / (3.0 + ctx->D.K)) * (w[4] - 0.5 * (w[1] * w[1] + w[2] * w[2] + w[3] * w[3]) / rho) / rho;
        if (!(rho > 0.0) || !(T > 0.0) || !std::isfinite(rho) || !std::isfinite(T))
            return fail(ctx, UGKWP_E_NONPHYS, "init_state: cell " + std::to_string(c) + " has rho <= 0 or T <= 0");
    }
    std::vector<double> Wt(5 * nc);
    for (size_t c = 0; c < nc; ++c)
        for (int k = 0; k < 5; ++k) Wt[k * nc + c] = W0[5 * c + k];
    Dev &D = ctx->D;
    hipStream_t s = ctx->stream;
    Scalars sc;
    std::memset(&sc, 0, sizeof(sc));
    sc.dtmin_bits = 0x7FF0000000000000ULL;
    HIPCHK(ctx, up(D.W, Wt, s));
    ugkwp::launch_fill_f64(D.P, 5 * (long long)nc, 0.0, s);
    ugkwp::launch_fill_i32(D.nleft, (long long)nc, 0, s);
    ugkwp::launch_fill_i32(D.segoff[0], (long long)nc + 1, 0, s);
    ugkwp::launch_fill_i32(D.segoff[1], (long long)nc + 1, 0, s);
    ugkwp::launch_fill_f64(D.avgA, 5 * (long long)nc, 0.0, s);
    ugkwp::launch_heat(D, 0, s);  // no particle yet: zero heat fluxes
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, hipMemcpyAsync(D.sc, &sc, sizeof(sc), hipMemcpyHostToDevice, s));
    std::vector<ugkwp::InstS> is((size_t)D.n_inst);
    std::memset(is.data(), 0, is.size() * sizeof(ugkwp::InstS));
    for (auto &v : is) v.dtmin_bits = 0x7FF0000000000000ULL;
    HIPCHK(ctx, up(D.is, is, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    ctx->buf = 0;
    ctx->have_state = true;
    ctx->poisoned = false;
    long long wo = ctx->ps.empty() ? 0 : (long long)ctx->ps[0].gks_steps;
    for (const auto &q : ctx->ps) wo = std::min(wo, (long long)q.gks_steps);
    ctx->wave_only_empty = wo;
    return UGKWP_OK;
}

int32_t ugkwp_step(ugkwp_ctx *ctx, int32_t n_steps, ugkwp_step_stats *stats) {
    if (!ctx || n_steps < 0) return fail(ctx, UGKWP_E_ARG, "bad argument");
    if (!ctx->have_state) return fail(ctx, UGKWP_E_STATE, "step before init_state");
    if (ctx->poisoned) return fail(ctx, UGKWP_E_STATE, "context poisoned by an earlier device error; call init_state");
    for (int32_t i = 0; i < n_steps; ++i) {
        const bool wave = ctx->wave_only_empty > 0;
        if (ctx->graph_on) {
            hipGraphExec_t &ge = wave ? ctx->gexec_wave[ctx->buf] : ctx->gexec[ctx->buf];
            if (!ge) {
                // capture the launch sequence of a step once; every count it needs is read
                // on the device, so the same graph serves every later step
                hipGraph_t g = nullptr;
                HIPCHK(ctx, hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
                if (wave)
                    ugkwp::launch_step_wave_only(ctx->D, ctx->buf, ctx->cfg, ctx->stream, nullptr);
                else
                    ugkwp::launch_step(ctx->D, ctx->buf, ctx->cfg, ctx->stream, nullptr);
                hipError_t e = hipStreamEndCapture(ctx->stream, &g);
                if (e != hipSuccess) return fail(ctx, UGKWP_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
                e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (e != hipSuccess) {
                    ge = nullptr;
                    return fail(ctx, UGKWP_E_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
                }
            }
            HIPCHK(ctx, hipGraphLaunch(ge, ctx->stream));
        } else if (wave) {
            ugkwp::launch_step_wave_only(ctx->D, ctx->buf, ctx->cfg, ctx->stream, &ctx->prof);
        } else {
            ugkwp::launch_step(ctx->D, ctx->buf, ctx->cfg, ctx->stream, &ctx->prof);
        }
        ctx->buf ^= 1;
        if (ctx->wave_only_empty > 0) --ctx->wave_only_empty;
    }
    HIPCHK(ctx, hipGetLastError());
    if (stats) {
        Scalars s;
        int32_t st = read_scalars(ctx, s);
        std::memset(stats, 0, sizeof(*stats));
        stats->dt = s.dt;
        stats->t = s.t;
        stats->step = s.step;
        stats->n_alive = s.n_alive;
        stats->n_sampled = (int64_t)s.n_sampled;
        stats->n_collided = (int64_t)s.n_collided;
        stats->n_escaped = (int64_t)s.n_escaped;
        stats->crossings = (int64_t)s.n_cross;
        stats->wall_hits = (int64_t)s.n_wall;
        stats->error_word = s.err;
        stats->moved_total = (int64_t)s.moved_total;
        stats->n_injected = (int64_t)s.n_injected;
        stats->max_crossings_seen = (int64_t)s.max_cross;
        // particles streamed in the last step: those alive at its start, the sampled and the
        // entering ones
        stats->n_moved = s.n_alive + (int64_t)s.n_collided + (int64_t)s.n_escaped;
        if (st != UGKWP_OK) return st;
    }
    return UGKWP_OK;
}

int32_t ugkwp_instance_stats(ugkwp_ctx *ctx, int32_t inst, ugkwp_step_stats *stats) {
    if (!ctx || !stats || inst < 0 || inst >= ctx->D.n_inst) return fail(ctx, UGKWP_E_ARG, "bad argument");
    if (!ctx->have_state) return fail(ctx, UGKWP_E_STATE, "no state");
    Scalars s;
    int32_t st = read_scalars(ctx, s);
    ugkwp::InstS I;
    HIPCHK(ctx, hipMemcpy(&I, ctx->D.is + inst, sizeof(I), hipMemcpyDeviceToHost));
    std::memset(stats, 0, sizeof(*stats));
    stats->dt = I.dt;
    stats->t = I.t;
    stats->step = I.step;
    stats->n_alive = I.n_alive;
    stats->n_sampled = I.n_sampled;
    stats->n_injected = I.n_injected;
    stats->n_collided = I.n_collided;
    stats->n_escaped = I.n_escaped;
    stats->n_moved = I.n_alive + I.n_collided + I.n_escaped;
    stats->moved_total = I.moved_total;
    stats->crossings = ctx->D.n_inst > 1 ? -1 : (int64_t)s.n_cross;
    stats->wall_hits = ctx->D.n_inst > 1 ? -1 : (int64_t)s.n_wall;
    stats->max_crossings_seen = ctx->D.n_inst > 1 ? -1 : (int64_t)s.max_cross;
    stats->error_word = s.err;
    return st;
}

int32_t ugkwp_instance_cells(const ugkwp_ctx *ctx, int32_t inst, int64_t *cell0, int64_t *cell1) {
    if (!ctx || !cell0 || !cell1 || inst < 0 || inst >= (int32_t)ctx->ranges.size())
        return fail(nullptr, UGKWP_E_ARG, "bad argument");
    *cell0 = ctx->ranges[inst].cell0;
    *cell1 = ctx->ranges[inst].cell1;
    return UGKWP_OK;
}

int32_t ugkwp_moments(ugkwp_ctx *ctx, int32_t which, double *out, int32_t out_is_device) {
    if (!ctx || !out || which < 0 || which > 3) return fail(ctx, UGKWP_E_ARG, "bad argument");
    if (!ctx->have_state) return fail(ctx, UGKWP_E_STATE, "moments before init_state");
    Dev &D = ctx->D;
    double *scratch = D.S;  // [5][nc] per-step scratch, free between steps
    ugkwp::launch_moments(D, which, scratch, ctx->stream);
    HIPCHK(ctx, hipGetLastError());
    size_t bytes = sizeof(double) * 5 * (size_t)D.nc;
    HIPCHK(ctx, hipMemcpyAsync(out, scratch, bytes, out_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                               ctx->stream));
    Scalars s;
    return read_scalars(ctx, s);
}

int32_t ugkwp_set_averaging(ugkwp_ctx *ctx, int64_t n_avg) {
    if (!ctx) return fail(ctx, UGKWP_E_ARG, "null argument");
    Dev &D = ctx->D;
    D.avg_from = n_avg < 0 ? -1 : (long long)n_avg;
    ctx->drop_graphs();  // a captured step holds the old setting
    if (!ctx->have_state) return UGKWP_OK;  // ugkwp_init_state clears the sums
    hipStream_t s = ctx->stream;
    ugkwp::launch_fill_f64(D.avgA, 5 * (long long)D.nc, 0.0, s);
    HIPCHK(ctx, hipGetLastError());
    std::vector<ugkwp::InstS> is((size_t)D.n_inst);
    HIPCHK(ctx, hipMemcpyAsync(is.data(), D.is, is.size() * sizeof(ugkwp::InstS), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    for (auto &v : is) {
        v.avg_D = 0.0;
        v.avg_n = 0;
        v.avg_res = 0.0;
    }
    HIPCHK(ctx, up(D.is, is, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    return UGKWP_OK;
}

int32_t ugkwp_average(ugkwp_ctx *ctx, double *Wbar, int32_t out_is_device, double *residual, int64_t *n_averaged) {
    if (!ctx) return fail(ctx, UGKWP_E_ARG, "null argument");
    if (!ctx->have_state) return fail(ctx, UGKWP_E_STATE, "average before init_state");
    Dev &D = ctx->D;
    if (D.avg_from < 0) return fail(ctx, UGKWP_E_STATE, "time averaging is off (ugkwp_set_averaging)");
    hipStream_t s = ctx->stream;
    std::vector<ugkwp::InstS> is((size_t)D.n_inst);
    HIPCHK(ctx, hipMemcpyAsync(is.data(), D.is, is.size() * sizeof(ugkwp::InstS), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    for (const auto &v : is)
        if (v.avg_n < 1) return fail(ctx, UGKWP_E_STATE, "no step has been averaged yet");
    if (Wbar) {
        double *scratch = D.S;  // [5][nc] per-step scratch, free between steps
        ugkwp::launch_avg_out(D, scratch, s);
        HIPCHK(ctx, hipGetLastError());
        HIPCHK(ctx, hipMemcpyAsync(Wbar, scratch, sizeof(double) * 5 * (size_t)D.nc,
                                   out_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
    }
    for (size_t i = 0; i < is.size(); ++i) {
        if (residual) residual[i] = is[i].avg_n >= 2 ? is[i].avg_res : HUGE_VAL;
        if (n_averaged) n_averaged[i] = is[i].avg_n;
    }
    Scalars sc;
    return read_scalars(ctx, sc);
}

int32_t ugkwp_particle_count(ugkwp_ctx *ctx, int64_t *n) {
    if (!ctx || !n) return fail(ctx, UGKWP_E_ARG, "bad argument");
    if (!ctx->have_state) return fail(ctx, UGKWP_E_STATE, "no state");
    Scalars s;
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    HIPCHK(ctx, hipMemcpy(&s, ctx->D.sc, sizeof(Scalars), hipMemcpyDeviceToHost));
    *n = s.n_old;
    return UGKWP_OK;
}

int32_t ugkwp_export_particles(ugkwp_ctx *ctx, double *x, double *u, double *m, int32_t *cell, uint64_t *uid,
                               double *e) {
    if (!ctx) return fail(ctx, UGKWP_E_ARG, "bad argument");
    int64_t n = 0;
    int32_t st = ugkwp_particle_count(ctx, &n);
    if (st != UGKWP_OK) return st;
    const ugkwp::Particles &P = ctx->D.pa[ctx->buf];
    if (n > 0 && ctx->D.prec == 1) {
        std::vector<ugkwp::PRec32> rec((size_t)n);
        std::vector<float> mm((size_t)n);
        HIPCHK(ctx, hipMemcpy(rec.data(), P.rec32, n * sizeof(ugkwp::PRec32), hipMemcpyDeviceToHost));
        HIPCHK(ctx, hipMemcpy(mm.data(), P.m32, n * sizeof(float), hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < n; ++i) {
            for (int d = 0; d < 3; ++d) {
                if (x) x[3 * i + d] = rec[i].x[d];
                if (u) u[3 * i + d] = rec[i].u[d];
            }
            if (m) m[i] = mm[i];
            if (uid) uid[i] = rec[i].uid;
        }
        if (cell) HIPCHK(ctx, hipMemcpy(cell, P.cell, n * sizeof(int32_t), hipMemcpyDeviceToHost));
        if (e && P.e32) {
            std::vector<float> ee((size_t)n);
            HIPCHK(ctx, hipMemcpy(ee.data(), P.e32, n * sizeof(float), hipMemcpyDeviceToHost));
            for (int64_t i = 0; i < n; ++i) e[i] = ee[i];
        } else if (e) {
            for (int64_t i = 0; i < n; ++i) e[i] = 0.0;
        }
    } else if (n > 0) {
        std::vector<ugkwp::PRec> rec((size_t)n);
        HIPCHK(ctx, hipMemcpy(rec.data(), P.rec, n * sizeof(ugkwp::PRec), hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < n; ++i) {
            for (int d = 0; d < 3; ++d) {
                if (x) x[3 * i + d] = rec[i].x[d];
                if (u) u[3 * i + d] = rec[i].u[d];
            }
            if (m) m[i] = rec[i].m;
            if (uid) uid[i] = rec[i].uid;
        }
        if (cell) HIPCHK(ctx, hipMemcpy(cell, P.cell, n * sizeof(int32_t), hipMemcpyDeviceToHost));
        if (e && P.e64) {
            HIPCHK(ctx, hipMemcpy(e, P.e64, n * sizeof(double), hipMemcpyDeviceToHost));
        } else if (e) {
            for (int64_t i = 0; i < n; ++i) e[i] = 0.0;
        }
    }
    return UGKWP_OK;
}

int32_t ugkwp_export_state(ugkwp_ctx *ctx, double *W, double *P, int64_t *step, double *t) {
    if (!ctx) return fail(ctx, UGKWP_E_ARG, "bad argument");
    if (!ctx->have_state) return fail(ctx, UGKWP_E_STATE, "export before init_state");
    Dev &D = ctx->D;
    const size_t nc = (size_t)D.nc;
    hipStream_t s = ctx->stream;
    Scalars sc;
    int32_t st = read_scalars(ctx, sc);
    if (st != UGKWP_OK) return st;
    std::vector<double> buf(5 * nc);
    const double *src[2] = {D.W, D.P};
    double *dst[2] = {W, P};
    for (int q = 0; q < 2; ++q) {
        if (!dst[q]) continue;
        HIPCHK(ctx, hipMemcpyAsync(buf.data(), src[q], 5 * nc * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(ctx, hipStreamSynchronize(s));
        for (size_t c = 0; c < nc; ++c)
            for (int k = 0; k < 5; ++k) dst[q][5 * c + k] = buf[k * nc + c];
    }
    if (step || t) {
        std::vector<ugkwp::InstS> is((size_t)D.n_inst);
        HIPCHK(ctx, hipMemcpyAsync(is.data(), D.is, is.size() * sizeof(ugkwp::InstS), hipMemcpyDeviceToHost, s));
        HIPCHK(ctx, hipStreamSynchronize(s));
        for (size_t k = 0; k < is.size(); ++k) {
            if (step) step[k] = is[k].step;
            if (t) t[k] = is[k].t;
        }
    }
    return UGKWP_OK;
}

int32_t ugkwp_import_state(ugkwp_ctx *ctx, const double *W, const double *P, int64_t n, const double *x,
                           const double *u, const double *m, const int32_t *cell, const uint64_t *uid,
                           const double *e, const int64_t *step, const double *t) {
    if (!ctx || !W || !P || !step || !t || n < 0 || (n > 0 && (!x || !u || !m || !cell || !uid)))
        return fail(ctx, UGKWP_E_ARG, "import_state: null argument or negative particle count");
    Dev &D = ctx->D;
    const size_t nc = (size_t)D.nc;
    if (n > D.cap) return fail(ctx, UGKWP_E_CAPACITY, "import_state: more particles than the capacity");
    for (size_t c = 0; c < nc; ++c) {
        const double *w = W + 5 * c;
        const double rho = w[0];
        const double T = (2.0 / (3.0 + D.K)) * (w[4] - 0.5 * (w[1] * w[1] + w[2] * w[2] + w[3] * w[3]) / rho) / rho;
        if (!(rho > 0.0) || !(T > 0.0) || !std::isfinite(rho) || !std::isfinite(T))
            return fail(ctx, UGKWP_E_NONPHYS, "import_state: cell " + std::to_string(c) + " has rho <= 0 or T <= 0");
    }
    // particles grouped by cell: cell indices non-decreasing and in range
    std::vector<int32_t> cnt(nc, 0), seg(nc + 1, 0);
    for (int64_t i = 0; i < n; ++i) {
        if (cell[i] < 0 || (size_t)cell[i] >= nc || (i > 0 && cell[i] < cell[i - 1]))
            return fail(ctx, UGKWP_E_ARG, "import_state: particle " + std::to_string(i) +
                                              ": cells must be in range and non-decreasing (grouped by cell)");
        ++cnt[(size_t)cell[i]];
    }
    for (size_t c = 0; c < nc; ++c) seg[c + 1] = seg[c] + cnt[c];
    for (int32_t k = 0; k < D.n_inst; ++k)
        if (step[k] < 0 || step[k] >= (1LL << 19) || !std::isfinite(t[k]) || t[k] < 0.0)
            return fail(ctx, UGKWP_E_ARG, "import_state: step must be in [0, 2^19) and t finite and >= 0");
    hipStream_t s = ctx->stream;
    const int b = ctx->buf;
    const ugkwp::Particles &pa = D.pa[b];
    std::vector<double> Wt(5 * nc), Pt(5 * nc);
    for (size_t c = 0; c < nc; ++c)
        for (int k = 0; k < 5; ++k) {
            Wt[k * nc + c] = W[5 * c + k];
            Pt[k * nc + c] = P[5 * c + k];
        }
    HIPCHK(ctx, up(D.W, Wt, s));
    HIPCHK(ctx, up(D.P, Pt, s));
    HIPCHK(ctx, up(D.nleft, cnt, s));
    HIPCHK(ctx, up(D.segoff[b], seg, s));
    std::vector<ugkwp::PRec> rec;
    std::vector<ugkwp::PRec32> rec32;
    std::vector<float> m32;
    if (n > 0) {
        if (D.prec == 1) {
            rec32.resize((size_t)n);
            m32.resize((size_t)n);
            for (int64_t i = 0; i < n; ++i) {
                for (int d = 0; d < 3; ++d) {
                    rec32[i].x[d] = (float)x[3 * i + d];
                    rec32[i].u[d] = (float)u[3 * i + d];
                }
                rec32[i].uid = uid[i];
                m32[i] = (float)m[i];
            }
            HIPCHK(ctx, up(pa.rec32, rec32, s));
            HIPCHK(ctx, up(pa.m32, m32, s));
            if (pa.e32) {
                std::vector<float> e32((size_t)n);
                for (int64_t i = 0; i < n; ++i) e32[i] = e ? (float)e[i] : 0.0f;
                HIPCHK(ctx, up(pa.e32, e32, s));
            }
        } else {
            rec.resize((size_t)n);
            for (int64_t i = 0; i < n; ++i) {
                for (int d = 0; d < 3; ++d) {
                    rec[i].x[d] = x[3 * i + d];
                    rec[i].u[d] = u[3 * i + d];
                }
                rec[i].m = m[i];
                rec[i].uid = uid[i];
            }
            HIPCHK(ctx, up(pa.rec, rec, s));
            if (pa.e64) {
                std::vector<double> e64((size_t)n);
                for (int64_t i = 0; i < n; ++i) e64[i] = e ? e[i] : 0.0;
                HIPCHK(ctx, up(pa.e64, e64, s));
            }
        }
        HIPCHK(ctx, hipMemcpyAsync(pa.cell, cell, (size_t)n * sizeof(int32_t), hipMemcpyHostToDevice, s));
    }
    // step bookkeeping as after a step: the particles are the old ones of the next step
    Scalars sc;
    std::memset(&sc, 0, sizeof(sc));
    sc.dtmin_bits = 0x7FF0000000000000ULL;
    sc.n_old = n;
    sc.n_alive = n;
    sc.step = step[0];
    sc.t = t[0];
    HIPCHK(ctx, hipMemcpyAsync(D.sc, &sc, sizeof(sc), hipMemcpyHostToDevice, s));
    std::vector<ugkwp::InstS> is((size_t)D.n_inst);
    std::memset(is.data(), 0, is.size() * sizeof(ugkwp::InstS));
    for (int32_t k = 0; k < D.n_inst; ++k) {
        const ugkwp::InstRange &r = ctx->ranges[k];
        is[k].dtmin_bits = 0x7FF0000000000000ULL;
        is[k].step = step[k];
        is[k].t = t[k];
        is[k].n_alive = seg[(size_t)r.cell1] - seg[(size_t)r.cell0];
    }
    HIPCHK(ctx, up(D.is, is, s));
    ugkwp::launch_fill_f64(D.avgA, 5 * (long long)nc, 0.0, s);
    ugkwp::launch_heat(D, b, s);  // the imported particles' heat fluxes (Shakhov model)
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, hipStreamSynchronize(s));
    ctx->have_state = true;
    ctx->poisoned = false;
    // wave-only steps ahead of every instance, if no particle was imported
    long long wo = n > 0 ? 0 : (long long)1 << 62;
    for (int32_t k = 0; k < D.n_inst && wo > 0; ++k)
        wo = std::min(wo, std::max(0LL, (long long)ctx->ps[k].gks_steps - (long long)step[k]));
    ctx->wave_only_empty = wo;
    return UGKWP_OK;
}

int32_t ugkwp_geometry(ugkwp_ctx *ctx, double *vol, double *xc, double *dS) {
    if (!ctx) return fail(ctx, UGKWP_E_ARG, "bad argument");
    const HostMesh &H = ctx->H;
    if (vol) std::memcpy(vol, H.vol.data(), H.vol.size() * sizeof(double));
    if (xc) std::memcpy(xc, H.xc.data(), H.xc.size() * sizeof(double));
    if (dS) std::memcpy(dS, H.dS.data(), H.dS.size() * sizeof(double));
    return UGKWP_OK;
}

int32_t ugkwp_graph_enable(ugkwp_ctx *ctx, int32_t on) {
    if (!ctx) return fail(ctx, UGKWP_E_ARG, "bad argument");
    if (on && !ctx->stream)
        return fail(ctx, UGKWP_E_ARG, "graph replay needs a created stream (the null stream cannot be captured)");
    if (!on) ctx->drop_graphs();
    ctx->graph_on = on != 0;
    return UGKWP_OK;
}

int32_t ugkwp_set_launch(ugkwp_ctx *ctx, const int32_t *cfg) {
    if (!ctx || !cfg) return fail(ctx, UGKWP_E_ARG, "bad argument");
    ugkwp::LaunchCfg c;
    c.stream_bs = cfg[0];
    c.stream_ilp = cfg[1];
    c.sample_wpb = cfg[2];
    c.flux_bs = cfg[3];
    if (!ugkwp::launch_cfg_valid(c)) return fail(ctx, UGKWP_E_ARG, "launch configuration out of range");
    ctx->cfg = c;
    ctx->drop_graphs();
    return UGKWP_OK;
}

int32_t ugkwp_get_launch(const ugkwp_ctx *ctx, int32_t *cfg) {
    if (!ctx || !cfg) return fail(nullptr, UGKWP_E_ARG, "bad argument");
    cfg[0] = ctx->cfg.stream_bs;
    cfg[1] = ctx->cfg.stream_ilp;
    cfg[2] = ctx->cfg.sample_wpb;
    cfg[3] = ctx->cfg.flux_bs;
    return UGKWP_OK;
}

int32_t ugkwp_autotune(ugkwp_ctx *ctx, int32_t steps_per_trial, int32_t *cfg_out) {
    if (!ctx || steps_per_trial < 1) return fail(ctx, UGKWP_E_ARG, "bad argument");
    if (!ctx->have_state) return fail(ctx, UGKWP_E_STATE, "autotune before init_state");
    if (ctx->poisoned) return fail(ctx, UGKWP_E_STATE, "context poisoned by an earlier device error; call init_state");
    // one pass of coordinate search: each tunable kernel is timed under each of its shapes
    // (hip events around that kernel only) over real steps, holding the others fixed
    const bool prof_was = ctx->prof.on;
    const uint32_t mask_was = ctx->prof.mask;
    const bool graph_was = ctx->graph_on;
    ctx->graph_on = false;
    ctx->prof.on = true;
    ctx->prof.mask = 0xFFFFFFFFu;
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    ctx->prof.drain(nullptr, nullptr, 0);
    ugkwp::LaunchCfg best = ctx->cfg;
    struct Dim {
        int slot;
        std::vector<ugkwp::LaunchCfg> cand;
    };
    std::vector<Dim> dims(3);
    dims[0].slot = ugkwp::kSlotStream;
    for (int ilp : {1, 2})
        for (int b : {128, 256, 512}) {
            ugkwp::LaunchCfg c;
            c.stream_bs = b;
            c.stream_ilp = ilp;
            dims[0].cand.push_back(c);
        }
    dims[1].slot = ugkwp::kSlotSample;
    for (int w : {1, 2, 4, 8}) {
        ugkwp::LaunchCfg c;
        c.sample_wpb = w;
        dims[1].cand.push_back(c);
    }
    dims[2].slot = ugkwp::kSlotFlux;
    for (int b : {64, 128, 256}) {
        ugkwp::LaunchCfg c;
        c.flux_bs = b;
        dims[2].cand.push_back(c);
    }
    int32_t st = UGKWP_OK;
    long long tuned_steps = 0;  // the trials are real steps (full launch sequences)
    for (int d = 0; d < 3 && st == UGKWP_OK; ++d) {
        double best_ms = INFINITY;
        ugkwp::LaunchCfg keep = best;
        for (const auto &c0 : dims[d].cand) {
            ugkwp::LaunchCfg c = best;
            if (d == 0) {
                c.stream_bs = c0.stream_bs;
                c.stream_ilp = c0.stream_ilp;
            } else if (d == 1) {
                c.sample_wpb = c0.sample_wpb;
            } else {
                c.flux_bs = c0.flux_bs;
            }
            ctx->cfg = c;
            // one untimed step (first use of a kernel variant), then the timed ones
            ugkwp::launch_step(ctx->D, ctx->buf, c, ctx->stream, nullptr);
            ctx->buf ^= 1;
            tuned_steps += 1 + steps_per_trial;
            Scalars s0, s1;
            st = read_scalars(ctx, s0);
            if (st != UGKWP_OK) break;
            ctx->prof.drain(nullptr, nullptr, 0);
            for (int32_t k = 0; k < steps_per_trial; ++k) {
                ugkwp::launch_step(ctx->D, ctx->buf, c, ctx->stream, &ctx->prof);
                ctx->buf ^= 1;
            }
            double ms[ugkwp::kNumSlots];
            int64_t cnt[ugkwp::kNumSlots];
            st = read_scalars(ctx, s1);
            if (st != UGKWP_OK) break;
            ctx->prof.drain(ms, cnt, ugkwp::kNumSlots);
            double t = ms[dims[d].slot] / (double)(cnt[dims[d].slot] ? cnt[dims[d].slot] : 1);
            // the particle count drifts between trials: the transport's candidates are compared
            // per particle move
            const unsigned long long moved = s1.moved_total - s0.moved_total;
            if (d == 0 && moved > 0) t = ms[dims[d].slot] / (double)moved;
            if (t < best_ms) {
                best_ms = t;
                keep = c;
            }
        }
        best = keep;
    }
    ctx->cfg = best;
    ctx->drop_graphs();
    ctx->graph_on = graph_was;
    ctx->wave_only_empty = std::max(0LL, ctx->wave_only_empty - tuned_steps);
    ctx->prof.on = prof_was;
    ctx->prof.mask = mask_was;
    if (cfg_out) (void)ugkwp_get_launch(ctx, cfg_out);
    return st;
}

}  // extern "C"

namespace {

// The workload signature that keys the autotuner's cache: the device, the precision, K, the
// sizes and every instance's reconstruction, sampling mode and collision model.
std::string tune_key(const ugkwp_ctx *ctx) {
    int dev = 0;
    hipDeviceProp_t prop{};
    std::string arch = "?";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
    std::string k = arch + " prec=" + std::to_string(ctx->D.prec) + " K=" + std::to_string(ctx->D.K) +
                    " inst=" + std::to_string(ctx->D.n_inst) + " cells=" + std::to_string(ctx->D.nc) +
                    " faces=" + std::to_string(ctx->D.nf) + " cap=" + std::to_string(ctx->D.cap) + " modes=";
    for (const ugkwp_params &p : ctx->ps) {
        char b[64];
        std::snprintf(b, sizeof b, "%d%d%s", p.recon, p.sampling, prandtl_of(p) != 1.0 ? "s" : "");
        k += b;
    }
    return k;
}

// the last line of the cache file with this key: {"key": "<key>", "launch": [a, b, c, d]}
bool tune_lookup(const char *path, const std::string &key, int32_t cfg[4]) {
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    bool found = false;
    char line[4096];
    const std::string want = "{\"key\": \"" + key + "\", \"launch\": [";
    while (std::fgets(line, sizeof line, f)) {
        if (std::strncmp(line, want.c_str(), want.size()) != 0) continue;
        int a, b, c, d;
        if (std::sscanf(line + want.size(), "%d, %d, %d, %d]", &a, &b, &c, &d) == 4) {
            cfg[0] = a;
            cfg[1] = b;
            cfg[2] = c;
            cfg[3] = d;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

}  // namespace

extern "C" {

int32_t ugkwp_autotune_cached(ugkwp_ctx *ctx, int32_t steps_per_trial, const char *cache_path, int32_t *cfg_out,
                              int32_t *hit) {
    if (!ctx || !cache_path || steps_per_trial < 1) return fail(ctx, UGKWP_E_ARG, "bad argument");
    if (hit) *hit = 0;
    const std::string key = tune_key(ctx);
    if (key.find('"') != std::string::npos || key.find('\n') != std::string::npos)
        return fail(ctx, UGKWP_E_ARG, "workload signature not storable");
    int32_t cfg[4];
    if (tune_lookup(cache_path, key, cfg)) {
        ugkwp::LaunchCfg c;
        c.stream_bs = cfg[0];
        c.stream_ilp = cfg[1];
        c.sample_wpb = cfg[2];
        c.flux_bs = cfg[3];
        if (ugkwp::launch_cfg_valid(c)) {
            const int32_t st = ugkwp_set_launch(ctx, cfg);
            if (st != UGKWP_OK) return st;
            if (hit) *hit = 1;
            if (cfg_out) (void)ugkwp_get_launch(ctx, cfg_out);
            return UGKWP_OK;
        }
        // an entry out of range (another build's shapes) counts as a miss
    }
    const int32_t st = ugkwp_autotune(ctx, steps_per_trial, cfg);
    if (st != UGKWP_OK) return st;
    FILE *f = std::fopen(cache_path, "a");
    if (!f) return fail(ctx, UGKWP_E_ARG, std::string("cannot append to the autotune cache ") + cache_path);
    std::fprintf(f, "{\"key\": \"%s\", \"launch\": [%d, %d, %d, %d]}\n", key.c_str(), cfg[0], cfg[1], cfg[2], cfg[3]);
    const bool ok = std::fclose(f) == 0;
    if (!ok) return fail(ctx, UGKWP_E_ARG, std::string("cannot write the autotune cache ") + cache_path);
    if (cfg_out) std::memcpy(cfg_out, cfg, sizeof cfg);
    return UGKWP_OK;
}

int32_t ugkwp_profile_enable(ugkwp_ctx *ctx, int32_t on) {
    if (!ctx) return fail(ctx, UGKWP_E_ARG, "bad argument");
    ctx->prof.on = on != 0;
    return UGKWP_OK;
}

int32_t ugkwp_profile_mask(ugkwp_ctx *ctx, uint32_t mask) {
    if (!ctx) return fail(ctx, UGKWP_E_ARG, "bad argument");
    ctx->prof.mask = mask;
    return UGKWP_OK;
}

int32_t ugkwp_profile_read(ugkwp_ctx *ctx, int32_t n_slots, double *total_ms, int64_t *launches) {
    if (!ctx || n_slots < 0) return fail(ctx, UGKWP_E_ARG, "bad argument");
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    ctx->prof.drain(total_ms, launches, n_slots);
    return UGKWP_OK;
}

const char *ugkwp_profile_slot_name(int32_t slot) {
    return (slot >= 0 && slot < ugkwp::kNumSlots) ? kSlotNames[slot] : "";
}

int32_t ugkwp_init_mesh_static(ugkwp_ctx **out, const ugkwp_mesh *m, int32_t n_inst, const ugkwp_params *p,
                               void *hip_stream) {
    if (!out || !m || !p) return fail(nullptr, UGKWP_E_ARG, "null argument");
    *out = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(nullptr, UGKWP_E_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxStaticDevices)
        return fail(nullptr, UGKWP_E_ARG, "init_mesh_static: device index beyond " + std::to_string(kMaxStaticDevices));
    size_t need = 0;
    int32_t st = ugkwp_workspace_bytes(m, n_inst, p, &need);
    if (st != UGKWP_OK) return st;
    if (need > kStaticWorkspaceBytes)
        return fail(nullptr, UGKWP_E_CAPACITY,
                    "init_mesh_static: this mesh and capacity need " + std::to_string(need) +
                        " bytes of workspace; the static workspace holds " + std::to_string(kStaticWorkspaceBytes) +
                        " (use ugkwp_init_mesh with a workspace of that size, or a smaller capacity)");
    void *ptr = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_static_mu);
        if (g_static_busy[dev])
            return fail(nullptr, UGKWP_E_STATE,
                        "init_mesh_static: the static workspace of device " + std::to_string(dev) +
                            " is in use by another context (destroy it first)");
        if (!g_static_ptr[dev]) {
            // the current device is `dev`: its copy of the array
            void *q = nullptr;
            e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !q)
                return fail(nullptr, UGKWP_E_DEVICE, std::string("hipGetSymbolAddress: ") + hipGetErrorString(e));
            g_static_ptr[dev] = q;
        }
        ptr = g_static_ptr[dev];
        g_static_busy[dev] = true;
    }
    st = ugkwp_init_mesh(out, m, n_inst, p, ptr, kStaticWorkspaceBytes, hip_stream);
    if (st != UGKWP_OK) {
        std::lock_guard<std::mutex> lock(g_static_mu);
        g_static_busy[dev] = false;
        return st;
    }
    (*out)->static_dev = dev;
    return UGKWP_OK;
}

size_t ugkwp_static_workspace_bytes(void) { return kStaticWorkspaceBytes; }

const char *ugkwp_last_error(const ugkwp_ctx *ctx) { return ctx ? ctx->err.c_str() : g_err.c_str(); }

void ugkwp_destroy(ugkwp_ctx *ctx) {
    if (!ctx) return;
    const int dev = ctx->static_dev;
    if (dev >= 0) {
        // the next context on this GPU's array must not overlap work still in flight
        (void)hipStreamSynchronize(ctx->stream);
    }
    delete ctx;
    if (dev >= 0) {
        std::lock_guard<std::mutex> lock(g_static_mu);
        g_static_busy[dev] = false;
    }
}

}  // extern "C"
