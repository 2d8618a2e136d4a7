// C-ABI entry points of libilu (see include/ilu.h) and the host-side layout
// and orchestration.  Every arithmetic step of the method runs in the HIP
// kernels; the host only builds index tables, allocates, launches and checks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstddef>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <queue>
#include <utility>
#include <vector>

#include "ilu.h"
#include "ctx.h"
#include "setup_kernels.h"
#include "sweep_kernels.h"
#include "krylov_kernels.h"
#include "lfa_kernels.h"
#include "residual_stage.h"

using namespace ilu;

namespace {

// Device bytes the library holds during one setup call on this thread: the
// current sum over its buffers and the largest it reached.  Buffers record
// the setup (epoch) they were allocated in, so only those count on release.
struct SetupMem {
    uint64_t epoch = 0;
    bool on = false;
    int64_t cur = 0, peak = 0;
};
thread_local SetupMem g_setup_mem;

// Owning device buffer (move-only: a copy would free the same pointer twice).
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    uint64_t epoch = 0;  // setup that allocated it (0: none)
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes), epoch(o.epoch) {
        o.p = nullptr;
        o.bytes = 0;
        o.epoch = 0;
    }
    DevBuf& operator=(DevBuf&& o) noexcept {
        if (this != &o) {
            release();
            p = o.p;
            bytes = o.bytes;
            epoch = o.epoch;
            o.p = nullptr;
            o.bytes = 0;
            o.epoch = 0;
        }
        return *this;
    }
    void swap(DevBuf& o) noexcept {
        std::swap(p, o.p);
        std::swap(bytes, o.bytes);
        std::swap(epoch, o.epoch);
    }
    ~DevBuf() { release(); }
    void release() {
        if (p) {
            (void)hipFree(p);
            if (g_setup_mem.on && epoch == g_setup_mem.epoch) g_setup_mem.cur -= (int64_t)bytes;
        }
        p = nullptr;
        bytes = 0;
        epoch = 0;
    }
    hipError_t alloc(size_t n, hipStream_t st, bool zero = true) {
        release();
        bytes = n ? n : 8;
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            p = nullptr;
            bytes = 0;
            return e;
        }
        if (g_setup_mem.on) {
            epoch = g_setup_mem.epoch;
            g_setup_mem.cur += (int64_t)bytes;
            g_setup_mem.peak = std::max(g_setup_mem.peak, g_setup_mem.cur);
        }
        if (zero) e = hipMemsetAsync(p, 0, bytes, st);
        return e;
    }
    template <typename T>
    T* as() const { return static_cast<T*>(p); }
};

int64_t choose3_h(int64_t k) { return k < 3 ? 0 : k * (k - 1) * (k - 2) / 6; }

}  // namespace

struct ilu_handle_s {
    int ntets = 0;
    int variant = 0;     // kernel variant: ILU_STORED_F64, ILU_SURR_F64 or ILU_SURR_F32
    bool sgs = false;    // stored factors are the symmetric Gauss-Seidel ones
    int schedule = 0;
    int deg[3] = {0, 0, 0};
    int NC = 0, K = 0;
    int bv = 8, bw = 8;  // block shape in rows
    int64_t S = 0;
    int64_t XE = 0;  // exchange entries (all blocks)
    int64_t nlex = 0;
    int tmin = 0, tmax = 0;
    std::vector<TetDev> tets;
    std::vector<BlockDev> blocks;
    std::vector<LaneDev> lanes;
    std::vector<double> coef_h;  // ntets * 8 * K
    DevBuf tets_d, blocks_d, lanes_d;
    DevBuf A8, Lf, Df, Lb, tab64, tab32, coef_d;
    DevBuf xs, bs, r, w;
    DevBuf partial, norms, flags;
    DevBuf order_fwd, order_bwd, xch, ticket;
    int64_t npartial = 0;      // partial sums of the residual kernel
    int64_t npartial_tag = 0;  // ... and of the tagged one (overlapped residual)
    int res_lds_t = RES_T;     // hyperplanes per workgroup of the sequential LDS-staged residual
    int flow_grid = 0;
    int64_t setup_peak = 0, setup_resident = 0;  // library device bytes: peak during setup, held after it
    int flow_grid_max = 0;               // resident workgroups of the dataflow sweeps (the default grid)
    hipEvent_t ev[8] = {};
    bool have_timing = false;
    bool kernel_timing = false;          // events around every kernel of every sweep
    std::vector<hipEvent_t> kev;         // 6 per sweep: res begin/end, fwd begin/end, bwd begin/end
    int kev_sweeps = 0;
    bool use_graph = true;               // replay fixed-count sweeps from a captured graph
    double tuned_ms = 0.0;               // autotuner: measured sweep time of the chosen block shape
    int last_sweeps = 0;                 // sweeps the last ilu_smooth call ran
    hipStream_t cap = nullptr;           // private stream the sweep graph is captured on
    hipGraphExec_t gexec = nullptr;      // one sweep: residual, forward and backward substitution
    hipGraphExec_t gexec_n = nullptr;    // gexec_count sweeps in one graph (the last fixed count asked for)
    int gexec_count = 0;
    DevBuf cg_r, cg_z, cg_p, cg_q, cg_sc;  // PCG vectors (stream layout) and scalars
    int a_mode = ILU_A_EXACT;            // operator of the residual
    int boundary = ILU_BOUNDARY_V2;      // boundary stencils of the surrogate variants
    int64_t v1_nf = 0, v1_nbk = 0;       // points of the V1 sets F and B
    DevBuf v1f, v1b;                     // their factor planes (variant V1 only)
    DevBuf coefA_d, tabA64, tabA32;      // surrogate operator: coefficients and row tables
    std::vector<double> coefA_h;
    hipGraphExec_t cg_exec = nullptr;    // one PCG iteration
    bool ovl_ok = false;                 // the overlapped residual is available (dataflow, exact A, V2)
    int ovl = ILU_OVERLAP_OFF;           // ILU_OVERLAP_* mode of ilu_smooth
    DevBuf rt;                           // its tagged residual entries
    DevBuf rflag;                        // its band marks (tag per 64-lane group and hyperplane band)
    hipStream_t st2 = nullptr;           // stream of the overlapped residual
    hipEvent_t oev[2] = {};              // fork and join events

    Ctx ctx() const {
        Ctx c;
        c.tets = tets_d.as<TetDev>();
        c.blocks = blocks_d.as<BlockDev>();
        c.lanes = lanes_d.as<LaneDev>();
        c.nblocks = (int)blocks.size();
        c.bv = bv;
        c.bw = bw;
        c.lpb = bv * bw;
        c.groups = c.lpb / WAVE;
        c.S = S;
        int maxlen = 1, tlast = 0;
        for (const auto& b : blocks) {
            maxlen = std::max(maxlen, b.te - b.tb + 1);
            tlast = std::max(tlast, b.te);
        }
        c.res_chunks = (maxlen + RES_T - 1) / RES_T;
        c.res_bands = (tlast + 1 + RES_T - 1) / RES_T;
        c.res_lds_t = res_lds_t;
        c.A8 = A8.as<double>();
        c.Lf = Lf.as<double>();
        c.Lb = Lb.as<double>();
        c.tab64 = tab64.as<double>();
        c.tab32 = tab32.as<float>();
        c.NC = NC;
        c.r = r.p;
        c.w = w.p;
        if (a_mode == ILU_A_SURROGATE) {
            if (variant == ILU_SURR_F32) c.tabA32 = tabA32.as<float>();
            else c.tabA64 = tabA64.as<double>();
        }
        if (boundary == ILU_BOUNDARY_V1) {
            c.v1f = v1f.p;
            c.v1b = v1b.p;
            c.v1f_stride = v1_nf + 1;
            c.v1b_stride = v1_nbk + 1;
        }
        return c;
    }
    Flow flow() const {
        Flow f;
        f.order_fwd = order_fwd.as<int32_t>();
        f.order_bwd = order_bwd.as<int32_t>();
        f.xch = xch.as<uint64_t>();
        f.ticket = ticket.as<int32_t>();
        f.flags = flags.as<int32_t>();
        f.grid = flow_grid;
        return f;
    }
    ~ilu_handle_s() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (gexec_n) (void)hipGraphExecDestroy(gexec_n);
        if (cg_exec) (void)hipGraphExecDestroy(cg_exec);
        if (cap) (void)hipStreamDestroy(cap);
        if (st2) (void)hipStreamDestroy(st2);
        for (auto& e : oev)
            if (e) (void)hipEventDestroy(e);
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
        for (auto& e : kev)
            if (e) (void)hipEventDestroy(e);
    }
};

namespace {

thread_local char g_last_error[256] = "";

int hip_fail(hipError_t e, const char* what, int line) {
    std::snprintf(g_last_error, sizeof(g_last_error), "%s failed: %s (abi.cpp:%d)", what, hipGetErrorName(e), line);
    return ILU_EHIP;
}

#define HIPCHK(x)                                            \
    do {                                                     \
        const hipError_t e_ = (x);                           \
        if (e_ != hipSuccess) return hip_fail(e_, #x, __LINE__); \
    } while (0)

// Sample sets S_d as lattice simplices of side M (see put_samples in the setup kernels).
int sample_side(int n, int fit, int stride) {
    static const int d[8][3] = {{-1, 0, 0}, {0, -1, 0}, {1, -1, 0}, {-1, 1, -1},
                                {0, 1, -1}, {0, 0, -1}, {1, 0, -1}, {0, 0, 0}};
    int sumd = d[fit][0] + d[fit][1] + d[fit][2];
    int shift = 0;
    for (int k = 0; k < 3; ++k) shift += 1 - std::min(d[fit][k], 0);
    int room = n - 1 - std::max(0, sumd) - shift;
    return room >= 0 ? room / stride : -1;
}

int build_layout(ilu_handle_t h) {
    const int bv = h->bv, bw = h->bw, lpb = bv * bw;
    int nmax = 0;
    for (auto& T : h->tets) nmax = std::max(nmax, T.n);
    const int64_t Z = (int64_t)lpb * (3 * nmax + 8);
    int64_t S = Z, XE = 0;
    std::vector<std::vector<int>> bmap(h->ntets);
    std::vector<int> nbv(h->ntets), nbw(h->ntets);
    int64_t lexoff = 0;
    for (int ti = 0; ti < h->ntets; ++ti) {
        TetDev& T = h->tets[ti];
        const int n = T.n;
        // rows: v in [2, n-2], w in [1, v-1]
        nbv[ti] = std::max(1, (n - 3 + bv - 1) / bv);
        nbw[ti] = std::max(1, (n - 3 + bw - 1) / bw);
        bmap[ti].assign((size_t)nbv[ti] * nbw[ti], -1);
        T.blk0 = (int)h->blocks.size();
        T.lex_off = lexoff;
        T.N = choose3_h(n - 1);
        lexoff += T.N;
        for (int kw = 0; kw < nbw[ti]; ++kw)
            for (int kv = 0; kv < nbv[ti]; ++kv) {
                const int V0 = 2 + bv * kv, W0 = 1 + bw * kw;
                int tb = 1 << 30, te = -1;
                for (int l = 0; l < lpb; ++l) {
                    int vl = 0, wl = 0;
                    lane_rc(l, bv, &vl, &wl);
                    const int v = V0 + vl, w = W0 + wl;
                    if (v > n - 2 || w > v - 1) continue;
                    tb = std::min(tb, 2 * v + w + 1);
                    te = std::max(te, n - 1 + v + w);
                }
                if (te < 0) continue;
                BlockDev B{};
                B.tet = ti;
                B.V0 = V0;
                B.W0 = W0;
                B.tb = tb;
                B.te = te;
                B.tlo = tb - PAD;
                B.len = te - tb + 1 + 2 * PAD;
                B.base = S;
                S += (int64_t)B.len * lpb;
                B.xoff = XE;
                XE += (int64_t)B.len * (bv + bw);
                bmap[ti][(size_t)kv * nbw[ti] + kw] = (int)h->blocks.size();
                h->blocks.push_back(B);
            }
        T.nblk = (int)h->blocks.size() - T.blk0;
    }
    S += (int64_t)lpb * TAIL;
    h->S = S;
    h->XE = XE;
    h->nlex = lexoff;
    auto block_at = [&](int ti, int kv, int kw) -> int {
        if (kv < 0 || kw < 0 || kv >= nbv[ti] || kw >= nbw[ti]) return -1;
        return bmap[ti][(size_t)kv * nbw[ti] + kw];
    };
    auto gl_of = [&](int ti, int v, int w) -> int32_t {
        const int n = h->tets[ti].n;
        if (v < 2 || v > n - 2 || w < 1 || w > v - 1) return -1;
        const int b = block_at(ti, (v - 2) / bv, (w - 1) / bw);
        const BlockDev& B = h->blocks[b];
        return (int32_t)((int64_t)b * lpb + lane_at(v - B.V0, w - B.W0, bv));
    };
    auto rp_of = [&](int ti, int v, int w) -> int64_t {
        const int n = h->tets[ti].n;
        if (v < 2 || v > n - 2 || w < 1 || w > v - 1) return 0;  // zero region
        const int b = block_at(ti, (v - 2) / bv, (w - 1) / bw);
        const BlockDev& B = h->blocks[b];
        const int l = lane_at(v - B.V0, w - B.W0, bv);
        return B.base - (int64_t)B.tlo * lpb + l;
    };
    // variant V1: the point sets F and B numbered row by row, rows of each
    // tetrahedron in (w, v) order (independent of the block shape)
    std::vector<std::vector<int32_t>> fbase(h->ntets), bbase(h->ntets);
    int64_t nf = 0, nbk = 0;
    for (int ti = 0; ti < h->ntets; ++ti) {
        const int n = h->tets[ti].n;
        fbase[ti].assign((size_t)n * n, -1);
        bbase[ti].assign((size_t)n * n, -1);
        for (int w = 1; w <= n - 3; ++w)
            for (int v = w + 1; v <= n - 2; ++v) {
                const int y = v - w, z = w, xmax = n - 1 - v;
                fbase[ti][(size_t)v * n + w] = (int32_t)nf;
                bbase[ti][(size_t)v * n + w] = (int32_t)nbk;
                nf += v1f_count(xmax, y, z);
                nbk += v1b_count(xmax, y, z);
            }
    }
    if (nf >= ((int64_t)1 << 31) - 1 || nbk >= ((int64_t)1 << 31) - 1) return ILU_EINVAL;
    h->v1_nf = nf;
    h->v1_nbk = nbk;
    auto base_of = [&](const std::vector<std::vector<int32_t>>& tab, int ti, int v, int w) -> int32_t {
        const int n = h->tets[ti].n;
        if (v < 2 || v > n - 2 || w < 1 || w > v - 1) return -1;
        return tab[ti][(size_t)v * n + w];
    };
    h->lanes.resize(h->blocks.size() * lpb);
    h->tmin = 1 << 30;
    h->tmax = 0;
    for (size_t bi = 0; bi < h->blocks.size(); ++bi) {
        BlockDev& B = h->blocks[bi];
        const int ti = B.tet, n = h->tets[ti].n;
        const int kv = (B.V0 - 2) / bv, kw = (B.W0 - 1) / bw;
        B.pred[0] = block_at(ti, kv - 1, kw);
        B.pred[1] = block_at(ti, kv, kw - 1);
        B.pred[2] = block_at(ti, kv - 1, kw - 1);
        B.succ[0] = block_at(ti, kv + 1, kw);
        B.succ[1] = block_at(ti, kv, kw + 1);
        B.succ[2] = block_at(ti, kv + 1, kw + 1);
        h->tmin = std::min(h->tmin, B.tb);
        h->tmax = std::max(h->tmax, B.te);
        for (int l = 0; l < lpb; ++l) {
            LaneDev& L = h->lanes[bi * lpb + l];
            int vl = 0, wl = 0;
            lane_rc(l, bv, &vl, &wl);
            const int v = B.V0 + vl, w = B.W0 + wl;
            const bool valid = v <= n - 2 && w <= v - 1;
            L.v = valid ? v : 0;
            L.w = w;
            L.rp[R_SELF] = valid ? B.base - (int64_t)B.tlo * lpb + l : 0;
            L.rp[R_VM] = rp_of(ti, v - 1, w);
            L.rp[R_WM] = rp_of(ti, v, w - 1);
            L.rp[R_VMWM] = rp_of(ti, v - 1, w - 1);
            L.rp[R_VP] = rp_of(ti, v + 1, w);
            L.rp[R_WP] = rp_of(ti, v, w + 1);
            L.rp[R_VPWP] = rp_of(ti, v + 1, w + 1);
            L.v1f[0] = valid ? base_of(fbase, ti, v, w) : -1;
            L.v1f[1] = valid ? base_of(fbase, ti, v + 1, w) : -1;
            L.v1f[2] = valid ? base_of(fbase, ti, v, w + 1) : -1;
            L.v1f[3] = valid ? base_of(fbase, ti, v + 1, w + 1) : -1;
            L.v1b = valid ? base_of(bbase, ti, v, w) : -1;
            L.gl[R_SELF] = valid ? (int32_t)(bi * lpb + l) : -1;
            L.gl[R_VM] = gl_of(ti, v - 1, w);
            L.gl[R_WM] = gl_of(ti, v, w - 1);
            L.gl[R_VMWM] = gl_of(ti, v - 1, w - 1);
            L.gl[R_VP] = gl_of(ti, v + 1, w);
            L.gl[R_WP] = gl_of(ti, v, w + 1);
            L.gl[R_VPWP] = gl_of(ti, v + 1, w + 1);
            L.pad_[0] = L.pad_[1] = 0;
            L.gt[0] = 1 << 30;
            L.gt[1] = -1;
            if (valid && (v - w <= 2 || w == 1)) B.edge = 1;
        }
        // hyperplane window of each 64-lane group (same value in all its lanes)
        for (int g = 0; g < lpb / WAVE; ++g) {
            int gtb = 1 << 30, gte = -1;
            for (int l = g * WAVE; l < (g + 1) * WAVE; ++l) {
                const LaneDev& L = h->lanes[bi * lpb + l];
                if (L.v == 0) continue;
                gtb = std::min(gtb, 2 * L.v + L.w + 1);
                gte = std::max(gte, n - 1 + L.v + L.w);
            }
            for (int l = g * WAVE; l < (g + 1) * WAVE; ++l) {
                h->lanes[bi * lpb + l].gt[0] = gtb;
                h->lanes[bi * lpb + l].gt[1] = gte;
            }
        }
    }
    return ILU_OK;
}

// Kahn topological order of the block DAG, ready blocks taken by priority.
std::vector<int32_t> topo_order(const std::vector<BlockDev>& blocks, bool forward) {
    const int nb = (int)blocks.size();
    std::vector<int> indeg(nb, 0);
    std::vector<std::vector<int>> out(nb);
    for (int b = 0; b < nb; ++b)
        for (int k = 0; k < 3; ++k) {
            const int p = forward ? blocks[b].pred[k] : blocks[b].succ[k];
            if (p >= 0) {
                indeg[b]++;
                out[p].push_back(b);
            }
        }
    auto key = [&](int b) -> int64_t {
        const BlockDev& B = blocks[b];
        return forward ? ((int64_t)B.tb << 20) + (B.V0 + B.W0) : ((int64_t)(-B.te) << 20) - (B.V0 + B.W0);
    };
    auto cmp = [&](int a, int b) { return key(a) > key(b) || (key(a) == key(b) && a > b); };
    std::priority_queue<int, std::vector<int>, decltype(cmp)> pq(cmp);
    for (int b = 0; b < nb; ++b)
        if (!indeg[b]) pq.push(b);
    std::vector<int32_t> order;
    order.reserve(nb);
    while (!pq.empty()) {
        const int b = pq.top();
        pq.pop();
        order.push_back(b);
        for (int s : out[b])
            if (--indeg[s] == 0) pq.push(s);
    }
    return order;
}

template <typename T>
int upload(DevBuf& buf, const std::vector<T>& v, hipStream_t st) {
    if (buf.alloc(v.size() * sizeof(T), st, false) != hipSuccess) return ILU_ENOMEM;
    if (!v.empty()) HIPCHK(hipMemcpyAsync(buf.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
    return ILU_OK;
}

int read_flags(ilu_handle_t h, hipStream_t st, int32_t out[4]) {
    HIPCHK(hipMemcpyAsync(out, h->flags.p, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return ILU_OK;
}

// Least squares for every (tet, fitted direction): TSQR on the device, then
// back substitution.  Level 0 splits the samples of each problem into runs of
// equal length, about QR_RUNS of them over all problems, each reduced to one
// triangular factor; every later level reduces each problem's stacked factors
// eight at a time, until one R per problem is left.
int solve_lsq(ilu_handle_t h, const DevBuf& samples, hipStream_t st, DevBuf& coef_out) {
    const int K = h->K, m = K + 1;
    if (m > 512) return ILU_EINVAL;
    const Ctx c = h->ctx();
    const int np = h->ntets * NFIT;
    constexpr int64_t QR_RUNS = 512, QR_MIN_RUN = 256;
    std::vector<int64_t> rows(np);
    int64_t total = 0;
    for (int ti = 0; ti < h->ntets; ++ti)
        for (int f = 0; f < NFIT; ++f) total += rows[ti * NFIT + f] = h->tets[ti].samp_cnt[f];
    const int64_t run0 = std::max<int64_t>(QR_MIN_RUN, (total + QR_RUNS - 1) / QR_RUNS);
    std::vector<int64_t> in_at(np, 0);  // row offset of each problem in the current input
    DevBuf in, out, jobs_d;
    for (int level = 0;; ++level) {
        std::vector<QrJob> jobs(np);
        int64_t outrows = 0;
        int runs = 0;
        bool more = false;
        for (int p = 0; p < np; ++p) {
            QrJob& J = jobs[p];
            J.tet = p / NFIT;
            J.fit = p % NFIT;
            J.in_rows = rows[p];
            J.in_off = level == 0 ? h->tets[J.tet].samp_off[J.fit] : in_at[p];
            J.run_rows = level == 0 ? run0 : (int64_t)8 * m;
            J.nchunk = (int)std::max<int64_t>(1, (rows[p] + J.run_rows - 1) / J.run_rows);
            J.chunk0 = runs;
            J.out_off = outrows;
            runs += J.nchunk;
            outrows += (int64_t)J.nchunk * m;
            more = more || J.nchunk > 1;
        }
        if (out.alloc((size_t)outrows * m * sizeof(double), st, false) != hipSuccess) return ILU_ENOMEM;
        if (upload(jobs_d, jobs, st)) return ILU_ENOMEM;
        launch_qr_stream(c, jobs_d.as<QrJob>(), np, level == 0 ? 1 : 0, m, samples.as<double>(), in.as<double>(),
                         out.as<double>(), (int)std::min<int64_t>(runs, QR_RUNS), runs, st);
        HIPCHK(hipGetLastError());
        for (int p = 0; p < np; ++p) {
            rows[p] = (int64_t)jobs[p].nchunk * m;
            in_at[p] = jobs[p].out_off;
        }
        in.swap(out);
        if (!more) break;
    }
    // solve: one R per problem, at row p * m of `in`
    std::vector<QrJob> sj(np);
    for (int p = 0; p < np; ++p) {
        sj[p] = QrJob{};
        sj[p].tet = p / NFIT;
        sj[p].fit = p % NFIT;
        sj[p].out_off = (int64_t)p * m;
    }
    if (upload(jobs_d, sj, st)) return ILU_ENOMEM;
    if (coef_out.alloc((size_t)np * K * sizeof(double), st) != hipSuccess) return ILU_ENOMEM;
    launch_qr_solve(jobs_d.as<QrJob>(), np, m, in.as<double>(), coef_out.as<double>(), h->flags.as<int>(), st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    return ILU_OK;
}

// Per-row evaluation tables of one set of 8 fitted polynomials (the ILU
// factors into tab64/tab32, or the operator into tabA64/tabA32); the FP32 copy
// only for the mixed variant.
int build_tables_from(ilu_handle_t h, hipStream_t st, const DevBuf& coef, DevBuf& t64, DevBuf& t32) {
    const int nslots = (int)h->blocks.size() * h->bv * h->bw;
    const size_t rec = 2 + 15 * (size_t)h->NC;
    if (t64.alloc(nslots * rec * sizeof(double), st) != hipSuccess) return ILU_ENOMEM;
    if (h->variant == ILU_SURR_F32 && t32.alloc(nslots * rec * sizeof(float), st) != hipSuccess) return ILU_ENOMEM;
    const Ctx c = h->ctx();
    launch_row_tables(c, nslots, coef.as<double>(), h->NC, t64.as<double>(),
                      h->variant == ILU_SURR_F32 ? t32.as<float>() : nullptr, st);
    HIPCHK(hipGetLastError());
    return ILU_OK;
}

int build_tables(ilu_handle_t h, hipStream_t st) { return build_tables_from(h, st, h->coef_d, h->tab64, h->tab32); }

// Host-only preparation: validated tetrahedron records, sample layout, block tables.
int prepare(const ilu_tet_desc* tets, int32_t ntets, const ilu_opts* opts, ilu_handle_t h, int64_t* nsamples) {
    h->ntets = ntets;
    h->sgs = opts->variant == ILU_STORED_SGS;
    h->variant = h->sgs ? ILU_STORED_F64 : opts->variant;
    h->a_mode = opts->a_mode;
    h->boundary = opts->boundary;
    h->schedule = opts->schedule == ILU_SCHED_PLANE ? ILU_SCHED_PLANE : ILU_SCHED_DATAFLOW;
    const bool surr = h->variant != ILU_STORED_F64;
    for (int k = 0; k < 3; ++k) h->deg[k] = surr ? opts->degree[k] : 0;
    h->NC = h->deg[0] + 1;
    h->K = (h->deg[0] + 1) * (h->deg[1] + 1) * (h->deg[2] + 1);
    const int stride0 = opts->sample_stride > 0 ? opts->sample_stride : 4;
    h->tets.resize(ntets);
    int64_t soff = 0;
    for (int i = 0; i < ntets; ++i) {
        const ilu_tet_desc& D = tets[i];
        TetDev& T = h->tets[i];
        std::memset(&T, 0, sizeof(T));
        T.level = D.level;
        T.n = 1 << D.level;
        T.kind = D.coeff_kind;
        for (int k = 0; k < 4; ++k) T.cp[k] = D.coeff_param[k];
        for (int r = 0; r < 3; ++r) {
            T.v0[r] = D.vertex[0][r];
            for (int c = 0; c < 3; ++c) T.J[3 * r + c] = D.vertex[c + 1][r] - D.vertex[0][r];
        }
        const double* J = T.J;
        const double det = J[0] * (J[4] * J[8] - J[5] * J[7]) - J[1] * (J[3] * J[8] - J[5] * J[6]) +
                           J[2] * (J[3] * J[7] - J[4] * J[6]);
        // either orientation: the element stiffness only uses |det| and metric terms
        if (!(std::fabs(det) > 0.0) || !std::isfinite(det)) return ILU_EGEOM;
        for (int k = 0; k < 3; ++k) T.deg[k] = h->deg[k];
        T.ncoef = h->K;
        if (surr) {
            const int need = h->deg[0] + h->deg[1] + h->deg[2];
            int s = stride0;
            while (s >= 1) {
                bool ok = true;
                for (int f = 0; f < NFIT; ++f) ok = ok && sample_side(T.n, f, s) >= need;
                if (ok) break;
                s /= 2;
            }
            if (s < 1) return ILU_ERANK;
            T.stride = s;
            for (int f = 0; f < NFIT; ++f) {
                T.samp_M[f] = sample_side(T.n, f, s);
                T.samp_cnt[f] = choose3_h(T.samp_M[f] + 3);
                T.samp_off[f] = soff;
                soff += T.samp_cnt[f];
            }
        }
    }
    if (opts->tile[0] && opts->tile[1]) {
        h->bv = opts->tile[0];
        h->bw = opts->tile[1];
    } else {
        // larger blocks cut the number of cross-workgroup hops on the critical
        // path of one big tetrahedron; many small ones keep 8 x 8 blocks
        int lmax = 0;
        for (const auto& T : h->tets) lmax = std::max(lmax, T.level);
        h->bv = h->bw = 8;
        if (ntets == 1 && lmax >= 8) { h->bv = 16; h->bw = 32; }
        else if (ntets == 1 && lmax == 7) { h->bv = 16; h->bw = 16; }
        // FP64 surrogate polynomials with 4+ coefficients per row do not fit the
        // registers of a 9-wave workgroup
        if (h->variant == ILU_SURR_F64 && h->NC >= 4 && h->bw == 32) h->bw = 16;
    }
    if (int e = build_layout(h)) return e;
    *nsamples = soff;
    return ILU_OK;
}

void sweep_fwd(ilu_handle_t h, const Ctx& c, hipStream_t st);
void sweep_bwd(ilu_handle_t h, const Ctx& c, hipStream_t st, double* target = nullptr);
int sweep_res_fwd(ilu_handle_t h, const Ctx& c, hipStream_t st, double* partial, hipEvent_t* mk);

// Variant V1: the backward weights of set B from F and the surrogate tables
// (after every change of the surrogate coefficients).  The buffer is
// allocated once; its last entries stay 0.
int build_v1b(ilu_handle_t h, hipStream_t st) {
    const bool f32 = h->variant == ILU_SURR_F32;
    const size_t es = f32 ? sizeof(float) : sizeof(double);
    if (!h->v1b.p && h->v1b.alloc((size_t)8 * (h->v1_nbk + 1) * es, st) != hipSuccess) return ILU_ENOMEM;
    launch_build_v1b(h->ctx(), h->tab64.as<double>(), h->v1f.p, h->v1b.p, f32, st);
    HIPCHK(hipGetLastError());
    return ILU_OK;
}

int setup_sweep_buffers(ilu_handle_t h, hipStream_t st);

// Fit of one set of 8 polynomials per tetrahedron from its samples (Sec. 4.1):
// TSQR least squares on the device, coefficients copied to the host too.
int fit_samples(ilu_handle_t h, const DevBuf& samples, hipStream_t st, DevBuf& coef_d, std::vector<double>& coef_h) {
    if (int e = solve_lsq(h, samples, st, coef_d)) return e;
    int32_t fl[4];
    if (int e = read_flags(h, st, fl)) return e;
    if (fl[1]) return ILU_ERANK;
    coef_h.resize((size_t)h->ntets * NFIT * h->K);
    HIPCHK(hipMemcpyAsync(coef_h.data(), coef_d.p, coef_h.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    return ILU_OK;
}

// Full setup of one handle (timing_only: layout and zeroed buffers only, for
// the tile autotuner).
//  * Stored variants: the stencil is assembled (A8), factored on the
//    hyperplane schedule into full factor planes and transposed into the
//    backward weights.
//  * Surrogate variants: Alg. 1 on a ring of four hyperplanes, each point
//    leaving its samples (and V1 boundary record) as it is factored, then the
//    least-squares fit and the per-row tables.  With the exact operator the
//    stencil is assembled first (the residual reads it); with the surrogate
//    operator no stencil array is ever formed: the ring kernel computes each
//    row on the fly and samples it for the operator's own fit.
int setup_impl(const ilu_tet_desc* tets, int32_t ntets, const ilu_opts* opts, hipStream_t st, ilu_handle_t h,
               bool timing_only = false) {
    int64_t soff = 0;
    if (int e = prepare(tets, ntets, opts, h, &soff)) return e;
    const bool surr = h->variant != ILU_STORED_F64;
    const bool v1 = h->boundary == ILU_BOUNDARY_V1;
    const bool a_surr = h->a_mode == ILU_A_SURROGATE;  // surrogate variants only
    if (upload(h->tets_d, h->tets, st) || upload(h->blocks_d, h->blocks, st) || upload(h->lanes_d, h->lanes, st))
        return ILU_ENOMEM;
    if (h->flags.alloc(4 * sizeof(int32_t), st) != hipSuccess) return ILU_ENOMEM;
    const int64_t S = h->S;
    if (!a_surr && h->A8.alloc((size_t)8 * S * sizeof(double), st) != hipSuccess) return ILU_ENOMEM;
    if (timing_only) {
        // every buffer the sweeps read, zero: their kernels have no
        // data-dependent control flow, so the time does not depend on values
        const bool f32 = h->variant == ILU_SURR_F32;
        const size_t nslots = (size_t)h->blocks.size() * h->bv * h->bw, rec = 2 + 15 * (size_t)h->NC;
        if (!surr) {
            if (h->Lf.alloc((size_t)7 * S * sizeof(double), st) || h->Lb.alloc((size_t)8 * S * sizeof(double), st))
                return ILU_ENOMEM;
        } else {
            h->coef_h.assign((size_t)ntets * NFIT * h->K, 0.0);
            if (h->tab64.alloc(nslots * rec * sizeof(double), st) ||
                (f32 && h->tab32.alloc(nslots * rec * sizeof(float), st)))
                return ILU_ENOMEM;
            if (a_surr && (h->tabA64.alloc(nslots * rec * sizeof(double), st) ||
                           (f32 && h->tabA32.alloc(nslots * rec * sizeof(float), st))))
                return ILU_ENOMEM;
            const size_t es = f32 ? sizeof(float) : sizeof(double);
            if (v1 && (h->v1f.alloc((size_t)8 * (h->v1_nf + 1) * es, st) ||
                       h->v1b.alloc((size_t)8 * (h->v1_nbk + 1) * es, st)))
                return ILU_ENOMEM;
        }
        return setup_sweep_buffers(h, st);
    }
    if (!a_surr) {
        launch_assemble(h->ctx(), h->A8.as<double>(), nullptr, st);
        HIPCHK(hipGetLastError());
    }
    int32_t fl[4];
    if (!surr) {
        if (h->Lf.alloc((size_t)7 * S * sizeof(double), st) != hipSuccess) return ILU_ENOMEM;
        if (h->Df.alloc((size_t)S * sizeof(double), st) != hipSuccess) return ILU_ENOMEM;
        const Ctx c = h->ctx();
        if (h->sgs)
            launch_sgs_factors(c, h->Lf.as<double>(), h->Df.as<double>(), h->flags.as<int>(), st);
        else
            for (int t = h->tmin; t <= h->tmax; ++t)
                launch_factor_plane(c, t, h->Lf.as<double>(), h->Df.as<double>(), h->flags.as<int>(), st);
        HIPCHK(hipGetLastError());
        if (int e = read_flags(h, st, fl)) return e;
        if (fl[0]) return ILU_EBREAKDOWN;
        if (h->Lb.alloc((size_t)8 * S * sizeof(double), st) != hipSuccess) return ILU_ENOMEM;
        launch_transpose(c, h->Lf.as<double>(), h->Df.as<double>(), h->Lb.as<double>(), st);
        HIPCHK(hipGetLastError());
        return setup_sweep_buffers(h, st);
    }
    const bool f32 = h->variant == ILU_SURR_F32;
    const size_t es = f32 ? sizeof(float) : sizeof(double);
    DevBuf samples, asamples;
    if (samples.alloc((size_t)soff * sizeof(double), st) != hipSuccess) return ILU_ENOMEM;
    if (a_surr && asamples.alloc((size_t)soff * sizeof(double), st) != hipSuccess) return ILU_ENOMEM;
    if (v1 && h->v1f.alloc((size_t)8 * (h->v1_nf + 1) * es, st) != hipSuccess) return ILU_ENOMEM;
    {
        const int64_t nring = (int64_t)h->blocks.size() * h->bv * h->bw + 1;
        DevBuf ring;
        if (ring.alloc((size_t)8 * 4 * nring * sizeof(double), st) != hipSuccess) return ILU_ENOMEM;
        const Ctx c = h->ctx();
        for (int t = h->tmin; t <= h->tmax; ++t)
            launch_factor_ring(c, t, ring.as<double>(), nring, samples.as<double>(),
                               a_surr ? asamples.as<double>() : nullptr, v1 ? h->v1f.p : nullptr, f32,
                               h->flags.as<int>(), st);
        HIPCHK(hipGetLastError());
        if (int e = read_flags(h, st, fl)) return e;
        if (fl[0]) return ILU_EBREAKDOWN;
    }
    if (int e = fit_samples(h, samples, st, h->coef_d, h->coef_h)) return e;
    samples.release();
    if (int e = build_tables(h, st)) return e;
    if (v1)
        if (int e = build_v1b(h, st)) return e;
    // surrogate operator: the centre and lower stencil weights, sampled on the
    // same sets and fitted like the factors
    if (a_surr) {
        if (int e = fit_samples(h, asamples, st, h->coefA_d, h->coefA_h)) return e;
        asamples.release();
        if (int e = build_tables_from(h, st, h->coefA_d, h->tabA64, h->tabA32)) return e;
    }
    return setup_sweep_buffers(h, st);
}

// The buffers of the smoothing step (streams, partial sums, exchange, the
// overlapped residual) and the default grid of the persistent sweeps.
int setup_sweep_buffers(ilu_handle_t h, hipStream_t st) {
    const int64_t S = h->S;
    const size_t es = h->variant == ILU_SURR_F32 ? sizeof(float) : sizeof(double);
    if (h->xs.alloc((size_t)S * 8, st) || h->bs.alloc((size_t)S * 8, st) || h->r.alloc((size_t)S * es, st) ||
        h->w.alloc((size_t)S * es, st))
        return ILU_ENOMEM;
    const Ctx c = h->ctx();
    h->npartial = res_partials(c);
    h->npartial_tag = res_tag_partials(c);
    if (h->partial.alloc((size_t)std::max(h->npartial, h->npartial_tag) * sizeof(double), st) || h->norms.alloc(16 * sizeof(double), st))
        return ILU_ENOMEM;
    if (upload(h->order_fwd, topo_order(h->blocks, true), st) || upload(h->order_bwd, topo_order(h->blocks, false), st))
        return ILU_ENOMEM;
    // exchange entries: one 64-bit word (FP32 values) or two (FP64), cleared to tag 0
    const size_t xwords = (size_t)h->XE * (h->variant == ILU_SURR_F32 ? 1 : 2);
    if (h->xch.alloc(std::max<size_t>(1, xwords) * sizeof(uint64_t), st) || h->ticket.alloc(4 * sizeof(int32_t), st))
        return ILU_ENOMEM;
    h->flow_grid_max = std::min<int>((int)h->blocks.size(), flow_max_resident(h->variant, h->NC, h->boundary == ILU_BOUNDARY_V1, h->bv, h->bw));
    h->flow_grid = h->flow_grid_max;
    for (auto& e : h->ev) HIPCHK(hipEventCreate(&e));
    // overlapped residual: tagged entries (one 64-bit word per FP32 value, two
    // per FP64 value), cleared to tag 0, a second stream and fork/join events
    h->ovl_ok = h->schedule == ILU_SCHED_DATAFLOW && h->a_mode == ILU_A_EXACT && h->boundary == ILU_BOUNDARY_V2;
    if (h->ovl_ok) {
        if (h->rt.alloc((size_t)S * (h->variant == ILU_SURR_F32 ? 1 : 2) * sizeof(uint64_t), st)) return ILU_ENOMEM;
        if (h->rflag.alloc((size_t)std::max<int64_t>(1, (int64_t)c.nblocks * c.groups * c.res_bands) * sizeof(uint64_t), st))
            return ILU_ENOMEM;
        HIPCHK(hipStreamCreateWithFlags(&h->st2, hipStreamNonBlocking));
        for (auto& e : h->oev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    HIPCHK(hipStreamSynchronize(st));
    return ILU_OK;
}

// Device time (ms) of one sweep (residual, forward and backward substitution)
// on zero vectors: the sweep kernels have no data-dependent control flow, so
// the values do not matter.  One warm-up sweep, then the mean of `reps`.
int time_sweep(ilu_handle_t h, hipStream_t st, int reps, double* ms, double cutoff_ms) {
    const Ctx c = h->ctx();
    HIPCHK(hipMemsetAsync(h->xs.p, 0, h->xs.bytes, st));
    HIPCHK(hipMemsetAsync(h->bs.p, 0, h->bs.bytes, st));
    float a = 0;
    for (int k = 0; k <= reps; ++k) {
        if (k <= 1) HIPCHK(hipEventRecord(h->ev[0], st));
        if (int e = sweep_res_fwd(h, c, st, nullptr, nullptr)) return e;
        sweep_bwd(h, c, st);
        if (k == 0 && cutoff_ms > 0.0) {
            // the untimed first sweep already far slower than the best
            // configuration so far (a residual kernel that finds no room beside
            // the sweep): report it without the timed ones
            HIPCHK(hipEventRecord(h->ev[1], st));
            HIPCHK(hipEventSynchronize(h->ev[1]));
            HIPCHK(hipEventElapsedTime(&a, h->ev[0], h->ev[1]));
            if (a > cutoff_ms) {
                reps = 0;
                break;
            }
        }
    }
    if (reps > 0) {
        HIPCHK(hipEventRecord(h->ev[1], st));
        HIPCHK(hipEventSynchronize(h->ev[1]));
        HIPCHK(hipEventElapsedTime(&a, h->ev[0], h->ev[1]));
        a /= reps;
    }
    *ms = a;
    int32_t fl[4];
    if (int e = read_flags(h, st, fl)) return e;
    return fl[2] ? ILU_EHIP : ILU_OK;
}

// Autotuner (tile (0, 0)).  For every supported block shape a timing-only
// handle (layout and zeroed buffers: no assembly, factorisation or fit) times
// a few sweeps with several persistent-grid sizes, in both residual modes
// where the overlapped one is available (a latency-bound sweep on a capped
// grid leaves room for the bandwidth-bound residual beside it), and the
// sequential LDS-staged residual with chunks of RES_T and 2 RES_T hyperplanes
// (the longer ones pay on batches of small lattices); the fastest
// combination is then set up in full, once.  Shapes whose sweep kernels would
// spill registers are skipped.
int setup_autotuned(const ilu_tet_desc* tets, int32_t ntets, const ilu_opts* opts, hipStream_t st, ilu_handle_t* out) {
    static const int shapes[3][2] = {{8, 8}, {16, 16}, {16, 32}};
    int best_sh = -1, best_grid = 0, best_ovl = ILU_OVERLAP_OFF, best_rt = RES_T;
    double best_ms = 0.0;
    for (int si = 0; si < 3; ++si) {
        const int* sh = shapes[si];
        if (opts->variant == ILU_SURR_F64 && opts->degree[0] >= 3 && sh[1] == 32) continue;
        ilu_opts o = *opts;
        o.tile[0] = sh[0];
        o.tile[1] = sh[1];
        ilu_handle_t h = new (std::nothrow) ilu_handle_s();
        if (!h) return ILU_ENOMEM;
        int rc = setup_impl(tets, ntets, &o, st, h, true);
        const int gmax = h->flow_grid_max;
        // rt: hyperplanes per workgroup of the sequential LDS-staged residual
        // (longer chunks: fewer ring prologues, fewer workgroups)
        struct Cand { int ovl, grid, rt; };
        const Cand cands[8] = {{ILU_OVERLAP_OFF, gmax, RES_T},     {ILU_OVERLAP_OFF, gmax / 2, RES_T},
                               {ILU_OVERLAP_OFF, gmax / 3, RES_T}, {ILU_OVERLAP_OFF, gmax, 2 * RES_T},
                               {ILU_OVERLAP_OFF, gmax / 2, 2 * RES_T}, {ILU_OVERLAP_ON, gmax, RES_T},
                               {ILU_OVERLAP_ON, gmax / 2, RES_T},  {ILU_OVERLAP_ON, gmax / 4, RES_T}};
        const bool lds_shape = sh[0] == sh[1] && (sh[0] == 8 || sh[0] == 16);
        for (const Cand& cd : cands) {
            if (rc != ILU_OK) break;
            if (cd.grid < 1 || (cd.ovl != ILU_OVERLAP_OFF && !h->ovl_ok)) continue;
            if (cd.rt != RES_T && !lds_shape) continue;
            h->flow_grid = cd.grid;
            h->ovl = cd.ovl;
            h->res_lds_t = cd.rt;
            double ms = 0.0;
            rc = time_sweep(h, st, 3, &ms, best_sh < 0 ? 0.0 : 4.0 * best_ms);
            if (rc == ILU_OK && (best_sh < 0 || ms < best_ms)) {
                best_sh = si;
                best_grid = cd.grid;
                best_ovl = cd.ovl;
                best_rt = cd.rt;
                best_ms = ms;
            }
        }
        (void)hipStreamSynchronize(st);
        delete h;
        if (rc != ILU_OK) return rc;
    }
    if (best_sh < 0) return ILU_EINVAL;
    ilu_opts o = *opts;
    o.tile[0] = shapes[best_sh][0];
    o.tile[1] = shapes[best_sh][1];
    ilu_handle_t h = new (std::nothrow) ilu_handle_s();
    if (!h) return ILU_ENOMEM;
    if (int rc = setup_impl(tets, ntets, &o, st, h)) {
        (void)hipStreamSynchronize(st);
        delete h;
        return rc;
    }
    h->flow_grid = std::min(best_grid, h->flow_grid_max);
    h->ovl = h->ovl_ok ? best_ovl : ILU_OVERLAP_OFF;
    h->res_lds_t = best_rt;
    h->tuned_ms = best_ms;
    *out = h;
    return ILU_OK;
}


// The LDS-staged residual of BV x BW blocks (both of its work splits): every
// load address of every slice (own rows, halo rows, b; the zero slot at 0 for
// points outside the lattice) lies in the streams, and every value an active
// point reads from an LDS cell was staged from the address k_residual reads it
// from, or both addresses are zero slots.
template <int BV, int BW>
int64_t check_residual_lds(ilu_handle_t h, const std::vector<int32_t>& owner) {
    using G = RlGeo<BV, BW>;
    constexpr int NT = G::NT;
    const int64_t S = h->S;
    int64_t bad = 0;
    auto zero_slot = [&](int64_t q) { return q >= 0 && q < S && owner[q] == -1; };
    struct Src {
        int64_t rp = 0;
        RlRow row{0, 0};
        int arr = -1;
    };
    std::vector<Src> xs(G::XC), as(G::AC);
    for (size_t b = 0; b < h->blocks.size(); ++b) {
        const BlockDev& B = h->blocks[b];
        const LaneDev* Lb = &h->lanes[b * NT];
        const int n = h->tets[B.tet].n;
        for (int l = 0; l < NT; ++l) {
            const Src own{Lb[l].rp[R_SELF], rl_row(n, Lb[l].v, Lb[l].w), -1};
            xs[l] = own;
            for (int a = 2; a < 8; ++a) {
                as[(a - 2) * NT + l] = own;
                as[(a - 2) * NT + l].arr = a;
            }
        }
        for (int j = 0; j < G::NH; ++j) {
            const RlHalo o = rl_halo<BV, BW>(j);
            int sv = 0, sw = 0;
            lane_rc(o.src, BV, &sv, &sw);
            const Src sr{Lb[o.src].rp[o.slot],
                         rl_row(n, B.V0 + sv + rl_slot_dv(o.slot), B.W0 + sw + rl_slot_dw(o.slot)), o.arr};
            if (o.arr < 0) xs[o.dst] = sr;
            else as[o.dst] = sr;
        }
        auto addr = [&](const Src& sr, int T) { return rl_active(sr.row, T) ? sr.rp + (int64_t)NT * T : 0; };
        // the workgroups' hyperplane ranges: chunks of RES_T and of 2 RES_T from
        // the block's first hyperplane, and the absolute bands of the tagged mode
        std::vector<std::pair<int, int>> ranges;
        for (int len = RES_T; len <= 2 * RES_T; len += RES_T)
            for (int t0 = B.tb; t0 <= B.te; t0 += len) ranges.push_back({t0, std::min(B.te + 1, t0 + len)});
        for (int band = B.tb / RES_T; band * RES_T <= B.te; ++band)
            ranges.push_back({std::max(B.tb, band * RES_T), std::min(B.te + 1, (band + 1) * RES_T)});
        for (const auto& rg : ranges) {
            const int t0 = rg.first, t1 = rg.second, ucap = t1 + 2;
            // loads: slices t0 - 3 .. ucap of x and the arrays, b of t0 - 6 .. ucap
            for (int T = t0 - 3; T <= ucap; ++T) {
                for (int c = 0; c < G::XC; ++c) {
                    const int64_t q = addr(xs[c], T);
                    bad += q < 0 || q >= S;
                }
                for (int c = 0; c < G::AC; ++c) {
                    const int64_t q = addr(as[c], T);
                    bad += q < 0 || q >= S;
                }
            }
            for (int l = 0; l < NT; ++l)
                for (int u = t0 - 6; u <= ucap; ++u) {
                    const int64_t q = addr(xs[l], u);
                    bad += q < 0 || q >= S;
                }
            // the values of every active point
            for (int l = 0; l < NT; ++l) {
                const LaneDev& L = Lb[l];
                if (L.v == 0) continue;
                int vl = 0, wl = 0;
                lane_rc(l, BV, &vl, &wl);
                for (int t = t0; t < t1; ++t) {
                    const int xx = t - 2 * L.v - L.w;
                    if (xx < 1 || xx > n - 1 - L.v) continue;
                    bad += !rl_active(xs[l].row, t);
                    for (int s = 0; s < NLOW; ++s) {
                        int xl = 0, xu = 0, au = 0;
                        rl_cells<BV, BW>(vl, wl, s, &xl, &xu, &au);
                        const int64_t ql = L.rp[low_row(s)] + (int64_t)NT * (t + low_dt(s));
                        const int64_t qu = L.rp[up_row(s)] + (int64_t)NT * (t + up_dt(s));
                        const int64_t sl = addr(xs[xl], t + low_dt(s)), su = addr(xs[xu], t + up_dt(s));
                        bad += xs[xl].arr != -1 || xs[xu].arr != -1;
                        bad += sl != ql && !(zero_slot(sl) && zero_slot(ql));
                        bad += su != qu && !(zero_slot(su) && zero_slot(qu));
                        // upper weight: array 1 of the own row from registers (s = 0),
                        // else the LDS cell of the upper neighbour; lower weight of
                        // s >= 1: the own row's cell of array 1 + s
                        int64_t sa = 0;
                        if (s == 0) {
                            sa = addr(xs[l], t + up_dt(s));
                            bad += au != -1;
                        } else {
                            sa = addr(as[au], t + up_dt(s));
                            const Src& lo = as[(s - 1) * NT + l];
                            bad += as[au].arr != 1 + s || lo.arr != 1 + s;
                            bad += addr(lo, t) != L.rp[R_SELF] + (int64_t)NT * t;
                        }
                        bad += sa != qu && !(zero_slot(sa) && zero_slot(qu));
                    }
                }
            }
        }
    }
    return bad;
}

// Replays, on the host, every global index the kernels form and checks that
// it stays inside the streams and addresses the intended point (or a slot that
// is never written, which holds zero).  Returns the number of violations.
int64_t check_layout(ilu_handle_t h) {
    const int64_t S = h->S;
    const int bv = h->bv, bw = h->bw, LANES = bv * bw;
    std::vector<int32_t> owner(S, -1);  // written slot -> point id (block*64+lane, t) packed
    std::vector<int32_t> owner_t(S, -1);
    int64_t bad = 0;
    auto active = [&](const BlockDev& B, const LaneDev& L, int t, int* x) {
        if (L.v == 0 || t < B.tb || t > B.te) return false;
        const int n = h->tets[B.tet].n;
        *x = t - 2 * L.v - L.w;
        return *x >= 1 && *x <= n - 1 - L.v;
    };
    std::vector<int64_t> seen_lex(h->nlex, -1);
    for (size_t b = 0; b < h->blocks.size(); ++b) {
        const BlockDev& B = h->blocks[b];
        for (int l = 0; l < LANES; ++l) {
            const LaneDev& L = h->lanes[b * LANES + l];
            for (int t = B.tb; t <= B.te; ++t) {
                int x;
                if (!active(B, L, t, &x)) continue;
                const int64_t q = L.rp[R_SELF] + (int64_t)LANES * t;
                if (q < B.base || q >= B.base + (int64_t)B.len * LANES) { ++bad; continue; }
                if (owner[q] != -1) ++bad;
                owner[q] = (int32_t)(b * LANES + l);
                owner_t[q] = t;
                const TetDev& T = h->tets[B.tet];
                const int y = L.v - L.w, z = L.w;
                const int64_t mz = T.n - 1 - z;
                const int64_t li = T.lex_off + choose3_h(T.n - 1) - choose3_h(T.n - z) + (int64_t)(y - 1) * mz -
                                   (int64_t)(y - 1) * y / 2 + (x - 1);
                if (li < T.lex_off || li >= T.lex_off + T.N || seen_lex[li] != -1) ++bad;
                else seen_lex[li] = q;
            }
        }
    }
    for (int64_t i = 0; i < h->nlex; ++i) bad += seen_lex[i] < 0;
    // global lanes of the neighbour rows (the setup's hyperplane ring): the
    // lane they name holds the row the row pointer names, or both are outside
    {
        static const int dv[7] = {0, -1, 0, -1, 1, 0, 1}, dw[7] = {0, 0, -1, -1, 0, 1, 1};
        for (size_t b = 0; b < h->blocks.size(); ++b)
            for (int l = 0; l < LANES; ++l) {
                const LaneDev& L = h->lanes[b * LANES + l];
                if (L.v == 0) {
                    bad += L.gl[R_SELF] != -1;
                    continue;
                }
                for (int sl = 0; sl < 7; ++sl) {
                    const int32_t g = L.gl[sl];
                    if (g < 0) {
                        bad += L.rp[sl] != 0;
                        continue;
                    }
                    if ((size_t)g >= h->lanes.size()) {
                        ++bad;
                        continue;
                    }
                    const LaneDev& M = h->lanes[g];
                    if (M.v != L.v + dv[sl] || M.w != L.w + dw[sl] || M.rp[R_SELF] != L.rp[sl] ||
                        h->blocks[g / LANES].tet != h->blocks[b].tet)
                        ++bad;
                }
            }
    }
    static const int dx[7] = {-1, 0, 1, -1, 0, 0, 1}, dy[7] = {0, -1, -1, 1, 1, 0, 0}, dz[7] = {0, 0, 0, -1, -1, -1, -1};
    static const int lrow[7] = {R_SELF, R_VM, R_VM, R_WM, R_WM, R_VMWM, R_VMWM};
    static const int urow[7] = {R_SELF, R_VP, R_VP, R_WP, R_WP, R_VPWP, R_VPWP};
    // neighbour accesses of the residual, plane and dataflow kernels
    for (size_t b = 0; b < h->blocks.size(); ++b) {
        const BlockDev& B = h->blocks[b];
        const int n = h->tets[B.tet].n;
        for (int l = 0; l < LANES; ++l) {
            const LaneDev& L = h->lanes[b * LANES + l];
            for (int t = B.tb; t <= B.te; ++t) {
                int x;
                if (!active(B, L, t, &x)) continue;
                const int y = L.v - L.w, z = L.w;
                for (int s = 0; s < 7; ++s)
                    for (int sg = -1; sg <= 1; sg += 2) {
                        const int ex = sg * dx[s], ey = sg * dy[s], ez = sg * dz[s];
                        const int dt = ex + 2 * ey + 3 * ez;
                        const int64_t q = L.rp[sg < 0 ? urow[s] : lrow[s]] + (int64_t)LANES * (t + dt);
                        if (q < 0 || q >= S) { ++bad; continue; }
                        const int nx = x + ex, ny = y + ey, nz = z + ez;
                        const bool in = nx >= 1 && ny >= 1 && nz >= 1 && nx + ny + nz <= n - 1;
                        if (!in) { bad += owner[q] != -1; continue; }
                        const int o = owner[q];
                        if (o < 0 || owner_t[q] != t + dt) { ++bad; continue; }
                        const LaneDev& M = h->lanes[o];
                        if (M.v != ny + nz || M.w != nz || h->blocks[o / LANES].tet != B.tet) ++bad;
                    }
            }
        }
    }
    // residual: every load and store address of every lane and hyperplane of
    // the block range (inactive points and the clamped second point included)
    for (size_t b = 0; b < h->blocks.size(); ++b) {
        const BlockDev& B = h->blocks[b];
        for (int l = 0; l < LANES; ++l) {
            const LaneDev& L = h->lanes[b * LANES + l];
            for (int t = B.tb; t <= B.te + 1; ++t) {
                const int64_t off = (int64_t)LANES * t;
                if (L.rp[R_SELF] + off < 0 || L.rp[R_SELF] + off >= S) ++bad;
                for (int s = 0; s < 7; ++s) {
                    const int64_t ql = L.rp[lrow[s]] + off + (int64_t)LANES * (dx[s] + 2 * dy[s] + 3 * dz[s]);
                    const int64_t qu = L.rp[urow[s]] + off - (int64_t)LANES * (dx[s] + 2 * dy[s] + 3 * dz[s]);
                    if (ql < 0 || ql >= S || qu < 0 || qu >= S) ++bad;
                }
            }
        }
    }
    if (bv == 8 && bw == 8) bad += check_residual_lds<8, 8>(h, owner);
    if (bv == 16 && bw == 16) bad += check_residual_lds<16, 16>(h, owner);
    // dataflow exchange: replay the outgoing-entry stores of every block and
    // hyperplane with the kernels' own index functions, then check that every
    // halo read lands on a word written by the producer lane that owns the
    // halo row (rows outside the lattice: no producer, or an unused producer
    // lane, which writes zeros)
    for (int dir = 0; dir < 2; ++dir)
        for (int wds = 1; wds <= 2; ++wds) {
            const int nx = bv + bw;
            const int64_t nw = h->XE * wds;
            std::vector<int64_t> wr_lane(nw, -1);
            std::vector<int32_t> wr_t(nw, -1);
            for (size_t b = 0; b < h->blocks.size(); ++b) {
                const BlockDev& B = h->blocks[b];
                for (int j = 0; j < nx; ++j) {
                    int vl, wl;
                    xch_out_lane(dir, j, bv, bw, &vl, &wl);
                    const int l = lane_at(vl, wl, bv);
                    if (vl < 0 || vl >= bv || wl < 0 || wl >= bw) { ++bad; continue; }
                    for (int t = B.tb; t <= B.te; ++t) {
                        const int64_t q = xch_word(B.xoff, B.tlo, nx, wds, t, j);
                        if (q < B.xoff * wds || q + wds > (B.xoff + (int64_t)B.len * nx) * wds || q + wds > nw) {
                            ++bad;
                            continue;
                        }
                        if (wr_lane[q] != -1) ++bad;  // one writer per word and sweep
                        wr_lane[q] = (int64_t)(b * LANES + l);
                        wr_t[q] = t;
                    }
                }
            }
            for (size_t b = 0; b < h->blocks.size(); ++b) {
                const BlockDev& B = h->blocks[b];
                const int n = h->tets[B.tet].n;
                for (int l = 0; l < LANES; ++l) {
                    int k, j;
                    if (!xch_halo_role(dir, l, bv, bw, &k, &j)) continue;
                    // the halo row this role stands for
                    const int edge_v = dir == 0 ? B.V0 - 1 : B.V0 + bv, edge_w = dir == 0 ? B.W0 - 1 : B.W0 + bw;
                    int v, w;
                    if (k == 0) { v = edge_v; w = B.W0 + l; }
                    else if (k == 1) { v = B.V0 + (l - bw); w = edge_w; }
                    else { v = edge_v; w = edge_w; }
                    const bool in = v >= 2 && v <= n - 2 && w >= 1 && w <= v - 1;
                    const int prod = dir == 0 ? B.pred[k] : B.succ[k];
                    if (prod < 0) { bad += in; continue; }
                    const BlockDev& PB = h->blocks[prod];
                    if (PB.tet != B.tet) { ++bad; continue; }
                    for (int s = PB.tb; s <= PB.te; ++s) {
                        const int64_t q = xch_word(PB.xoff, PB.tlo, nx, wds, s, j);
                        if (q < 0 || q + wds > nw || wr_lane[q] < 0 || wr_t[q] != s || wr_lane[q] / LANES != prod) {
                            ++bad;
                            continue;
                        }
                        const LaneDev& PL = h->lanes[wr_lane[q]];
                        if (in ? (PL.v != v || PL.w != w) : PL.v != 0) ++bad;
                    }
                }
            }
        }
    // topological orders
    for (int dir = 0; dir < 2; ++dir) {
        std::vector<int32_t> ord = topo_order(h->blocks, dir == 0);
        if (ord.size() != h->blocks.size()) { ++bad; continue; }
        std::vector<int> pos(ord.size());
        for (size_t k = 0; k < ord.size(); ++k) pos[ord[k]] = (int)k;
        for (size_t b = 0; b < h->blocks.size(); ++b)
            for (int k = 0; k < 3; ++k) {
                const int p = dir == 0 ? h->blocks[b].pred[k] : h->blocks[b].succ[k];
                if (p >= 0 && pos[p] >= pos[b]) ++bad;
            }
    }
    // sample indices: every sample point maps to a distinct slot of its simplex
    if (h->variant != ILU_STORED_F64) {
        static const int fd[8][3] = {{-1, 0, 0}, {0, -1, 0}, {1, -1, 0}, {-1, 1, -1},
                                     {0, 1, -1}, {0, 0, -1}, {1, 0, -1}, {0, 0, 0}};
        for (const TetDev& T : h->tets)
            for (int f = 0; f < NFIT; ++f) {
                std::vector<char> hit(T.samp_cnt[f], 0);
                const int st = T.stride, M = T.samp_M[f];
                const int sx = 1 - std::min(fd[f][0], 0), sy = 1 - std::min(fd[f][1], 0), sz = 1 - std::min(fd[f][2], 0);
                for (int z = 1; z <= T.n - 3; ++z)
                    for (int y = 1; y <= T.n - 2 - z; ++y)
                        for (int x = 1; x <= T.n - 1 - y - z; ++x) {
                            if ((x - sx) % st || (y - sy) % st || (z - sz) % st) continue;
                            const int qx = x + fd[f][0], qy = y + fd[f][1], qz = z + fd[f][2];
                            if (!(qx >= 1 && qy >= 1 && qz >= 1 && qx + qy + qz <= T.n - 1)) continue;
                            const int kx = (x - sx) / st, ky = (y - sy) / st, kz = (z - sz) / st;
                            const int64_t Mz = M - kz;
                            const int64_t si = choose3_h(M + 3) - choose3_h(M + 3 - kz) + (int64_t)ky * (Mz + 1) -
                                               (int64_t)ky * (ky - 1) / 2 + kx;
                            if (si < 0 || si >= T.samp_cnt[f] || hit[si]) ++bad;
                            else hit[si] = 1;
                        }
                for (char c : hit) bad += !c;
            }
    }
    return bad;
}

void sweep_fwd(ilu_handle_t h, const Ctx& c, hipStream_t st) {
    if (h->schedule == ILU_SCHED_PLANE) {
        for (int t = h->tmin; t <= h->tmax; ++t) launch_fwd_plane(c, h->variant, t, st);
    } else {
        const Flow f = h->flow();
        launch_flow_reset(f, st);
        launch_fwd_flow(c, f, h->variant, st);
    }
}

// Backward substitution; the correction is added to `target` (default: the
// iterate x of the smoother).
void sweep_bwd(ilu_handle_t h, const Ctx& c, hipStream_t st, double* target) {
    double* x = target ? target : h->xs.as<double>();
    if (h->schedule == ILU_SCHED_PLANE) {
        for (int t = h->tmax; t >= h->tmin; --t) launch_bwd_plane(c, h->variant, t, x, st);
    } else {
        const Flow f = h->flow();
        launch_flow_reset(f, st);
        launch_bwd_flow(c, f, h->variant, x, st);
    }
}

// Residual and forward substitution of one sweep.  With the overlap the
// residual kernel runs on the handle's second stream and writes tagged entries
// that the forward sweep consumes as they appear (a missing one it computes
// itself); the join makes later work on `st` (norms, the backward sweep) see
// the finished residual kernel, its partial sums included.  mk: six timing
// events of this sweep (residual begin/end, forward begin/end; the backward
// pair is recorded by the caller) or null.
int sweep_res_fwd(ilu_handle_t h, const Ctx& c, hipStream_t st, double* partial, hipEvent_t* mk) {
    const bool f32 = h->variant == ILU_SURR_F32;
    if (!h->ovl) {
        if (mk) HIPCHK(hipEventRecord(mk[0], st));
        launch_residual(c, h->xs.as<double>(), h->bs.as<double>(), h->r.p, f32, 1, partial, st);
        if (mk) HIPCHK(hipEventRecord(mk[1], st));
        if (mk) HIPCHK(hipEventRecord(mk[2], st));
        sweep_fwd(h, c, st);
        if (mk) HIPCHK(hipEventRecord(mk[3], st));
        return ILU_OK;
    }
    Flow f = h->flow();
    f.rt = h->rt.as<uint64_t>();
    f.rflag = h->rflag.as<uint64_t>();
    f.nbands = c.res_bands;
    f.xo = h->xs.as<double>();
    f.bo = h->bs.as<double>();
    launch_flow_reset(f, st);  // the tag of this sweep, read by both kernels
    if (h->ovl == ILU_OVERLAP_FUSED && !partial) {
        // no residual kernel: no entry carries this sweep's tag, and the
        // forward sweep computes every residual itself without polling
        f.rspin = 0;
        if (mk) HIPCHK(hipEventRecord(mk[0], st));
        if (mk) HIPCHK(hipEventRecord(mk[1], st));
        if (mk) HIPCHK(hipEventRecord(mk[2], st));
        launch_fwd_flow(c, f, h->variant, st);
        if (mk) HIPCHK(hipEventRecord(mk[3], st));
        return ILU_OK;
    }
    f.rspin = 64;  // about 64 us of polling before computing a missing value
    HIPCHK(hipEventRecord(h->oev[0], st));
    HIPCHK(hipStreamWaitEvent(h->st2, h->oev[0], 0));
    if (mk) HIPCHK(hipEventRecord(mk[0], h->st2));
    launch_residual_tagged(c, h->xs.as<double>(), h->bs.as<double>(), h->rt.as<uint64_t>(), f32, f.ticket + 2,
                           h->rflag.as<uint64_t>(),
                           partial, h->st2);
    if (mk) HIPCHK(hipEventRecord(mk[1], h->st2));
    HIPCHK(hipEventRecord(h->oev[1], h->st2));
    if (mk) HIPCHK(hipEventRecord(mk[2], st));
    launch_fwd_flow(c, f, h->variant, st);
    if (mk) HIPCHK(hipEventRecord(mk[3], st));
    HIPCHK(hipStreamWaitEvent(st, h->oev[1], 0));
    return ILU_OK;
}

// One PCG iteration, entirely on the device (scalars in cg_sc):
//   q = A p;  alpha = (r.z) / (p.q);  x += alpha p;  r -= alpha q;
//   z = C^{-1} r (forward and backward substitution from zero);
//   beta = (r.z)_new / (r.z);  p = z + beta p.
// Once the tolerance is met the scalar kernels freeze x, r and p, so extra
// iterations change nothing.  Kernel nodes only: it can be captured.
void cg_iteration(ilu_handle_t h, const Ctx& c, hipStream_t st) {
    double* sc = h->cg_sc.as<double>();
    double* part = h->partial.as<double>();
    double *p = h->cg_p.as<double>(), *q = h->cg_q.as<double>(), *r = h->cg_r.as<double>(),
           *z = h->cg_z.as<double>();
    launch_residual(c, p, nullptr, q, false, 0, nullptr, st);
    launch_dot(c, p, q, part, st);
    launch_reduce(part, h->npartial, sc, CG_PQ, st);
    launch_cg_scalar(sc, CG_STEP_ALPHA, 0.0, 0.0, st);
    launch_cg_update(c, h->variant == ILU_SURR_F32, h->xs.as<double>(), p, r, q, z, h->r.p, sc, part, st);
    launch_reduce(part, h->npartial, sc, CG_RR, st);
    launch_cg_scalar(sc, CG_CHECK, 0.0, 0.0, st);
    sweep_fwd(h, c, st);
    sweep_bwd(h, c, st, z);
    launch_dot(c, r, z, part, st);
    launch_reduce(part, h->npartial, sc, CG_RZNEW, st);
    launch_cg_scalar(sc, CG_STEP_BETA, 0.0, 0.0, st);
    launch_cg_direction(c, p, z, sc, st);
}

int capture_cg(ilu_handle_t h, const Ctx& c) {
    if (!h->cap) HIPCHK(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
    cg_iteration(h, c, h->cap);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(h->cap, &g);
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture", __LINE__);
    const hipError_t e2 = hipGraphInstantiate(&h->cg_exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e2 != hipSuccess) {
        h->cg_exec = nullptr;
        return hip_fail(e2, "hipGraphInstantiate", __LINE__);
    }
    return ILU_OK;
}

// Capture `count` sweeps (each: residual, forward and backward substitution
// over every tetrahedron of the handle) into one executable graph.  It only
// touches handle-owned buffers, so it stays valid for the life of the handle;
// it holds kernel nodes only, and the dataflow tag is advanced by a kernel on
// device before every substitution, so every replay runs fresh sweeps.
int capture_sweeps(ilu_handle_t h, const Ctx& c, int count, hipGraphExec_t* out) {
    if (!h->cap) HIPCHK(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
    int rc = ILU_OK;
    for (int k = 0; k < count && rc == ILU_OK; ++k) {
        rc = sweep_res_fwd(h, c, h->cap, nullptr, nullptr);
        if (rc == ILU_OK) sweep_bwd(h, c, h->cap);
    }
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(h->cap, &g);  // also after a failed launch: leave no open capture
    if (rc != ILU_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture", __LINE__);
    const hipError_t e2 = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e2 != hipSuccess) {
        *out = nullptr;
        return hip_fail(e2, "hipGraphInstantiate", __LINE__);
    }
    return ILU_OK;
}

// Forget the captured graphs (they are recaptured on the next call): their
// kernel nodes hold buffer addresses that a table rebuild replaces.
int drop_graphs(ilu_handle_t h, hipStream_t st) {
    (void)st;
    HIPCHK(hipDeviceSynchronize());  // a replay may be in flight on any stream
    if (h->gexec) HIPCHK(hipGraphExecDestroy(h->gexec));
    if (h->gexec_n) HIPCHK(hipGraphExecDestroy(h->gexec_n));
    h->gexec_n = nullptr;
    h->gexec_count = 0;
    if (h->cg_exec) HIPCHK(hipGraphExecDestroy(h->cg_exec));
    h->gexec = nullptr;
    h->cg_exec = nullptr;
    return ILU_OK;
}

double host_norm(ilu_handle_t h, int slot, hipStream_t st, int* err) {
    double v = 0.0;
    *err = hipMemcpyAsync(&v, h->norms.as<double>() + slot, sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
           hipStreamSynchronize(st) != hipSuccess;
    return v;
}

}  // namespace

namespace {
// Arguments of the LFA orientation calls: sizes, finite vertices, and a
// non-degenerate tetrahedron (either orientation).
int lfa_check_args(const ilu_tet_desc* tets, int32_t ntets, int32_t samples, const double* mu_out,
                   const int32_t* best_out) {
    if (!tets || ntets <= 0 || (!mu_out && !best_out) || samples < 4 || samples > 256 || samples % 4) return ILU_EINVAL;
    for (int i = 0; i < ntets; ++i) {
        for (int a = 0; a < 4; ++a)
            for (int r = 0; r < 3; ++r)
                if (!std::isfinite(tets[i].vertex[a][r])) return ILU_EINVAL;
        double E[3][3];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) E[r][c] = tets[i].vertex[c + 1][r] - tets[i].vertex[0][r];
        const double det = E[0][0] * (E[1][1] * E[2][2] - E[1][2] * E[2][1]) -
                           E[0][1] * (E[1][0] * E[2][2] - E[1][2] * E[2][0]) +
                           E[0][2] * (E[1][0] * E[2][1] - E[1][1] * E[2][0]);
        if (!(std::fabs(det) > 0.0) || !std::isfinite(det)) return ILU_EGEOM;
    }
    return ILU_OK;
}

// Scratch of ilu_lfa_orientation_noalloc: one statically sized device array,
// carved into the descriptors as given (the kernel reads the vertices with the
// descriptor stride), the per-(tetrahedron, permutation) records, mu and the
// chosen permutations.  Every part is fully written before it is read, so no
// clearing is needed.  Host code never passes `scratch` itself to a kernel
// (its name is a host-side stand-in): it uses the per-device address from
// hipGetSymbolAddress.
constexpr size_t align256(size_t b) { return (b + 255) / 256 * 256; }
constexpr size_t LFA_SCR_DESC = 0;
constexpr size_t LFA_SCR_REC = LFA_SCR_DESC + align256(sizeof(ilu_tet_desc) * ILU_LFA_NOALLOC_MAX_TETS);
constexpr size_t LFA_SCR_MU = LFA_SCR_REC + align256(sizeof(double) * LFA_REC * LFA_PERMS * ILU_LFA_NOALLOC_MAX_TETS);
constexpr size_t LFA_SCR_BEST = LFA_SCR_MU + align256(sizeof(double) * LFA_PERMS * ILU_LFA_NOALLOC_MAX_TETS);
constexpr size_t LFA_SCR_BYTES = LFA_SCR_BEST + align256(sizeof(int32_t) * ILU_LFA_NOALLOC_MAX_TETS);
static_assert(sizeof(ilu_tet_desc) % sizeof(double) == 0, "descriptor stride in doubles");
static_assert(offsetof(ilu_tet_desc, vertex) == 0, "vertices lead the descriptor");

}  // namespace

static __device__ __align__(256) unsigned char scratch[LFA_SCR_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on the current device, looked up once per
// device (each device holds its own copy of the array).
int scratch_address(void** out) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return ILU_EINVAL;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return ILU_EHIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return ILU_OK;
}

int validate_args(const ilu_tet_desc* tets, int32_t ntets, const ilu_opts* opts) {
    if (opts->variant < ILU_STORED_F64 || opts->variant > ILU_STORED_SGS) return ILU_EINVAL;
    if (opts->boundary != ILU_BOUNDARY_V2 && opts->boundary != ILU_BOUNDARY_V1) return ILU_EINVAL;
    if (opts->boundary == ILU_BOUNDARY_V1 && opts->variant != ILU_SURR_F64 && opts->variant != ILU_SURR_F32)
        return ILU_EINVAL;
    if (opts->a_mode != ILU_A_EXACT && opts->a_mode != ILU_A_SURROGATE) return ILU_EINVAL;
    if (opts->a_mode == ILU_A_SURROGATE && opts->variant != ILU_SURR_F64 && opts->variant != ILU_SURR_F32)
        return ILU_EINVAL;
    if ((opts->tile[0] || opts->tile[1]) && !flow_shape_supported(opts->tile[0], opts->tile[1])) return ILU_EINVAL;
    if (opts->variant == ILU_SURR_F64 || opts->variant == ILU_SURR_F32) {
        for (int k = 0; k < 3; ++k)
            if (opts->degree[k] < 0 || opts->degree[k] > 6) return ILU_EINVAL;
        if (opts->sample_stride < 0 || (opts->sample_stride & (opts->sample_stride - 1))) return ILU_EINVAL;
    }
    for (int i = 0; i < ntets; ++i) {
        if (tets[i].level < 2 || tets[i].level > 10) return ILU_EINVAL;
        if (tets[i].coeff_kind < 0 || tets[i].coeff_kind > 3) return ILU_EINVAL;
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 3; ++b)
                if (!std::isfinite(tets[i].vertex[a][b])) return ILU_EINVAL;
    }
    return ILU_OK;
}
}  // namespace

extern "C" {

const char* ilu_last_error(void) { return g_last_error; }

const char* ilu_strerror(int code) {
    switch (code) {
    case ILU_OK: return "success";
    case ILU_EINVAL: return "invalid argument";
    case ILU_ENOMEM: return "device allocation failed";
    case ILU_EHIP: return "HIP runtime error";
    case ILU_EBREAKDOWN: return "ILU(0) breakdown: non-positive pivot";
    case ILU_ERANK: return "rank-deficient least-squares problem";
    case ILU_EGEOM: return "degenerate or inverted tetrahedron";
    case ILU_ENOTCONV: return "relative residual tolerance not reached";
    default: return "unknown error";
    }
}

namespace {
int setup_any(const ilu_tet_desc* tets, int32_t ntets, const ilu_opts* opts, hipStream_t st, ilu_handle_t* out) {
    if (opts->tile[0] == 0 && opts->tile[1] == 0 && opts->schedule != ILU_SCHED_PLANE)
        return setup_autotuned(tets, ntets, opts, st, out);
    ilu_handle_t h = new (std::nothrow) ilu_handle_s();
    if (!h) return ILU_ENOMEM;
    const int rc = setup_impl(tets, ntets, opts, st, h);
    if (rc != ILU_OK) {
        (void)hipStreamSynchronize(st);
        delete h;
        return rc;
    }
    *out = h;
    return ILU_OK;
}
}  // namespace

int ilu_setup_surrogate(const ilu_tet_desc* tets, int32_t ntets, const ilu_opts* opts, void* hip_stream,
                        ilu_handle_t* out) {
    if (!tets || !opts || !out || ntets <= 0) return ILU_EINVAL;
    *out = nullptr;
    if (int e = validate_args(tets, ntets, opts)) return e;
    static std::atomic<uint64_t> epochs{0};
    SetupMem& m = g_setup_mem;
    m = SetupMem{++epochs, true, 0, 0};
    const int rc = setup_any(tets, ntets, opts, (hipStream_t)hip_stream, out);
    m.on = false;
    if (rc == ILU_OK) {
        (*out)->setup_peak = m.peak;
        (*out)->setup_resident = m.cur;
    }
    return rc;
}

int ilu_setup_memory(ilu_handle_t h, int64_t* peak_bytes, int64_t* resident_bytes) {
    if (!h) return ILU_EINVAL;
    if (peak_bytes) *peak_bytes = h->setup_peak;
    if (resident_bytes) *resident_bytes = h->setup_resident;
    return ILU_OK;
}

int ilu_check_layout(const ilu_tet_desc* tets, int32_t ntets, const ilu_opts* opts, int64_t* violations) {
    if (!tets || !opts || !violations || ntets <= 0) return ILU_EINVAL;
    if (int e = validate_args(tets, ntets, opts)) return e;
    ilu_handle_t h = new (std::nothrow) ilu_handle_s();
    if (!h) return ILU_ENOMEM;
    int64_t ns = 0;
    int rc = prepare(tets, ntets, opts, h, &ns);
    if (rc == ILU_OK) *violations = check_layout(h);
    delete h;
    return rc;
}

int ilu_destroy(ilu_handle_t h) {
    if (!h) return ILU_OK;
    (void)hipDeviceSynchronize();
    delete h;
    return ILU_OK;
}

int ilu_layout(ilu_handle_t h, int32_t tet, int64_t* offset, int64_t* count_interior) {
    if (!h || tet < 0 || tet >= h->ntets) return ILU_EINVAL;
    if (offset) *offset = h->tets[tet].lex_off;
    if (count_interior) *count_interior = h->tets[tet].N;
    return ILU_OK;
}

int ilu_smooth(ilu_handle_t h, double* x, const double* b, int32_t nsweeps, double rel_tol, double* relres_out,
               void* hip_stream) {
    if (!h || !x || !b || nsweeps < 0 || !(rel_tol >= 0.0)) return ILU_EINVAL;
    hipStream_t st = (hipStream_t)hip_stream;
    const Ctx c = h->ctx();
    const bool f32 = h->variant == ILU_SURR_F32;
    launch_permute_in2(c, x, h->xs.as<double>(), b, h->bs.as<double>(), st);
    HIPCHK(hipGetLastError());
    const bool want_norm = rel_tol > 0.0 || relres_out;
    double bn = 1.0;
    int err = 0;
    if (want_norm) {
        launch_sumsq(c, h->bs.as<double>(), h->partial.as<double>(), st);
        launch_reduce(h->partial.as<double>(), h->npartial, h->norms.as<double>(), 0, st);
        bn = std::sqrt(host_norm(h, 0, st, &err));
        if (err) return ILU_EHIP;
        if (bn == 0.0) bn = 1.0;
    }
    double rel = -1.0;
    bool converged = false;
    if (h->kernel_timing && (int)h->kev.size() < 6 * nsweeps) {
        const size_t old = h->kev.size();
        h->kev.resize(6 * (size_t)nsweeps, nullptr);
        for (size_t i = old; i < h->kev.size(); ++i) HIPCHK(hipEventCreate(&h->kev[i]));
    }
    // timing events of sweep k: all sweeps with kernel timing on, else the first
    auto marks = [&](int k) -> hipEvent_t* {
        if (h->kernel_timing) return &h->kev[6 * (size_t)k];
        return k == 0 ? &h->ev[2] : nullptr;
    };
    int done = 0;
    // fixed number of sweeps: replay the captured one-sweep graph
    const bool graph = h->use_graph && rel_tol == 0.0 && !h->kernel_timing && nsweeps > 0;
    // up to MULTI sweeps run as one graph holding all of them (captured for the
    // count asked for, kept until another count is asked for); longer runs
    // replay the one-sweep graph
    constexpr int MULTI = 64;
    const bool multi = graph && nsweeps > 1 && nsweeps <= MULTI;
    if (multi && h->gexec_count != nsweeps) {
        if (h->gexec_n) HIPCHK(hipGraphExecDestroy(h->gexec_n));
        h->gexec_n = nullptr;
        h->gexec_count = 0;
        if (int e = capture_sweeps(h, c, nsweeps, &h->gexec_n)) return e;
        h->gexec_count = nsweeps;
    }
    if (graph && !multi && !h->gexec)
        if (int e = capture_sweeps(h, c, 1, &h->gexec)) return e;
    HIPCHK(hipEventRecord(h->ev[0], st));
    if (multi) {
        HIPCHK(hipGraphLaunch(h->gexec_n, st));
        done = nsweeps;
    }
    for (int k = 0; graph && !multi && k < nsweeps; ++k) {
        HIPCHK(hipGraphLaunch(h->gexec, st));
        ++done;
    }
    // eager sweeps.  With rel_tol > 0 they run in chunks of CHK: every sweep's
    // residual kernel also reduces ||b - A x||^2 into its own slot, and after
    // a chunk one read of those slots tells whether the tolerance was met; if
    // so, the current x is checked directly (the residual need not fall
    // monotonically) and the loop ends once it passes.
    constexpr int CHK = 8;
    bool final_known = false;
    while (!graph && done < nsweeps) {
        const int m = rel_tol > 0.0 ? std::min(CHK, nsweeps - done) : nsweeps - done;
        for (int j = 0; j < m; ++j) {
            hipEvent_t* mk = marks(done + j);
            if (int e = sweep_res_fwd(h, c, st, rel_tol > 0.0 ? h->partial.as<double>() : nullptr, mk)) return e;
            if (rel_tol > 0.0)
                launch_reduce(h->partial.as<double>(), h->ovl ? h->npartial_tag : h->npartial, h->norms.as<double>(),
                              2 + j, st);
            if (mk) HIPCHK(hipEventRecord(mk[4], st));
            sweep_bwd(h, c, st);
            if (mk) HIPCHK(hipEventRecord(mk[5], st));
        }
        done += m;
        if (rel_tol > 0.0) {
            double nv[CHK];
            HIPCHK(hipMemcpyAsync(nv, h->norms.as<double>() + 2, m * sizeof(double), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            bool hit = false;
            for (int j = 0; j < m; ++j) hit = hit || std::sqrt(nv[j]) / bn <= rel_tol;
            if (hit) {
                launch_residual(c, h->xs.as<double>(), h->bs.as<double>(), h->r.p, f32, 1, h->partial.as<double>(), st);
                launch_reduce(h->partial.as<double>(), h->npartial, h->norms.as<double>(), 1, st);
                rel = std::sqrt(host_norm(h, 1, st, &err)) / bn;
                if (err) return ILU_EHIP;
                final_known = true;
                if (rel <= rel_tol) {
                    converged = true;
                    break;
                }
            }
        }
    }
    HIPCHK(hipEventRecord(h->ev[1], st));
    HIPCHK(hipGetLastError());
    h->have_timing = done > 0;
    h->kev_sweeps = graph ? 0 : h->kernel_timing ? done : (done > 0 ? 1 : 0);
    h->last_sweeps = done;
    if (want_norm && !final_known) {
        launch_residual(c, h->xs.as<double>(), h->bs.as<double>(), h->r.p, f32, 1, h->partial.as<double>(), st);
        launch_reduce(h->partial.as<double>(), h->npartial, h->norms.as<double>(), 1, st);
        rel = std::sqrt(host_norm(h, 1, st, &err)) / bn;
        if (err) return ILU_EHIP;
        converged = rel <= rel_tol;
    }
    if (relres_out) *relres_out = rel;
    launch_permute(c, 0, 1, h->xs.as<double>(), x, h->S, 1, -1, st);
    HIPCHK(hipGetLastError());
    if (h->schedule != ILU_SCHED_PLANE) {
        int32_t fl[4];
        if (int e = read_flags(h, st, fl)) return e;
        if (fl[2]) return ILU_EHIP;  // a dataflow wait exceeded its bound
    }
    if (rel_tol > 0.0 && !converged) return ILU_ENOTCONV;
    return ILU_OK;
}

int stencil_apply(ilu_handle_t h, const double* x, double* y, void* hip_stream) {
    if (!h || !x || !y) return ILU_EINVAL;
    hipStream_t st = (hipStream_t)hip_stream;
    const Ctx c = h->ctx();
    launch_permute(c, 1, 1, x, h->xs.as<double>(), h->S, 1, -1, st);
    // y = A x in FP64 (the residual kernel with subtract = 0), stored in bs
    launch_residual(c, h->xs.as<double>(), nullptr, h->bs.as<double>(), false, 0, nullptr, st);
    launch_permute(c, 0, 1, h->bs.as<double>(), y, h->S, 1, -1, st);
    HIPCHK(hipGetLastError());
    return ILU_OK;
}

int ilu_pcg(ilu_handle_t h, double* x, const double* b, int32_t maxit, double rel_tol, double abs_tol,
            int32_t* iters_out, double* resnorm_out, void* hip_stream) {
    if (!h || !x || !b || maxit < 0 || !(rel_tol >= 0.0) || !(abs_tol >= 0.0)) return ILU_EINVAL;
    hipStream_t st = (hipStream_t)hip_stream;
    const Ctx c = h->ctx();
    const size_t vb = (size_t)h->S * sizeof(double);
    if (!h->cg_sc.p) {
        if (h->cg_r.alloc(vb, st) || h->cg_z.alloc(vb, st) || h->cg_p.alloc(vb, st) || h->cg_q.alloc(vb, st) ||
            h->cg_sc.alloc(CG_NSLOT * sizeof(double), st))
            return ILU_ENOMEM;
    }
    double* sc = h->cg_sc.as<double>();
    double* part = h->partial.as<double>();
    double *r = h->cg_r.as<double>(), *z = h->cg_z.as<double>(), *p = h->cg_p.as<double>();
    launch_permute_in2(c, x, h->xs.as<double>(), b, h->bs.as<double>(), st);
    HIPCHK(hipMemsetAsync(p, 0, vb, st));
    HIPCHK(hipMemsetAsync(h->cg_q.p, 0, vb, st));
    launch_sumsq(c, h->bs.as<double>(), part, st);
    launch_reduce(part, h->npartial, sc, CG_BB, st);
    launch_cg_scalar(sc, CG_SETUP, rel_tol, abs_tol, st);
    // r = b - A x, z = C^{-1} r, p = z
    launch_residual(c, h->xs.as<double>(), h->bs.as<double>(), r, false, 1, nullptr, st);
    launch_cg_update(c, h->variant == ILU_SURR_F32, h->xs.as<double>(), p, r, h->cg_q.as<double>(), z, h->r.p, sc,
                     part, st);
    launch_reduce(part, h->npartial, sc, CG_RR, st);
    sweep_fwd(h, c, st);
    sweep_bwd(h, c, st, z);
    launch_dot(c, r, z, part, st);
    launch_reduce(part, h->npartial, sc, CG_RZNEW, st);
    launch_cg_scalar(sc, CG_INIT, 0.0, 0.0, st);
    launch_cg_direction(c, p, z, sc, st);
    HIPCHK(hipGetLastError());
    const bool graph = h->use_graph && !h->kernel_timing && maxit > 0;
    if (graph && !h->cg_exec)
        if (int e = capture_cg(h, c)) return e;
    // the host looks at the device state after every CHK iterations
    constexpr int CHK = 8;
    double state[CG_NSLOT];
    int issued = 0;
    for (;;) {
        HIPCHK(hipMemcpyAsync(state, sc, sizeof(state), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (state[CG_DONE] != 0.0 || issued >= maxit) break;
        const int m = std::min(CHK, maxit - issued);
        for (int j = 0; j < m; ++j) {
            if (graph) HIPCHK(hipGraphLaunch(h->cg_exec, st));
            else cg_iteration(h, c, st);
        }
        HIPCHK(hipGetLastError());
        issued += m;
    }
    if (iters_out) *iters_out = (int32_t)state[CG_ITERS];
    if (resnorm_out) {
        // true residual of the returned iterate (q is free here)
        launch_residual(c, h->xs.as<double>(), h->bs.as<double>(), h->cg_q.as<double>(), false, 1, part, st);
        launch_reduce(part, h->npartial, h->norms.as<double>(), 1, st);
        int err = 0;
        *resnorm_out = std::sqrt(host_norm(h, 1, st, &err));
        if (err) return ILU_EHIP;
    }
    launch_permute(c, 0, 1, h->xs.as<double>(), x, h->S, 1, -1, st);
    HIPCHK(hipGetLastError());
    int32_t fl[4];
    if (int e = read_flags(h, st, fl)) return e;
    if (h->schedule != ILU_SCHED_PLANE && fl[2]) return ILU_EHIP;  // a dataflow wait exceeded its bound
    if (state[CG_BREAK] != 0.0) return ILU_EBREAKDOWN;
    if (state[CG_DONE] == 0.0) return ILU_ENOTCONV;
    return ILU_OK;
}

int ilu_contraction(ilu_handle_t h, double* x, int32_t nsteps, double* rho_out, double* rho_res_out,
                    void* hip_stream) {
    if (!h || !x || nsteps < 1 || !rho_out) return ILU_EINVAL;
    hipStream_t st = (hipStream_t)hip_stream;
    const Ctx c = h->ctx();
    const bool f32 = h->variant == ILU_SURR_F32;
    double* nr = h->norms.as<double>();
    double* part = h->partial.as<double>();
    double* xs = h->xs.as<double>();
    launch_permute(c, 1, 1, x, xs, h->S, 1, -1, st);
    HIPCHK(hipMemsetAsync(h->bs.p, 0, h->bs.bytes, st));  // b = 0: a step maps e to (I - C^{-1} A) e
    launch_sumsq(c, xs, part, st);
    launch_reduce(part, h->npartial, nr, 3, st);
    int err = 0;
    const double n0 = host_norm(h, 3, st, &err);
    if (err) return ILU_EHIP;
    if (!(n0 > 0.0) || !std::isfinite(n0)) return ILU_EINVAL;
    launch_scale_rsqrt(c, xs, nr, 3, st);
    double rho = 0.0, logsum = 0.0, ra0 = 0.0;
    int k = 0;
    for (; k < nsteps; ++k) {
        // ||A y||^2 of the normalised iterate comes with the step's residual
        launch_residual(c, xs, h->bs.as<double>(), h->r.p, f32, 1, part, st);
        launch_reduce(part, h->npartial, nr, 4, st);
        sweep_fwd(h, c, st);
        sweep_bwd(h, c, st);
        launch_sumsq(c, xs, part, st);
        launch_reduce(part, h->npartial, nr, 3, st);
        launch_scale_rsqrt(c, xs, nr, 3, st);
        double v[2];
        HIPCHK(hipMemcpyAsync(v, nr + 3, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (k == 0) ra0 = std::sqrt(v[1]);
        rho = std::sqrt(v[0]);
        if (!(rho > 0.0)) break;  // the step removed the error completely
        logsum += std::log(rho);
    }
    double rho_res = 0.0;
    if (rho > 0.0 && ra0 > 0.0) {
        // ||A x_K|| / ||A x_0|| = (||A y_K|| / ||A y_0||) prod rho_k
        launch_residual(c, xs, h->bs.as<double>(), h->r.p, f32, 1, part, st);
        launch_reduce(part, h->npartial, nr, 4, st);
        const double raK = std::sqrt(host_norm(h, 4, st, &err));
        if (err) return ILU_EHIP;
        rho_res = raK > 0.0 ? std::exp((std::log(raK / ra0) + logsum) / nsteps) : 0.0;
    }
    *rho_out = rho;
    if (rho_res_out) *rho_res_out = rho_res;
    launch_permute(c, 0, 1, xs, x, h->S, 1, -1, st);
    HIPCHK(hipGetLastError());
    int32_t fl[4];
    if (int e = read_flags(h, st, fl)) return e;
    if (h->schedule != ILU_SCHED_PLANE && fl[2]) return ILU_EHIP;
    return ILU_OK;
}

int ilu_lfa_orientation(const ilu_tet_desc* tets, int32_t ntets, int32_t samples, double* mu_out,
                        int32_t* best_out, void* hip_stream) {
    if (int e = lfa_check_args(tets, ntets, samples, mu_out, best_out)) return e;
    hipStream_t st = (hipStream_t)hip_stream;
    std::vector<double> v((size_t)ntets * 12);
    for (int i = 0; i < ntets; ++i)
        for (int a = 0; a < 4; ++a)
            for (int r = 0; r < 3; ++r) v[(size_t)i * 12 + 3 * a + r] = tets[i].vertex[a][r];
    DevBuf dv, drec, dmu;
    const size_t np = (size_t)ntets * LFA_PERMS;
    if (dv.alloc(v.size() * sizeof(double), st, false) || drec.alloc(np * LFA_REC * sizeof(double), st, false) ||
        dmu.alloc(np * sizeof(double), st, false))
        return ILU_ENOMEM;
    HIPCHK(hipMemcpyAsync(dv.p, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice, st));
    launch_lfa_stencils(dv.as<double>(), 12, ntets, drec.as<double>(), st);
    launch_lfa_symbols(drec.as<double>(), ntets, samples, dmu.as<double>(), st);
    HIPCHK(hipGetLastError());
    std::vector<double> mu(np);
    HIPCHK(hipMemcpyAsync(mu.data(), dmu.p, np * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int i = 0; i < ntets; ++i) {
        int best = 0;
        for (int k = 1; k < LFA_PERMS; ++k)
            if (mu[(size_t)i * LFA_PERMS + k] < mu[(size_t)i * LFA_PERMS + best]) best = k;
        if (best_out) best_out[i] = best;
    }
    if (mu_out) std::memcpy(mu_out, mu.data(), np * sizeof(double));
    return ILU_OK;
}

int ilu_lfa_orientation_noalloc(const ilu_tet_desc* tets, int32_t ntets, int32_t samples, double* mu_out,
                                int32_t* best_out, void* hip_stream) {
    if (int e = lfa_check_args(tets, ntets, samples, mu_out, best_out)) return e;
    if (ntets > ILU_LFA_NOALLOC_MAX_TETS) return ILU_EINVAL;
    hipStream_t st = (hipStream_t)hip_stream;
    void* base = nullptr;
    if (int e = scratch_address(&base)) return e;
    unsigned char* scr = static_cast<unsigned char*>(base);
    double* desc = reinterpret_cast<double*>(scr + LFA_SCR_DESC);
    double* rec = reinterpret_cast<double*>(scr + LFA_SCR_REC);
    double* mu = reinterpret_cast<double*>(scr + LFA_SCR_MU);
    int32_t* best = reinterpret_cast<int32_t*>(scr + LFA_SCR_BEST);
    HIPCHK(hipMemcpyAsync(desc, tets, sizeof(ilu_tet_desc) * (size_t)ntets, hipMemcpyHostToDevice, st));
    launch_lfa_stencils(desc, (int64_t)(sizeof(ilu_tet_desc) / sizeof(double)), ntets, rec, st);
    launch_lfa_symbols(rec, ntets, samples, mu, st);
    launch_lfa_best(mu, ntets, best, st);
    HIPCHK(hipGetLastError());
    if (mu_out)
        HIPCHK(hipMemcpyAsync(mu_out, mu, sizeof(double) * LFA_PERMS * (size_t)ntets, hipMemcpyDeviceToHost, st));
    if (best_out)
        HIPCHK(hipMemcpyAsync(best_out, best, sizeof(int32_t) * (size_t)ntets, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return ILU_OK;
}

int ilu_get_stencil(ilu_handle_t h, int32_t tet, double* A_out, void* hip_stream) {
    if (!h || !A_out || tet < 0 || tet >= h->ntets) return ILU_EINVAL;
    hipStream_t st = (hipStream_t)hip_stream;
    DevBuf full, a8;
    if (full.alloc((size_t)15 * h->S * sizeof(double), st) || a8.alloc((size_t)8 * h->S * sizeof(double), st))
        return ILU_ENOMEM;
    const Ctx c = h->ctx();
    launch_assemble(c, a8.as<double>(), full.as<double>(), st);
    launch_permute(c, 0, 15, full.as<double>(), A_out, h->S, 15, tet, st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    return ILU_OK;
}

int ilu_get_factors(ilu_handle_t h, int32_t tet, double* L_out, double* D_out, void* hip_stream) {
    if (!h || tet < 0 || tet >= h->ntets || h->variant != ILU_STORED_F64) return ILU_EINVAL;
    hipStream_t st = (hipStream_t)hip_stream;
    const Ctx c = h->ctx();
    if (L_out) launch_permute(c, 0, 7, h->Lf.as<double>(), L_out, h->S, 7, tet, st);
    if (D_out) launch_permute(c, 0, 1, h->Df.as<double>(), D_out, h->S, 1, tet, st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    return ILU_OK;
}

int ilu_get_surrogate(ilu_handle_t h, int32_t tet, double* coeffs_out) {
    if (!h || !coeffs_out || tet < 0 || tet >= h->ntets || h->variant == ILU_STORED_F64) return ILU_EINVAL;
    std::memcpy(coeffs_out, h->coef_h.data() + (size_t)tet * NFIT * h->K, (size_t)NFIT * h->K * sizeof(double));
    return ILU_OK;
}

int ilu_set_surrogate(ilu_handle_t h, int32_t tet, const double* coeffs, void* hip_stream) {
    if (!h || !coeffs || tet < 0 || tet >= h->ntets || h->variant == ILU_STORED_F64) return ILU_EINVAL;
    hipStream_t st = (hipStream_t)hip_stream;
    std::memcpy(h->coef_h.data() + (size_t)tet * NFIT * h->K, coeffs, (size_t)NFIT * h->K * sizeof(double));
    HIPCHK(hipMemcpyAsync(h->coef_d.p, h->coef_h.data(), h->coef_h.size() * sizeof(double), hipMemcpyHostToDevice,
                          st));
    if (int e = drop_graphs(h, st)) return e;  // captured launches hold the old table pointers
    if (int e = build_tables(h, st)) return e;
    if (h->boundary == ILU_BOUNDARY_V1)
        if (int e = build_v1b(h, st)) return e;
    HIPCHK(hipStreamSynchronize(st));
    return ILU_OK;
}

int ilu_get_surrogate_a(ilu_handle_t h, int32_t tet, double* coeffs_out) {
    if (!h || !coeffs_out || tet < 0 || tet >= h->ntets || h->a_mode != ILU_A_SURROGATE) return ILU_EINVAL;
    std::memcpy(coeffs_out, h->coefA_h.data() + (size_t)tet * NFIT * h->K, (size_t)NFIT * h->K * sizeof(double));
    return ILU_OK;
}

int ilu_set_surrogate_a(ilu_handle_t h, int32_t tet, const double* coeffs, void* hip_stream) {
    if (!h || !coeffs || tet < 0 || tet >= h->ntets || h->a_mode != ILU_A_SURROGATE) return ILU_EINVAL;
    hipStream_t st = (hipStream_t)hip_stream;
    std::memcpy(h->coefA_h.data() + (size_t)tet * NFIT * h->K, coeffs, (size_t)NFIT * h->K * sizeof(double));
    HIPCHK(hipMemcpyAsync(h->coefA_d.p, h->coefA_h.data(), h->coefA_h.size() * sizeof(double),
                          hipMemcpyHostToDevice, st));
    if (int e = drop_graphs(h, st)) return e;
    if (int e = build_tables_from(h, st, h->coefA_d, h->tabA64, h->tabA32)) return e;
    HIPCHK(hipStreamSynchronize(st));
    return ILU_OK;
}

int ilu_get_surrogate_values(ilu_handle_t h, int32_t tet, double* L_out, double* Dinv_out, void* hip_stream) {
    if (!h || tet < 0 || tet >= h->ntets || h->variant == ILU_STORED_F64) return ILU_EINVAL;
    hipStream_t st = (hipStream_t)hip_stream;
    launch_export_surrogate(h->ctx(), h->variant == ILU_SURR_F32, tet, L_out, Dinv_out, st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    return ILU_OK;
}

int ilu_last_sweeps(ilu_handle_t h, int32_t* sweeps_out) {
    if (!h || !sweeps_out) return ILU_EINVAL;
    *sweeps_out = h->last_sweeps;
    return ILU_OK;
}

int ilu_tile(ilu_handle_t h, int32_t* bv_out, int32_t* bw_out) {
    if (!h || !bv_out || !bw_out) return ILU_EINVAL;
    *bv_out = h->bv;
    *bw_out = h->bw;
    return ILU_OK;
}

int ilu_sample_stride(ilu_handle_t h, int32_t tet, int32_t* stride_out) {
    if (!h || !stride_out || tet < 0 || tet >= h->ntets) return ILU_EINVAL;
    *stride_out = h->tets[tet].stride;
    return ILU_OK;
}

int ilu_last_timing(ilu_handle_t h, double* sweep_ms, double* fwd_kernel_ms, double* bwd_kernel_ms,
                    double* res_kernel_ms) {
    if (!h || !h->have_timing) return ILU_EINVAL;
    float a = 0;
    HIPCHK(hipEventSynchronize(h->ev[1]));
    HIPCHK(hipEventElapsedTime(&a, h->ev[0], h->ev[1]));
    double f = 0, b = 0, r = 0;
    const int ns = h->kev_sweeps;
    for (int k = 0; k < ns; ++k) {
        hipEvent_t* e = h->kernel_timing ? &h->kev[6 * (size_t)k] : &h->ev[2];
        float tr = 0, tf = 0, tb = 0;
        HIPCHK(hipEventElapsedTime(&tr, e[0], e[1]));
        HIPCHK(hipEventElapsedTime(&tf, e[2], e[3]));
        HIPCHK(hipEventElapsedTime(&tb, e[4], e[5]));
        r += tr;
        f += tf;
        b += tb;
    }
    if (sweep_ms) *sweep_ms = a;
    if (fwd_kernel_ms) *fwd_kernel_ms = ns ? f / ns : 0.0;
    if (bwd_kernel_ms) *bwd_kernel_ms = ns ? b / ns : 0.0;
    if (res_kernel_ms) *res_kernel_ms = ns ? r / ns : 0.0;
    return ILU_OK;
}

int ilu_set_overlap(ilu_handle_t h, int32_t mode) {
    if (!h || mode < ILU_OVERLAP_OFF || mode > ILU_OVERLAP_FUSED) return ILU_EINVAL;
    if (mode != ILU_OVERLAP_OFF && !h->ovl_ok) return ILU_EINVAL;
    if (h->ovl != mode)
        if (int e = drop_graphs(h, nullptr)) return e;  // the captured sweep has the other form
    h->ovl = mode;
    return ILU_OK;
}

int ilu_get_overlap(ilu_handle_t h, int32_t* mode) {
    if (!h || !mode) return ILU_EINVAL;
    *mode = h->ovl;
    return ILU_OK;
}

int ilu_set_kernel_timing(ilu_handle_t h, int32_t enable) {
    if (!h) return ILU_EINVAL;
    h->kernel_timing = enable != 0;
    return ILU_OK;
}

int ilu_set_graph(ilu_handle_t h, int32_t enable) {
    if (!h) return ILU_EINVAL;
    h->use_graph = enable != 0;
    return ILU_OK;
}

int ilu_get_flow_grid(ilu_handle_t h, int32_t* grid_out, int32_t* grid_max_out) {
    if (!h || !grid_out) return ILU_EINVAL;
    *grid_out = h->flow_grid;
    if (grid_max_out) *grid_max_out = h->flow_grid_max;
    return ILU_OK;
}

int ilu_set_residual_chunk(ilu_handle_t h, int32_t hyperplanes) {
    if (!h || (hyperplanes != RES_T && hyperplanes != 2 * RES_T)) return ILU_EINVAL;
    if (h->res_lds_t != hyperplanes)
        if (int e = drop_graphs(h, nullptr)) return e;  // the captured residual launches have the old grid
    h->res_lds_t = hyperplanes;
    return ILU_OK;
}

int ilu_get_residual_chunk(ilu_handle_t h, int32_t* hyperplanes) {
    if (!h || !hyperplanes) return ILU_EINVAL;
    *hyperplanes = h->res_lds_t;
    return ILU_OK;
}

int ilu_set_flow_grid(ilu_handle_t h, int32_t grid, int32_t* grid_out) {
    if (!h || grid < 0) return ILU_EINVAL;
    const int g = grid == 0 ? h->flow_grid_max : std::min<int>(grid, h->flow_grid_max);
    if (g != h->flow_grid)
        if (int e = drop_graphs(h, nullptr)) return e;  // the captured launches carry the old grid
    h->flow_grid = g;
    if (grid_out) *grid_out = g;
    return ILU_OK;
}

}  // extern "C"
