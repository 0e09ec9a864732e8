// C ABI of liblbm: argument checking, workspace carving, launches and graph
// replay around the kernels of lbm_kernels.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "lbm_internal.h"

namespace lbm {
hipError_t launch_step(int lattice, int fp64, int scheme, int parity, void *a, void *b, const Box &box, const Model &m,
                       double tau, double rho_ref, int block, const uint32_t *lm, const double *F, hipStream_t s);
hipError_t launch_init(int lattice, int fp64, void *lat, const double *n0, const double *u0, const Box &box,
                       const Model &m, double tau, double rho_ref, int block, hipStream_t s);
hipError_t launch_moments(int lattice, int fp64, const void *lat, double *n, double *u, const Box &box, double rho_ref,
                          int odd, int block, const uint32_t *lm, const double *F, int row0, int nrows,
                          int64_t ostride, hipStream_t s);
hipError_t launch_totals(int lattice, int fp64, const void *lat, double *part, double *out, const Box &box,
                         double rho_ref, int odd, int block, const uint32_t *lm, hipStream_t s);
hipError_t launch_link_mask(int D, const unsigned char *solid, uint32_t *lm, const Box &box, int block,
                            hipStream_t s);
}  // namespace lbm

namespace lbm {
namespace {
thread_local std::string g_err;
}  // namespace
void set_last_error(const std::string &msg) { g_err = msg; }
}  // namespace lbm

using namespace lbm;

namespace {

lbm_status fail(lbm_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

lbm_status hip_fail(hipError_t e, const char *what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return LBM_ERR_HIP;
}

constexpr size_t kAlign = 256;
constexpr size_t kPlanePadBytes = 33 * 256;
constexpr size_t kStageBytes = size_t(4) << 20;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    int64_t cells = 0, plane = 0;  // plane: elements between population planes
    int rows = 0;
    size_t elt = 0, lattice_bytes = 0, part_off = 0, out_off = 0, mask_off = 0, stage_off = 0, total = 0;
    int stage_rows = 0;  // rows of moments staged per chunk of the host lbm_moments
    int nlat = 0;
    bool porous = false;  // obstacles or a body force: link mask in the workspace, porous kernels
};

lbm_status check_config(const lbm_config *cfg, Model *m, Layout *lay) {
    std::string err;
    lbm_status s = build_model(cfg, m, &err);
    if (s != LBM_OK) return fail(s, err);
    if (cfg->nx < 1 || cfg->ny < 1 || cfg->nz < 1) return fail(LBM_ERR_ARG, "box sizes must be >= 1");
    if (m->D < 2 && cfg->ny != 1) return fail(LBM_ERR_ARG, "d1v3 needs ny = 1");
    if (m->D < 3 && cfg->nz != 1) return fail(LBM_ERR_ARG, "2D lattices need nz = 1");
    if (cfg->lattice == LBM_D2V41) {
        if (cfg->nx < 4 || cfg->ny < 4) return fail(LBM_ERR_ARG, "d2v41 needs nx, ny >= 4 (links of four cells)");
        if (cfg->block > D2Q41::MAXB) return fail(LBM_ERR_ARG, "d2v41 kernels take at most 512 threads per workgroup");
        if (cfg->bc[0] != LBM_PERIODIC || cfg->bc[1] != LBM_PERIODIC)
            return fail(LBM_ERR_UNSUPPORTED, "d2v41 runs on periodic boxes only");
        if (cfg->obstacles || cfg->force[0] != 0.0 || cfg->force[1] != 0.0 || cfg->force[2] != 0.0)
            return fail(LBM_ERR_UNSUPPORTED, "d2v41 has no obstacles or body force (41 links exceed the link mask)");
    }
    for (int d = 0; d < 3; ++d)
        if (cfg->bc[d] != LBM_PERIODIC && cfg->bc[d] != LBM_BOUNCEBACK) return fail(LBM_ERR_ARG, "bad bc");
    if (cfg->precision != LBM_FP32_DEV && cfg->precision != LBM_FP64) return fail(LBM_ERR_ARG, "bad precision");
    if (cfg->scheme != LBM_SCHEME_PUSH && cfg->scheme != LBM_SCHEME_AA) return fail(LBM_ERR_ARG, "bad scheme");
    if (cfg->block != 0 && (cfg->block < 64 || cfg->block > 1024 || cfg->block % 64))
        return fail(LBM_ERR_ARG, "block must be 0 or a multiple of 64 in [64, 1024]");
    if (cfg->graph_steps < 0 || cfg->graph_steps % 2) return fail(LBM_ERR_ARG, "graph_steps must be even, >= 0");
    if (cfg->obstacles != 0 && cfg->obstacles != 1) return fail(LBM_ERR_ARG, "obstacles must be 0 or 1");
    for (int d = 0; d < 3; ++d)
        if (!std::isfinite(cfg->force[d])) return fail(LBM_ERR_ARG, "force must be finite");
    const int64_t rows = (int64_t)cfg->ny * cfg->nz;
    const int64_t cells = rows * cfg->nx;
    if (rows > 0x7fffffff) return fail(LBM_ERR_ARG, "too many rows for one launch");
    lay->cells = cells;
    lay->rows = (int)rows;
    lay->elt = cfg->precision == LBM_FP64 ? sizeof(double) : sizeof(float);
    lay->nlat = cfg->scheme == LBM_SCHEME_AA ? 1 : 2;
    // population planes cells + pad apart: 33 x 256 B, so that the planes of a
    // power-of-two box do not all start on the same HBM channel
    lay->plane = cells + (int64_t)(kPlanePadBytes / lay->elt);
    lay->lattice_bytes = align_up((size_t)m->Q * (size_t)lay->plane * lay->elt);
    lay->part_off = lay->lattice_bytes * lay->nlat;
    lay->out_off = lay->part_off + align_up((size_t)rows * 5 * sizeof(double));
    lay->mask_off = lay->out_off + align_up(5 * sizeof(double));
    lay->porous = cfg->obstacles || cfg->force[0] != 0.0 || cfg->force[1] != 0.0 || cfg->force[2] != 0.0;
    lay->stage_off = lay->mask_off + (lay->porous ? align_up((size_t)cells * sizeof(uint32_t)) : 0);
    // staging of the host lbm_moments: whole rows of n and u0 (float64), about
    // kStageBytes at a time (at least one row)
    const size_t row_bytes = (size_t)(m->D + 1) * sizeof(double) * (size_t)cfg->nx;
    int64_t srows = (int64_t)(kStageBytes / row_bytes);
    if (srows < 1) srows = 1;
    if (srows > rows) srows = rows;
    lay->stage_rows = (int)srows;
    lay->total = lay->stage_off + align_up((size_t)srows * row_bytes);
    return LBM_OK;
}

int default_block(int nx) {
    int b = 256;
    if (nx < b) b = (nx + 63) / 64 * 64;
    return b < 64 ? 64 : b;
}

}  // namespace

struct lbm_ctx_s {
    lbm_config cfg{};
    Model model{};
    Layout lay{};
    Box box{};
    char *ws = nullptr;
    void *lat[2] = {nullptr, nullptr};
    double *part = nullptr, *out = nullptr;
    uint32_t *lm = nullptr;  // link mask (porous runs only)
    double F[3] = {0.0, 0.0, 0.0};
    int cur = 0;          // push: index of the lattice holding the state
    int64_t steps = 0;    // steps done
    int block = 256;
    int fp64 = 0;
    double rho_ref = 1.0;
    hipStream_t stream = nullptr;
    hipStream_t cap = nullptr;  // private stream for graph capture
    hipGraphExec_t graph[2] = {nullptr, nullptr};  // by starting parity / lattice index
};

namespace {

int phase(const lbm_ctx_s *c) {
    // push: which lattice is current; AA: parity of the steps done
    return c->cfg.scheme == LBM_SCHEME_PUSH ? c->cur : (int)(c->steps & 1);
}

hipError_t one_step(lbm_ctx_s *c, hipStream_t s) {
    const int ph = phase(c);
    void *a = c->cfg.scheme == LBM_SCHEME_PUSH ? c->lat[ph] : c->lat[0];
    void *b = c->cfg.scheme == LBM_SCHEME_PUSH ? c->lat[1 - ph] : nullptr;
    hipError_t e = launch_step(c->model.lattice, c->fp64, c->cfg.scheme, ph, a, b, c->box, c->model, c->cfg.tau,
                               c->rho_ref, c->block, c->lm, c->F, s);
    if (e == hipSuccess) {
        if (c->cfg.scheme == LBM_SCHEME_PUSH) c->cur = 1 - c->cur;
        c->steps++;
    }
    return e;
}

lbm_status build_graph(lbm_ctx_s *c, int ph) {
    hipError_t e;
    if (!c->cap) {
        e = hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(e, "hipStreamCreateWithFlags");
    }
    const int save_cur = c->cur;
    const int64_t save_steps = c->steps;
    e = hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    hipError_t le = hipSuccess;
    for (int k = 0; k < c->cfg.graph_steps && le == hipSuccess; ++k) le = one_step(c, c->cap);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(c->cap, &g);
    c->cur = save_cur;
    c->steps = save_steps;
    if (le != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(le, "kernel launch during capture");
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&c->graph[ph], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    return LBM_OK;
}

}  // namespace

extern "C" {

const char *lbm_last_error(void) { return g_err.c_str(); }

lbm_status lbm_coefficients(const lbm_config *cfg, double *out, int cap, int *n_written) {
    if (!cfg || !out || !n_written) return fail(LBM_ERR_ARG, "null argument");
    Model m;
    std::string err;
    lbm_status s = build_model(cfg, &m, &err);
    if (s != LBM_OK) return fail(s, err);
    const bool o4 = cfg->lattice == LBM_D2V41;
    const int need = 6 * m.ncls + 4 + (o4 ? 3 * m.ncls + 1 : 0);
    if (cap < need) return fail(LBM_ERR_ARG, "output capacity too small");
    for (int k = 0; k < m.ncls; ++k) {
        const ClassCoef &cc = m.cls[k];
        const double v[6] = {cc.w, cc.l1, cc.q, cc.s, cc.c3, cc.k4};
        std::memcpy(out + 6 * k, v, sizeof v);
    }
    out[6 * m.ncls + 0] = m.J2;
    out[6 * m.ncls + 1] = m.J4;
    out[6 * m.ncls + 2] = m.d2sq;
    out[6 * m.ncls + 3] = m.d4sq;
    if (o4) {
        double *o = out + 6 * m.ncls + 4;
        for (int k = 0; k < m.ncls; ++k) {
            o[3 * k + 0] = m.cls[k].p4;
            o[3 * k + 1] = m.cls[k].r4;
            o[3 * k + 2] = m.cls[k].t4;
        }
        o[3 * m.ncls] = m.scale;
    }
    *n_written = need;
    return LBM_OK;
}

lbm_status lbm_workspace_bytes(const lbm_config *cfg, size_t *bytes) {
    if (!cfg || !bytes) return fail(LBM_ERR_ARG, "null argument");
    Model m;
    Layout lay;
    lbm_status s = check_config(cfg, &m, &lay);
    if (s != LBM_OK) return s;
    *bytes = lay.total;
    return LBM_OK;
}

lbm_status lbm_init(const lbm_config *cfg, void *workspace, size_t bytes, void *stream, const double *n0_dev,
                    const double *u0_dev, lbm_ctx *out) {
    if (!cfg || !workspace || !n0_dev || !u0_dev || !out) return fail(LBM_ERR_ARG, "null argument");
    *out = nullptr;
    Model m;
    Layout lay;
    lbm_status s = check_config(cfg, &m, &lay);
    if (s != LBM_OK) return s;
    if (bytes < lay.total) return fail(LBM_ERR_ARG, "workspace smaller than lbm_workspace_bytes()");
    if ((uintptr_t)workspace % kAlign) return fail(LBM_ERR_ARG, "workspace must be 256-byte aligned");
    lbm_ctx_s *c = new (std::nothrow) lbm_ctx_s;
    if (!c) return fail(LBM_ERR_ARG, "out of host memory");
    c->cfg = *cfg;
    c->model = m;
    c->lay = lay;
    c->box = Box{cfg->nx, cfg->ny, cfg->nz, cfg->bc[0] == LBM_BOUNCEBACK, cfg->bc[1] == LBM_BOUNCEBACK,
                 cfg->bc[2] == LBM_BOUNCEBACK, lay.plane, lay.cells};
    c->ws = (char *)workspace;
    c->lat[0] = c->ws;
    c->lat[1] = lay.nlat == 2 ? c->ws + lay.lattice_bytes : nullptr;
    c->part = (double *)(c->ws + lay.part_off);
    c->out = (double *)(c->ws + lay.out_off);
    c->block = cfg->block ? cfg->block : default_block(cfg->nx);
    c->fp64 = cfg->precision == LBM_FP64;
    c->rho_ref = cfg->rho_ref > 0 ? cfg->rho_ref : 1.0;
    c->stream = (hipStream_t)stream;
    if (lay.porous) {
        c->lm = (uint32_t *)(c->ws + lay.mask_off);
        for (int d = 0; d < 3; ++d) c->F[d] = cfg->force[d];
    }
    hipError_t e = hipSuccess;
    if (c->lm) e = hipMemsetAsync(c->lm, 0, (size_t)lay.cells * sizeof(uint32_t), c->stream);  // no solids yet
    if (e == hipSuccess)
        e = launch_init(m.lattice, c->fp64, c->lat[0], n0_dev, u0_dev, c->box, m, cfg->tau, c->rho_ref, c->block,
                        c->stream);
    if (e != hipSuccess) {
        delete c;
        return hip_fail(e, "init kernel launch");
    }
    *out = c;
    return LBM_OK;
}

lbm_status lbm_step(lbm_ctx c, int64_t nsteps) {
    if (!c) return fail(LBM_ERR_ARG, "null context");
    if (nsteps < 0) return fail(LBM_ERR_ARG, "nsteps < 0");
    const int G = c->cfg.graph_steps;
    int64_t left = nsteps;
    while (G > 0 && left >= G) {
        const int ph = phase(c);
        if (!c->graph[ph]) {
            lbm_status s = build_graph(c, ph);
            if (s != LBM_OK) return s;
        }
        hipError_t e = hipGraphLaunch(c->graph[ph], c->stream);
        if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
        c->steps += G;  // G even: the lattice index and the AA parity are unchanged
        left -= G;
    }
    for (; left > 0; --left) {
        hipError_t e = one_step(c, c->stream);
        if (e != hipSuccess) return hip_fail(e, "step kernel launch");
    }
    return LBM_OK;
}

lbm_status lbm_moments_device(lbm_ctx c, double *n_dev, double *u_dev) {
    if (!c || !n_dev || !u_dev) return fail(LBM_ERR_ARG, "null argument");
    const int odd = c->cfg.scheme == LBM_SCHEME_AA ? (int)(c->steps & 1) : 0;
    const void *lat = c->cfg.scheme == LBM_SCHEME_PUSH ? c->lat[c->cur] : c->lat[0];
    hipError_t e = launch_moments(c->model.lattice, c->fp64, lat, n_dev, u_dev, c->box, c->rho_ref, odd, c->block,
                                  c->lm, c->F, 0, c->lay.rows, c->lay.cells, c->stream);
    if (e != hipSuccess) return hip_fail(e, "moments kernel launch");
    return LBM_OK;
}

lbm_status lbm_moments(lbm_ctx c, double *n_host, double *u_host) {
    if (!c || !n_host || !u_host) return fail(LBM_ERR_ARG, "null argument");
    const int odd = c->cfg.scheme == LBM_SCHEME_AA ? (int)(c->steps & 1) : 0;
    const void *lat = c->cfg.scheme == LBM_SCHEME_PUSH ? c->lat[c->cur] : c->lat[0];
    const int D = c->model.D, nx = c->cfg.nx, rows = c->lay.rows, chunk = c->lay.stage_rows;
    const int64_t cells = c->lay.cells, cstride = (int64_t)chunk * nx;
    double *sn = (double *)(c->ws + c->lay.stage_off), *su = sn + cstride;
    // chunks of whole rows through the staging area, in stream order (a chunk's
    // kernel runs after the previous chunk's copy has drained the staging area)
    for (int r0 = 0; r0 < rows; r0 += chunk) {
        const int nr = rows - r0 < chunk ? rows - r0 : chunk;
        const int64_t off = (int64_t)r0 * nx, cnt = (int64_t)nr * nx;
        hipError_t e = launch_moments(c->model.lattice, c->fp64, lat, sn, su, c->box, c->rho_ref, odd, c->block, c->lm,
                                      c->F, r0, nr, cstride, c->stream);
        if (e != hipSuccess) return hip_fail(e, "moments kernel launch");
        e = hipMemcpyAsync(n_host + off, sn, cnt * sizeof(double), hipMemcpyDeviceToHost, c->stream);
        for (int d = 0; e == hipSuccess && d < D; ++d)
            e = hipMemcpyAsync(u_host + d * cells + off, su + d * cstride, cnt * sizeof(double),
                               hipMemcpyDeviceToHost, c->stream);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
    }
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return LBM_OK;
}

lbm_status lbm_totals(lbm_ctx c, double *out_host) {
    if (!c || !out_host) return fail(LBM_ERR_ARG, "null argument");
    const int odd = c->cfg.scheme == LBM_SCHEME_AA ? (int)(c->steps & 1) : 0;
    const void *lat = c->cfg.scheme == LBM_SCHEME_PUSH ? c->lat[c->cur] : c->lat[0];
    hipError_t e = launch_totals(c->model.lattice, c->fp64, lat, c->part, c->out, c->box, c->rho_ref, odd, c->block,
                                 c->lm, c->stream);
    if (e != hipSuccess) return hip_fail(e, "totals kernel launch");
    double tmp[5];
    e = hipMemcpyAsync(tmp, c->out, sizeof tmp, hipMemcpyDeviceToHost, c->stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    for (int d = 0; d <= c->model.D; ++d) out_host[d] = tmp[d];
    for (int d = 0; d <= c->model.D; ++d)
        if (!std::isfinite(tmp[d])) return fail(LBM_ERR_NUMERIC, "non-finite total");
    if (tmp[4] != 0.0) return fail(LBM_ERR_NUMERIC, "cells with non-positive or non-finite density");
    return LBM_OK;
}

lbm_status lbm_set_solid(lbm_ctx c, const unsigned char *solid_dev) {
    if (!c || !solid_dev) return fail(LBM_ERR_ARG, "null argument");
    if (!c->cfg.obstacles) return fail(LBM_ERR_STATE, "the context was created without obstacles");
    if (c->cfg.scheme == LBM_SCHEME_AA && (c->steps & 1))
        return fail(LBM_ERR_STATE, "solids can change only after an even number of AA steps");
    hipError_t e = launch_link_mask(c->model.D, solid_dev, c->lm, c->box, c->block, c->stream);
    if (e != hipSuccess) return hip_fail(e, "link mask kernel launch");
    return LBM_OK;
}

}  // extern "C"

namespace {

// Host-side permutation between the natural layout (g_a at its own cell) and
// the AA storage after an odd number of steps (g_a of cell x held in the slot
// of -a at x - e_a, or in slot a at x for a link that bounced at a wall or a
// solid cell; lm is the link mask of a run with solids, else null).
// `gather` maps storage -> natural; otherwise natural -> storage.
template <typename T>
void aa_odd_permute(const lbm_ctx_s *c, const T *in, T *out, bool gather, const uint32_t *lm) {
    const Box &b = c->box;
    const int64_t P = c->lay.cells;  // host copies hold the planes back to back
    const int Q = c->model.Q;
    const int(*e)[3] = D2Q9::e;
    const int *opp = D2Q9::opp;
    switch (c->model.lattice) {
    case LBM_D1V3: e = D1Q3::e; opp = D1Q3::opp; break;
    case LBM_D3V19: e = D3Q19::e; opp = D3Q19::opp; break;
    case LBM_D2V41: e = D2Q41::e; opp = D2Q41::opp; break;
    default: break;
    }
    const int dims[3] = {b.nx, b.ny, b.nz};
    const int bbs[3] = {b.bbx, b.bby, b.bbz};
    for (int z = 0; z < b.nz; ++z)
        for (int y = 0; y < b.ny; ++y)
            for (int x = 0; x < b.nx; ++x) {
                const int64_t cell = ((int64_t)z * b.ny + y) * b.nx + x;
                const int p[3] = {x, y, z};
                if (lm && (lm[cell] & kSolidBit)) {  // a solid cell owns only its own slots
                    if (gather)
                        for (int q = 0; q < Q; ++q) out[(int64_t)q * P + cell] = in[(int64_t)q * P + cell];
                    continue;
                }
                for (int q = 0; q < Q; ++q) {
                    int s[3];
                    bool bb = lm && opp[q] < 32 && ((lm[cell] >> opp[q]) & 1u);  // x - e_q is a solid cell
                    for (int d = 0; d < 3; ++d) {
                        s[d] = p[d] - e[q][d];
                        if (s[d] < 0 || s[d] >= dims[d]) {
                            if (bbs[d]) bb = true;
                            else s[d] = (s[d] + dims[d]) % dims[d];
                        }
                    }
                    const int64_t slot = bb ? (int64_t)q * P + cell
                                            : (int64_t)opp[q] * P + ((int64_t)s[2] * b.ny + s[1]) * b.nx + s[0];
                    const int64_t nat = (int64_t)q * P + cell;
                    if (gather) out[nat] = in[slot];
                    else out[slot] = in[nat];
                }
            }
}

}  // namespace

extern "C" {

lbm_status lbm_get_state(lbm_ctx c, void *host, size_t bytes) {
    if (!c || !host) return fail(LBM_ERR_ARG, "null argument");
    const size_t need = (size_t)c->model.Q * c->lay.cells * c->lay.elt;
    if (bytes != need) return fail(LBM_ERR_ARG, "state size mismatch");
    const void *lat = c->cfg.scheme == LBM_SCHEME_PUSH ? c->lat[c->cur] : c->lat[0];
    const bool odd = c->cfg.scheme == LBM_SCHEME_AA && (c->steps & 1);
    std::vector<char> raw;
    void *dst = host;
    if (odd) {
        raw.resize(need);
        dst = raw.data();
    }
    std::vector<uint32_t> lm;
    const size_t row = (size_t)c->lay.cells * c->lay.elt, pitch = (size_t)c->lay.plane * c->lay.elt;
    hipError_t e = hipMemcpy2DAsync(dst, row, lat, pitch, row, c->model.Q, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && odd && c->lm) {
        lm.resize(c->lay.cells);
        e = hipMemcpyAsync(lm.data(), c->lm, lm.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "state copy");
    if (odd) {
        const uint32_t *m = lm.empty() ? nullptr : lm.data();
        if (c->fp64) aa_odd_permute<double>(c, (const double *)raw.data(), (double *)host, true, m);
        else aa_odd_permute<float>(c, (const float *)raw.data(), (float *)host, true, m);
    }
    return LBM_OK;
}

lbm_status lbm_set_state(lbm_ctx c, const void *host, size_t bytes) {
    if (!c || !host) return fail(LBM_ERR_ARG, "null argument");
    const size_t need = (size_t)c->model.Q * c->lay.cells * c->lay.elt;
    if (bytes != need) return fail(LBM_ERR_ARG, "state size mismatch");
    void *lat = c->cfg.scheme == LBM_SCHEME_PUSH ? c->lat[c->cur] : c->lat[0];
    const bool odd = c->cfg.scheme == LBM_SCHEME_AA && (c->steps & 1);
    std::vector<char> raw;
    const void *src = host;
    hipError_t e = hipSuccess;
    const size_t row = (size_t)c->lay.cells * c->lay.elt, pitch = (size_t)c->lay.plane * c->lay.elt;
    if (odd) {
        // the slots of the odd AA layout depend on the solids: read the stored
        // state first so that slots no cell owns (inside solids) keep their values
        std::vector<uint32_t> lm;
        raw.resize(need);
        e = hipMemcpy2DAsync(raw.data(), row, lat, pitch, row, c->model.Q, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess && c->lm) {
            lm.resize(c->lay.cells);
            e = hipMemcpyAsync(lm.data(), c->lm, lm.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return hip_fail(e, "state copy");
        const uint32_t *m = lm.empty() ? nullptr : lm.data();
        if (c->fp64) aa_odd_permute<double>(c, (const double *)host, (double *)raw.data(), false, m);
        else aa_odd_permute<float>(c, (const float *)host, (float *)raw.data(), false, m);
        src = raw.data();
    }
    e = hipMemcpy2DAsync(lat, pitch, src, row, row, c->model.Q, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "state copy");
    return LBM_OK;
}

lbm_status lbm_steps_done(lbm_ctx c, int64_t *steps) {
    if (!c || !steps) return fail(LBM_ERR_ARG, "null argument");
    *steps = c->steps;
    return LBM_OK;
}

lbm_status lbm_info(lbm_ctx c, int64_t *cells, int *Q, int64_t *bytes_per_step) {
    if (!c || !cells || !Q || !bytes_per_step) return fail(LBM_ERR_ARG, "null argument");
    *cells = c->lay.cells;
    *Q = c->model.Q;
    *bytes_per_step = 2 * (int64_t)c->model.Q * c->lay.cells * (int64_t)c->lay.elt;
    return LBM_OK;
}

lbm_status lbm_velocities(int lattice, int *e_out, int cap, int *Q) {
    if (!e_out || !Q) return fail(LBM_ERR_ARG, "null argument");
    const int(*e)[3] = nullptr;
    int q = 0;
    if (lattice == LBM_D1V3) { e = D1Q3::e; q = D1Q3::Q; }
    else if (lattice == LBM_D2V9) { e = D2Q9::e; q = D2Q9::Q; }
    else if (lattice == LBM_D3V19) { e = D3Q19::e; q = D3Q19::Q; }
    else if (lattice == LBM_D2V41) { e = D2Q41::e; q = D2Q41::Q; }
    else return fail(LBM_ERR_ARG, "unknown lattice");
    if (cap < 3 * q) return fail(LBM_ERR_ARG, "output capacity too small");
    for (int a = 0; a < q; ++a)
        for (int d = 0; d < 3; ++d) e_out[3 * a + d] = e[a][d];
    *Q = q;
    return LBM_OK;
}

lbm_status lbm_free(lbm_ctx c) {
    if (!c) return LBM_OK;
    lbm_status st = LBM_OK;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) st = hip_fail(e, "hipStreamSynchronize");
    for (auto &g : c->graph)
        if (g) (void)hipGraphExecDestroy(g);
    if (c->cap) (void)hipStreamDestroy(c->cap);
    delete c;
    return st;
}

}  // extern "C"
