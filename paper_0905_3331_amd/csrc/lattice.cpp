// lattice.cpp -- lattice object: creation, gauge ingest, operator application.
#include "lattice.h"

#include "engine.h"

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

namespace tmq {

static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }
const char *get_error() { return g_err.c_str(); }

size_t field_bytes(int prec, long n)
{
    size_t b = (size_t)n * field_blocks(prec) * 16;
    if (prec == P16 || prec == PB16) b += (size_t)n * sizeof(float);
    return b;
}

int field_alloc(Field &f, int prec, long n, int nrhs)
{
    field_free(f);
    if (n % 8 || nrhs < 1) {
        set_error("internal: field sizes must be multiples of 8 sites");
        return TMQ_EINVAL;
    }
    const size_t per = (size_t)n * field_blocks(prec) * 16;
    if (hipMalloc(&f.mem, per * nrhs) != hipSuccess) {
        f.mem = nullptr;
        set_error("device allocation of a spinor field failed");
        return TMQ_ENOMEM;
    }
    if (prec == P16 || prec == PB16) {
        if (hipMalloc((void **)&f.scale, (size_t)n * nrhs * sizeof(float)) != hipSuccess) {
            hipFree(f.mem);
            f.mem = nullptr;
            f.scale = nullptr;
            set_error("device allocation of a spinor scale array failed");
            return TMQ_ENOMEM;
        }
    }
    f.d.prec = prec;
    f.d.data = f.mem;
    f.d.scale = f.scale;
    f.d.n = n;
    f.d.nrhs = nrhs;
    f.d.rhs_elems = n * field_blocks(prec);
    f.d.rhs_sites = n;
    return TMQ_OK;
}

FieldDesc field_at(void *mem, int prec, long n, size_t *bytes)
{
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t data = up((size_t)n * field_blocks(prec) * 16);
    const bool coded = prec == P16 || prec == PB16;
    FieldDesc d;
    d.prec = prec;
    d.data = mem;
    d.scale = coded ? (float *)((char *)mem + data) : nullptr;
    d.n = n;
    d.nrhs = 1;
    d.rhs_elems = n * field_blocks(prec);
    d.rhs_sites = n;
    if (bytes) *bytes = data + (coded ? up((size_t)n * sizeof(float)) : 0);
    return d;
}

void field_free(Field &f)
{
    if (f.mem) hipFree(f.mem);
    if (f.scale) hipFree(f.scale);
    f.mem = nullptr;
    f.scale = nullptr;
    f.d = FieldDesc{};
}

Lattice::~Lattice()
{
    int cur = 0;
    hipGetDevice(&cur);
    hipSetDevice(device);
    if (own) hipStreamSynchronize(own);
    for (Engine *e : engines) delete e;
    for (auto &w : work) field_free(w.second);
    for (void *p : {(void *)u64f, (void *)u64r, (void *)u32r, (void *)u16a, (void *)u16b, (void *)u32f})
        if (p) hipFree(p);
    for (double *p : partial)
        if (p) hipFree(p);
    if (scal) hipFree(scal);
    if (ring) hipHostFree(ring);
    if (bicg) hipFree(bicg);
    if (bicg_ring) hipHostFree(bicg_ring);
    for (auto &e : bicg_ev)
        if (e) hipEventDestroy(e);
    for (auto &e : ring_ev)
        if (e) hipEventDestroy(e);
    for (void *s : stage)
        if (s) hipFree(s);
    for (auto &t : timed) {
        hipEventDestroy(t.a);
        hipEventDestroy(t.b);
    }
    for (auto e : event_pool) hipEventDestroy(e);
    if (own) hipStreamDestroy(own);
    hipSetDevice(cur);
}

int lattice_create(const int dims[4], int device, Lattice **out)
{
    if (!dims || !out) {
        set_error("tmq_lattice_create: NULL argument");
        return TMQ_EINVAL;
    }
    for (int i = 0; i < 4; i++)
        if (dims[i] < 2 || dims[i] % 2) {
            set_error("tmq_lattice_create: every extent must be even and >= 2 (periodic checkerboard)");
            return TMQ_EINVAL;
        }
    const double V = (double)dims[0] * dims[1] * dims[2] * dims[3];
    if (V / 2 * 24 >= 2147483647.0) {
        set_error("tmq_lattice_create: lattice too large for 32-bit site indexing");
        return TMQ_EINVAL;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        set_error("tmq_lattice_create: no such HIP device");
        return TMQ_EDEVICE;
    }
    Lattice *L = new Lattice();
    L->device = device;
    for (int k = 0; k < Lattice::NKEY; k++) {
        L->hop_variant[k] = -1;
        L->hop_occ[k] = 0;
        for (int v = 0; v < HOP_VARIANTS; v++) L->hop_tune_us[k][v] = -1.f;
        for (int c = 0; c < 6; c++) L->hop_occ_us[k][c] = -1.f;
    }
    if (const char *fv = getenv("TMQ_HOP_VARIANT")) {
        const int v = atoi(fv);
        if (v >= 0 && v < HOP_VARIANTS) L->forced_variant = v;
    }
    if (const char *fr = getenv("TMQ_HOP_RPL")) {
        const int r = atoi(fr);
        if (r == 1 || r == 2) L->forced_rpl = r;
    }
    if (const char *fc = getenv("TMQ_HOP_CAP")) {
        const int c = atoi(fc);
        if (c >= 0 && c <= 5) L->forced_cap = c;
    }
    memcpy(L->dims, dims, sizeof(L->dims));
    L->g.T = dims[0];
    L->g.LZ = dims[1];
    L->g.LY = dims[2];
    L->g.LX = dims[3];
    L->g.XH = dims[3] / 2;
    L->g.vh = (long)(V / 2);

    int cur = 0;
    hipGetDevice(&cur);
    auto fail = [&](int code, const char *what) {
        set_error(what);
        delete L;
        hipSetDevice(cur);
        return code;
    };
    if (hipSetDevice(device) != hipSuccess) return fail(TMQ_EDEVICE, "hipSetDevice failed");
    // the device's copy of the allocation-free work space (a failure is
    // reported by the allocation-free call only)
    (void)noalloc_scratch_init(device);
    if (hipStreamCreateWithFlags(&L->own, hipStreamNonBlocking) != hipSuccess)
        return fail(TMQ_EDEVICE, "hipStreamCreate failed");
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, device) == hipSuccess &&
        lds > 0)
        L->lds_per_cu = lds;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess && lds > 0)
        L->lds_per_block = lds;
    // per RHS: at least as many partials as any hop variant or vector kernel writes
    L->pstride = hop_grid(2 * L->g.vh) + 64;
    for (auto &p : L->partial)
        if (hipMalloc((void **)&p, sizeof(double) * L->pstride * MAX_RHS) != hipSuccess)
            return fail(TMQ_ENOMEM, "partials");
    if (hipMalloc((void **)&L->scal, sizeof(CgScalars) * MAX_RHS) != hipSuccess) return fail(TMQ_ENOMEM, "scalars");
    if (hipMemset(L->scal, 0, sizeof(CgScalars) * MAX_RHS) != hipSuccess) return fail(TMQ_EDEVICE, "memset");
    if (hipHostMalloc((void **)&L->ring, sizeof(CgScalars) * MAX_RHS * Lattice::RING, hipHostMallocMapped) !=
        hipSuccess)
        return fail(TMQ_ENOMEM, "pinned ring");
    if (hipHostGetDevicePointer((void **)&L->ring_dev, L->ring, 0) != hipSuccess)
        return fail(TMQ_EDEVICE, "device view of the pinned ring");
    for (auto &e : L->ring_ev)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return fail(TMQ_EDEVICE, "event");
    hipSetDevice(cur);
    *out = L;
    return TMQ_OK;
}

int stage_buffer(Lattice *L, int slot, size_t bytes, void **out)
{
    if (L->stage_bytes[slot] < bytes) {
        if (L->stage[slot]) hipFree(L->stage[slot]);
        L->stage[slot] = nullptr;
        L->stage_bytes[slot] = 0;
        if (hipMalloc(&L->stage[slot], bytes) != hipSuccess) {
            L->stage[slot] = nullptr;
            set_error("device allocation of a staging buffer failed");
            return TMQ_ENOMEM;
        }
        L->stage_bytes[slot] = bytes;
    }
    *out = L->stage[slot];
    return TMQ_OK;
}

int work_field(Lattice *L, const char *role, int prec, long n, FieldDesc *out, int nrhs)
{
    for (auto &w : L->work)
        if (w.first == role) {
            if (w.second.d.prec == prec && w.second.d.n == n && w.second.d.nrhs >= nrhs) {
                *out = w.second.d;
                out->nrhs = nrhs;
                return TMQ_OK;
            }
            TMQ_TRY(field_alloc(w.second, prec, n, nrhs));
            *out = w.second.d;
            return TMQ_OK;
        }
    L->work.emplace_back(role, Field{});
    TMQ_TRY(field_alloc(L->work.back().second, prec, n, nrhs));
    *out = L->work.back().second.d;
    return TMQ_OK;
}

// ------------------------------------------------------------------ gauge

int lattice_load_gauge(Lattice *L, const double2 *U, hipStream_t st)
{
    const long vh = L->g.vh;
    auto alloc = [&](void **p, size_t bytes) -> int {
        if (*p) return TMQ_OK;
        if (hipMalloc(p, bytes) != hipSuccess) {
            *p = nullptr;
            set_error("device allocation of gauge copies failed");
            return TMQ_ENOMEM;
        }
        return TMQ_OK;
    };
    TMQ_TRY(alloc((void **)&L->u64f, (size_t)8 * 9 * vh * sizeof(double2)));
    TMQ_TRY(alloc((void **)&L->u64r, (size_t)8 * 6 * vh * sizeof(double2)));
    TMQ_TRY(alloc((void **)&L->u32r, (size_t)8 * 3 * vh * sizeof(float4)));
    TMQ_TRY(alloc((void **)&L->u16a, (size_t)8 * vh * sizeof(uint4)));
    TMQ_TRY(alloc((void **)&L->u16b, (size_t)8 * ((vh + 15) & ~15L) * sizeof(uint2)));  // 16-site chunks
    GaugeOut o{L->u64f, L->u64r, L->u32r, L->u16a, L->u16b, nullptr};
    L->gauge = false;
    TMQ_HIP(launch_gauge_ingest(L->g, U, o, L->partial[0], st));
    TMQ_HIP(launch_max(L->partial[0], blas_grid(2 * vh), L->partial[1], st));
    double dev = 0.0;
    TMQ_HIP(hipMemcpyAsync(&dev, L->partial[1], sizeof(double), hipMemcpyDeviceToHost, st));
    TMQ_HIP(hipStreamSynchronize(st));
    L->su3_dev = dev;
    L->su3 = std::isfinite(dev) && dev < 1e-12;
    if (!L->su3) {
        // two-row copies cannot represent these links (row 2 is rebuilt as
        // conj(row0 x row1)): the reduced-precision operators use a full FP32 copy
        TMQ_TRY(alloc((void **)&L->u32f, (size_t)8 * 9 * vh * sizeof(float2)));
        GaugeOut f{nullptr, nullptr, nullptr, nullptr, nullptr, L->u32f};
        TMQ_HIP(launch_gauge_ingest(L->g, U, f, L->partial[0], st));
        TMQ_HIP(hipStreamSynchronize(st));
    }
    L->gauge = true;
    return TMQ_OK;
}

LinkDesc lattice_links(const Lattice *L, int fmt)
{
    LinkDesc d;
    d.fmt = fmt;
    d.vh = L->g.vh;
    switch (fmt) {
    case LK64F: d.a = L->u64f; break;
    case LK64R: d.a = L->u64r; break;
    case LK32R: d.a = L->u32r; break;
    case LK16R: d.a = L->u16a; d.b = L->u16b; break;
    case LK32F: d.a = L->u32f; break;
    }
    return d;
}

int link_fmt_for(const Lattice *L, int prec, int sloppy_link)
{
    if (prec == P64) return L->su3 ? LK64R : LK64F;
    if (!L->su3) return LK32F;  // any U: rows 0-2 stored, whatever the link precision asked for
    if (prec == P32 && sloppy_link != P16) return LK32R;
    if (sloppy_link == P32) return LK32R;
    return LK16R;
}

// ------------------------------------------------------------ operators

OpParams make_op(const Lattice *L, const tmq_params *p, int n)
{
    OpParams op{};
    const int Lmu[4] = {L->g.T, L->g.LX, L->g.LY, L->g.LZ};
    for (int mu = 0; mu < 4; mu++) {
        const double a = M_PI * p[0].theta[mu] / Lmu[mu];
        op.ph[mu][0] = p[0].theta[mu] == 0.0 ? 1.0 : cos(a);
        op.ph[mu][1] = p[0].theta[mu] == 0.0 ? 0.0 : sin(a);
    }
    for (int r = 0; r < n && r < MAX_RHS; r++) {
        op.kappa[r] = p[r].kappa;
        op.mut[r] = p[r].mu_tilde;
    }
    return op;
}

double hop_bytes_per_site(int prec, int link_fmt, bool self, int nrhs)
{
    const double sp = prec == P64 ? 192.0 : prec == P32 ? 96.0 : 52.0;
    const double lk = link_fmt == LK64F   ? 144.0
                      : link_fmt == LK64R ? 96.0
                      : link_fmt == LK32F ? 72.0
                      : link_fmt == LK32R ? 48.0
                                          : 24.0;
    return 8.0 * lk + nrhs * (sp + sp + (self ? sp : 0.0));
}

static hipEvent_t pool_event(Lattice *L)
{
    if (!L->event_pool.empty()) {
        hipEvent_t e = L->event_pool.back();
        L->event_pool.pop_back();
        return e;
    }
    // timing only: no system-scope fence when the event completes (the
    // default one writes back and invalidates the caches, which lengthens
    // the measured interval and makes the next kernel start cold)
    hipEvent_t e = nullptr;
    hipEventCreateWithFlags(&e, hipEventDisableSystemFence);
    return e;
}

// LDS bytes per block that let at most c blocks share a CU (0: no cap);
// ~0u when that needs more than a block may reserve
static unsigned occ_lds(const Lattice *L, int c)
{
    if (c <= 0) return 0;
    const unsigned b = (unsigned)(L->lds_per_cu / (c + 1)) + 256u;
    return b > (unsigned)L->lds_per_block ? ~0u : b;
}

// Time every valid variant of this hop launch (same operands, the reduction
// redirected to a scratch array, no skip flags) and keep the fastest for this
// lattice, spinor precision and link format.
static int tune_hop(Lattice *L, int key, int out_par, const FieldDesc &in, const FieldDesc &self,
                    const FieldDesc &out, const LinkDesc &lk, const OpParams &op, int epi, int sign,
                    const RhsList &rl, bool norm, hipStream_t st)
{
    hipEvent_t e0 = pool_event(L), e1 = pool_event(L);
    double *tp = norm ? L->partial[2] : nullptr;
    const int reps = L->g.vh * rl.n >= (1L << 18) ? 3 : 10;
    int best = 0;
    float best_us = 0.f;
    auto time_one = [&](int v, unsigned lds, float *us) -> int {
        HopTune tu;
        tu.variant = v;
        tu.lds = lds;
        TMQ_HIP(launch_hop(L->g, out_par, in, self, out, lk, op, epi, sign, rl, tp, L->pstride, nullptr, tu, st));
        TMQ_HIP(hipEventRecord(e0, st));
        for (int r = 0; r < reps; r++)
            TMQ_HIP(launch_hop(L->g, out_par, in, self, out, lk, op, epi, sign, rl, tp, L->pstride, nullptr, tu, st));
        TMQ_HIP(hipEventRecord(e1, st));
        TMQ_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        TMQ_HIP(hipEventElapsedTime(&ms, e0, e1));
        *us = ms * 1e3f / reps;
        return TMQ_OK;
    };
    const int nv = hop_all_variants(in.prec, lk.fmt) ? HOP_VARIANTS : 1;
    for (int v = 0; v < nv; v++) {
        if (!hop_variant_valid(L->g, v)) continue;
        float us = 0.f;
        TMQ_TRY(time_one(v, 0, &us));
        L->hop_tune_us[key][v] = us;
        if (best_us == 0.f || us < best_us) {
            best = v;
            best_us = us;
        }
    }
    // then a cap on the blocks per CU for the chosen variant (fewer sites in
    // flight per XCD: a smaller working set in its L2)
    int occ = 0;
    L->hop_occ_us[key][0] = best_us;
    for (int c = 1; c <= 5; c++) {
        const unsigned lds = occ_lds(L, c);
        if (lds == ~0u) continue;
        float us = 0.f;
        TMQ_TRY(time_one(best, lds, &us));
        L->hop_occ_us[key][c] = us;
        if (us < best_us) {
            occ = c;
            best_us = us;
        }
    }
    L->event_pool.push_back(e0);
    L->event_pool.push_back(e1);
    L->hop_variant[key] = best;
    L->hop_occ[key] = occ;
    return TMQ_OK;
}

// formats with kernels that take 2 or 4 RHS per lane (see hop_f32/f16/b16.hip)
static bool multi_rhs_format(int prec, int link_fmt)
{
    return (prec == P32 && link_fmt == LK32R) || ((prec == P16 || prec == PB16) && link_fmt == LK16R);
}

// For a batched launch, time the RHS per lane (1, or 2 where the format has
// them) and RHS groups (the variant and cap of the single-field tuning), then
// caps on the resident blocks per CU for the fastest of those, and keep the
// fastest for this format and batch size class.  None changes any result.
static int tune_batch(Lattice *L, int key, int cls, int out_par, const FieldDesc &in, const FieldDesc &self,
                      const FieldDesc &out, const LinkDesc &lk, const OpParams &op, int epi, int sign,
                      const RhsList &rl, bool norm, hipStream_t st, HopTune *res)
{
    hipEvent_t e0 = pool_event(L), e1 = pool_event(L);
    double *tp = norm ? L->partial[2] : nullptr;
    Lattice::BatchTune bt;
    bt.key = key;
    bt.cls = cls;
    HopTune base;
    base.variant = L->hop_variant[key];
    base.lds = occ_lds(L, L->hop_occ[key]);
    bt.cap = L->hop_occ[key];
    float best_us = 0.f;
    auto time_one = [&](const HopTune &tu, float *us) -> int {
        TMQ_HIP(launch_hop(L->g, out_par, in, self, out, lk, op, epi, sign, rl, tp, L->pstride, nullptr, tu, st));
        TMQ_HIP(hipEventRecord(e0, st));
        for (int r = 0; r < 2; r++)
            TMQ_HIP(launch_hop(L->g, out_par, in, self, out, lk, op, epi, sign, rl, tp, L->pstride, nullptr, tu, st));
        TMQ_HIP(hipEventRecord(e1, st));
        TMQ_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        TMQ_HIP(hipEventElapsedTime(&ms, e0, e1));
        *us = ms * 1e3f / 2;
        return TMQ_OK;
    };
    const int max_rpl = multi_rhs_format(in.prec, lk.fmt) ? 2 : 1;
    for (int rpl = 1; rpl <= max_rpl && rpl <= rl.n; rpl *= 2)
        for (int G = rpl;; G *= 2) {
            if (G > rl.n) G = rl.n;
            HopTune tu = base;
            tu.rpl = rpl;
            tu.group = G;
            float us = 0.f;
            TMQ_TRY(time_one(tu, &us));
            bt.tried.push_back({(float)rpl, (float)G, us});
            if (best_us == 0.f || us < best_us) {
                bt.tu = tu;
                best_us = us;
            }
            if (G == rl.n) break;
        }
    // fewer resident blocks shrink the set of (site, RHS) pairs in flight per
    // XCD, whose neighbour spinors compete for its L2
    bt.cap_us[bt.cap] = best_us;
    if (L->forced_cap < 0) {
        const HopTune shape = bt.tu;
        for (int c = 0; c <= 5; c++) {
            if (c == bt.cap) continue;
            HopTune tu = shape;
            tu.lds = occ_lds(L, c);
            if (tu.lds == ~0u) continue;
            float us = 0.f;
            TMQ_TRY(time_one(tu, &us));
            bt.cap_us[c] = us;
            if (us < best_us) {
                bt.tu = tu;
                bt.cap = c;
                best_us = us;
            }
        }
    }
    L->event_pool.push_back(e0);
    L->event_pool.push_back(e1);
    *res = bt.tu;
    L->hop_batch.push_back(bt);
    return TMQ_OK;
}

std::string tuning_report(const Lattice *L)
{
    static const char *pn[4] = {"fp64", "fp32", "fp16", "bf16"};
    static const char *ln[N_LINK_FMT] = {"fp64_full", "fp64_two_row", "fp32_two_row", "fp16_two_row",
                                         "fp32_full",  "?",            "?",            "?"};
    std::string s = "{\"hop\": [";
    bool first = true;
    for (int k = 0; k < Lattice::NKEY; k++) {
        if (L->hop_variant[k] < 0) continue;
        char buf[256];
        snprintf(buf, sizeof(buf), "%s{\"spinor\": \"%s\", \"links\": \"%s\", \"variant\": %d, \"us\": [",
                 first ? "" : ", ", pn[k / N_LINK_FMT], ln[k % N_LINK_FMT], L->hop_variant[k]);
        s += buf;
        for (int v = 0; v < HOP_VARIANTS; v++) {
            snprintf(buf, sizeof(buf), "%s%.2f", v ? ", " : "", L->hop_tune_us[k][v]);
            s += buf;
        }
        snprintf(buf, sizeof(buf), "], \"blocks_per_cu_cap\": %d, \"cap_us\": [", L->hop_occ[k]);
        s += buf;
        for (int c = 0; c < 6; c++) {
            snprintf(buf, sizeof(buf), "%s%.2f", c ? ", " : "", L->hop_occ_us[k][c]);
            s += buf;
        }
        s += "]}";
        first = false;
    }
    s += "], \"batch\": [";
    for (size_t i = 0; i < L->hop_batch.size(); i++) {
        const Lattice::BatchTune &b = L->hop_batch[i];
        char buf[256];
        snprintf(buf, sizeof(buf),
                 "%s{\"spinor\": \"%s\", \"links\": \"%s\", \"nrhs_class\": %d, \"rhs_per_lane\": %d, "
                 "\"group\": %d, \"blocks_per_cu_cap\": %d, \"cap_us\": [",
                 i ? ", " : "", pn[b.key / N_LINK_FMT], ln[b.key % N_LINK_FMT], b.cls, b.tu.rpl, b.tu.group, b.cap);
        s += buf;
        for (int c = 0; c < 6; c++) {
            snprintf(buf, sizeof(buf), "%s%.1f", c ? ", " : "", b.cap_us[c]);
            s += buf;
        }
        s += "], \"tried\": [";
        for (size_t j = 0; j < b.tried.size(); j++) {
            snprintf(buf, sizeof(buf), "%s[%d, %d, %.1f]", j ? ", " : "", (int)b.tried[j][0], (int)b.tried[j][1],
                     b.tried[j][2]);
            s += buf;
        }
        s += "]}";
    }
    s += "]}";
    return s;
}

// A doublet field (2 V/2 sites, upper flavour first) seen as a batch of two
// single-flavour fields per doublet: doublet d becomes the pair 2d, 2d + 1.
static FieldDesc flavour_view(const FieldDesc &f)
{
    FieldDesc o = f;
    if (!f.data) return o;
    o.n = f.n / 2;
    o.nrhs = 2 * f.nrhs;
    o.rhs_elems = f.rhs_elems / 2;
    o.rhs_sites = f.rhs_sites / 2;
    return o;
}

static double fused_extra_bytes(int prec, int epi)
{
    // the epilogue's own vectors beside the half-sweep's (whose output write
    // stands for the write of r): CG reads r and p and reads and writes x;
    // the residual reads b
    const double sp = prec == P64 ? 192.0 : prec == P32 ? 96.0 : 52.0;
    const double xsp = prec == P64 ? 192.0 : 96.0;
    return epi == EPI_K2_CG ? (2 * sp + 2 * xsp) : epi == EPI_K2_RES ? sp : 0.0;
}

// hop half-sweep of a batch of doublets (op.nd): the two flavours of a site
// in a lane pair, the block order of the format's single-field tuning
static int hop_nd(Lattice *L, int out_par, const FieldDesc &in, const FieldDesc &self, const FieldDesc &out,
                  const LinkDesc &lk, const OpParams &op, int epi, int sign, const RhsList &rl, double *partial,
                  const CgScalars *scal, hipStream_t st, const CgFields *cg)
{
    const long n2 = 2 * L->g.vh;
    const bool fused = epi == EPI_K2_CG || epi == EPI_K2_RES;
    if (2 * rl.n > MAX_RHS || in.n != n2 || (!fused && out.n != n2) || (self.data && self.n != n2) ||
        (in.rhs_elems != n2 * field_blocks(in.prec))) {
        set_error("internal: doublet fields must hold 2 V/2 sites per doublet, at most 32 doublets");
        return TMQ_EINVAL;
    }
    const FieldDesc fi = flavour_view(in), fs = flavour_view(self), fo = flavour_view(out);
    CgFields c2;
    if (cg) {
        c2.r = flavour_view(cg->r);
        c2.p = flavour_view(cg->p);
        c2.x = flavour_view(cg->x);
    }
    RhsList fl;
    fl.n = 2 * rl.n;
    for (int i = 0; i < rl.n; i++) {
        fl.idx[2 * i] = (unsigned char)(2 * rl.idx[i]);
        fl.idx[2 * i + 1] = (unsigned char)(2 * rl.idx[i] + 1);
    }
    const int key = in.prec * N_LINK_FMT + lk.fmt;
    if (L->forced_variant >= 0) {
        L->hop_variant[key] = hop_variant_valid(L->g, L->forced_variant) ? L->forced_variant : 0;
    } else if (L->hop_variant[key] < 0) {
        if (fused) {
            set_error("internal: fused hop epilogue before the format was tuned");
            return TMQ_ESTATE;
        }
        // tune the format on single-field launches of the first upper flavour
        OpParams o1 = op;
        o1.nd = 0;
        RhsList one;
        one.n = 1;
        one.idx[0] = fl.idx[0];
        TMQ_TRY(tune_hop(L, key, out_par, fi, fs, fo, lk, o1, epi, sign, one, false, st));
    }
    if (L->forced_cap >= 0) L->hop_occ[key] = occ_lds(L, L->forced_cap) == ~0u ? 0 : L->forced_cap;
    HopTune tu;
    tu.variant = L->hop_variant[key];
    tu.lds = occ_lds(L, L->hop_occ[key]);
    TimedLaunch t{};
    if (L->timing) {
        t.a = pool_event(L);
        t.b = pool_event(L);
        t.bytes = (hop_bytes_per_site(in.prec, lk.fmt, epi != EPI_K1, fl.n) + fused_extra_bytes(in.prec, epi) * fl.n) *
                  (double)L->g.vh;
        t.flops = 1320.0 * (double)L->g.vh * fl.n;
        t.prec = in.prec;
        t.nrhs = fl.n;
        t.epi = epi;
        TMQ_HIP(hipEventRecord(t.a, st));
    }
    TMQ_HIP(launch_hop(L->g, out_par, fi, fs, fo, lk, op, epi, sign, fl, partial, L->pstride, scal, tu, st,
                       cg ? &c2 : nullptr));
    // partial sums of the launch: its blocks per field, from the variant it ran
    L->hop_blocks_last = hop_grid_variant(L->g, hop_all_variants(in.prec, lk.fmt) ? L->hop_variant[key] : 0,
                                          hop_nd_lanes(L->g, in.prec, lk.fmt, op));
    if (L->timing) {
        TMQ_HIP(hipEventRecord(t.b, st));
        L->timed.push_back(t);
    }
    return TMQ_OK;
}

int hop(Lattice *L, int out_par, const FieldDesc &in, const FieldDesc &self, const FieldDesc &out,
        const LinkDesc &lk, const OpParams &op, int epi, int sign, const RhsList &rl, double *partial,
        const CgScalars *scal, hipStream_t st, const CgFields *cg)
{
    if (rl.n <= 0) return TMQ_OK;
    if (op.nd) return hop_nd(L, out_par, in, self, out, lk, op, epi, sign, rl, partial, scal, st, cg);
    const int key = in.prec * N_LINK_FMT + lk.fmt;
    const bool fused = epi == EPI_K2_CG || epi == EPI_K2_RES;
    if (fused && L->forced_variant < 0 && L->hop_variant[key] < 0) {
        // the tuner re-runs its launch, which a fused epilogue must not (it
        // updates vectors in place); the plain half-sweeps before it tune the format
        set_error("internal: fused hop epilogue before the format was tuned");
        return TMQ_ESTATE;
    }
    if (L->no_alloc) {
        // an allocation-free call: the tuned shape if there is one, else variant 0
        if (rl.n != 1) {
            set_error("internal: allocation-free hop launches take one right-hand side");
            return TMQ_EINVAL;
        }
        HopTune tu;
        const bool tuned = L->forced_variant < 0 && L->hop_variant[key] >= 0;
        tu.variant = tuned ? L->hop_variant[key] : 0;
        tu.lds = tuned ? occ_lds(L, L->hop_occ[key]) : 0;
        TMQ_HIP(launch_hop(L->g, out_par, in, self, out, lk, op, epi, sign, rl, partial, L->pstride, scal, tu, st,
                           cg));
        L->hop_blocks_last = hop_grid_variant(L->g, hop_all_variants(in.prec, lk.fmt) ? tu.variant : 0);
        return TMQ_OK;
    }
    if (L->forced_variant >= 0)
        L->hop_variant[key] = hop_variant_valid(L->g, L->forced_variant) ? L->forced_variant : 0;
    else if (L->hop_variant[key] < 0)
        TMQ_TRY(tune_hop(L, key, out_par, in, self, out, lk, op, epi, sign, rl, partial != nullptr, st));
    if (L->forced_cap >= 0) L->hop_occ[key] = occ_lds(L, L->forced_cap) == ~0u ? 0 : L->forced_cap;
    // batches use the launch shape tuned for their power-of-two size class
    HopTune tu;
    tu.variant = L->hop_variant[key];
    tu.lds = occ_lds(L, L->hop_occ[key]);
    if (rl.n > 1) {
        int cls = 2;
        while (cls < rl.n) cls *= 2;
        bool found = false;
        for (auto &e : L->hop_batch)
            if (e.key == key && e.cls == cls) {
                tu = e.tu;
                found = true;
            }
        if (!found && fused) {
            set_error("internal: fused hop epilogue before the batch shape was tuned");
            return TMQ_ESTATE;
        }
        if (!found)
            TMQ_TRY(tune_batch(L, key, cls, out_par, in, self, out, lk, op, epi, sign, rl, partial != nullptr, st,
                               &tu));
        if (L->forced_rpl) tu.rpl = L->forced_rpl;
        if (L->forced_cap >= 0) tu.lds = occ_lds(L, L->forced_cap) == ~0u ? 0 : occ_lds(L, L->forced_cap);
        // TMQ_HOP_GROUP (diagnostics): right-hand sides per L2 group of batched launches
        if (const char *fg = getenv("TMQ_HOP_GROUP")) {
            const int gsz = atoi(fg);
            if (gsz >= 1 && gsz <= MAX_RHS) tu.group = gsz;
        }
    }
    TimedLaunch t{};
    if (L->timing) {
        t.a = pool_event(L);
        t.b = pool_event(L);
        t.bytes = (hop_bytes_per_site(in.prec, lk.fmt, epi != EPI_K1, rl.n) + fused_extra_bytes(in.prec, epi) * rl.n) *
                  (double)L->g.vh;
        t.flops = 1320.0 * (double)L->g.vh * rl.n;
        t.prec = in.prec;
        t.nrhs = rl.n;
        t.epi = epi;
        TMQ_HIP(hipEventRecord(t.a, st));
    }
    TMQ_HIP(launch_hop(L->g, out_par, in, self, out, lk, op, epi, sign, rl, partial, L->pstride, scal, tu, st, cg));
    // partial sums of the launch: its blocks per field, from the variant it ran
    L->hop_blocks_last = hop_grid_variant(L->g, hop_all_variants(in.prec, lk.fmt) ? L->hop_variant[key] : 0);
    if (L->timing) {
        TMQ_HIP(hipEventRecord(t.b, st));
        L->timed.push_back(t);
    }
    return TMQ_OK;
}

int apply_Qhat(Lattice *L, const OpParams &op, int sign, const FieldDesc &in, const FieldDesc &out,
               const FieldDesc &tmp_e, const LinkDesc &lk, const RhsList &rl, double *partial,
               const CgScalars *scal, hipStream_t st)
{
    const FieldDesc none{};
    TMQ_TRY(hop(L, 0, in, none, tmp_e, lk, op, EPI_K1, sign, rl, nullptr, scal, st));
    TMQ_TRY(hop(L, 1, tmp_e, in, out, lk, op, EPI_K2, sign, rl, partial, scal, st));
    return TMQ_OK;
}

int apply_Qhat_cg(Lattice *L, const OpParams &op, const FieldDesc &in, const FieldDesc &tmp_e, const LinkDesc &lk,
                  const RhsList &rl, const CgFields &cg, double *partial, const CgScalars *scal, hipStream_t st)
{
    const FieldDesc none{};
    TMQ_TRY(hop(L, 0, in, none, tmp_e, lk, op, EPI_K1, +1, rl, nullptr, scal, st));
    TMQ_TRY(hop(L, 1, tmp_e, in, none, lk, op, EPI_K2_CG, +1, rl, partial, scal, st, &cg));
    return TMQ_OK;
}

int residual_QhatQhat(Lattice *L, const OpParams &op, const FieldDesc &x, const FieldDesc &b, const FieldDesc &r,
                      const FieldDesc &tmp_e, const FieldDesc &tmp_o, const LinkDesc &lk, const RhsList &rl,
                      double *partial, hipStream_t st)
{
    const FieldDesc none{};
    CgFields cg;
    cg.r = r;
    cg.p = b;
    TMQ_TRY(apply_Qhat(L, op, -1, x, tmp_o, tmp_e, lk, rl, nullptr, nullptr, st));
    TMQ_TRY(hop(L, 0, tmp_o, none, tmp_e, lk, op, EPI_K1, +1, rl, nullptr, nullptr, st));
    TMQ_TRY(hop(L, 1, tmp_e, tmp_o, none, lk, op, EPI_K2_RES, +1, rl, partial, nullptr, st, &cg));
    return TMQ_OK;
}

int apply_QhatQhat(Lattice *L, const OpParams &op, const FieldDesc &in, const FieldDesc &out,
                   const FieldDesc &tmp_e, const FieldDesc &tmp_o, const LinkDesc &lk, const RhsList &rl,
                   double *partial, const CgScalars *scal, hipStream_t st)
{
    TMQ_TRY(apply_Qhat(L, op, -1, in, tmp_o, tmp_e, lk, rl, partial, scal, st));
    TMQ_TRY(apply_Qhat(L, op, +1, tmp_o, out, tmp_e, lk, rl, nullptr, scal, st));
    return TMQ_OK;
}

int apply_Q_full(Lattice *L, const OpParams &op, int sign, const FieldDesc &in, const FieldDesc &out,
                 const LinkDesc &lk, const RhsList &rl, hipStream_t st)
{
    const long vh = L->g.vh;
    const FieldDesc ie = field_sub(in, 0, vh), io = field_sub(in, vh, vh);
    const FieldDesc oe = field_sub(out, 0, vh), oo = field_sub(out, vh, vh);
    TMQ_TRY(hop(L, 0, io, ie, oe, lk, op, EPI_FULL, sign, rl, nullptr, nullptr, st));
    TMQ_TRY(hop(L, 1, ie, io, oo, lk, op, EPI_FULL, sign, rl, nullptr, nullptr, st));
    return TMQ_OK;
}

int check_prec(int prec)
{
    if (prec < TMQ_FP64 || prec > TMQ_BF16) {
        set_error("invalid tmq_prec");
        return TMQ_EINVAL;
    }
    return TMQ_OK;
}

int check_opts(const tmq_solver_opts *o)
{
    if (!o) {
        set_error("NULL tmq_solver_opts");
        return TMQ_EINVAL;
    }
    if (!(o->tol > 0.0) || !std::isfinite(o->tol)) {
        set_error("tol must be a positive finite number");
        return TMQ_EINVAL;
    }
    TMQ_TRY(check_prec(o->sloppy));
    if (o->sloppy != TMQ_FP64 && o->sloppy_link != TMQ_FP32 && o->sloppy_link != TMQ_FP16) {
        set_error("sloppy_link must be TMQ_FP32 or TMQ_FP16");
        return TMQ_EINVAL;
    }
    if (o->mode != TMQ_MODE_RELIABLE && o->mode != TMQ_MODE_SWITCH && o->mode != TMQ_MODE_BICGSTAB) {
        set_error("mode must be TMQ_MODE_RELIABLE, TMQ_MODE_SWITCH or TMQ_MODE_BICGSTAB");
        return TMQ_EINVAL;
    }
    if (o->mode == TMQ_MODE_BICGSTAB && o->sloppy != TMQ_FP64) {
        set_error("TMQ_MODE_BICGSTAB runs in FP64 only (sloppy = TMQ_FP64)");
        return TMQ_EINVAL;
    }
    return TMQ_OK;
}

int check_params(const tmq_params *p)
{
    if (!p) {
        set_error("NULL tmq_params");
        return TMQ_EINVAL;
    }
    if (!std::isfinite(p->kappa) || !std::isfinite(p->mu_tilde)) {
        set_error("kappa and mu_tilde must be finite");
        return TMQ_EINVAL;
    }
    for (double t : p->theta)
        if (!std::isfinite(t)) {
            set_error("theta must be finite");
            return TMQ_EINVAL;
        }
    return TMQ_OK;
}

}  // namespace tmq
