// Host engine behind the C interface in include/pcfgsmc.h.
//
// The engine owns device memory (through the context's allocator), builds the
// (run, tile) tables the kernels are launched over, enforces the call order of
// Algorithm 1 (Sec. 3.2: propagation and resampling alternate) and turns the
// device control block into status codes. Every kernel of a round reads the
// round number and status from device memory, so the host never waits between
// rounds; it synchronises only to answer a query.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "pcfgsmc.h"

#include "engine.hpp"
#include "launch.hpp"
#include "program.hpp"

using namespace pcfg;

namespace {

thread_local std::string g_error;

smc_status fail(smc_status code, const std::string& msg)
{
    g_error = msg;
    return code;
}

#define HIP_TRY(expr)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(SMC_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));   \
    } while (0)

constexpr uint64_t kMaxParticles = 1ull << 24;

// Device memory of smc_resample_weights_noalloc: control block, propagation
// group slots and three per-tile partial arrays for up to kMaxParticles
// weights, carved from one static device array. Every GPU the library runs on
// holds its own copy (about 390 KB) until the process ends; host code reaches
// it only through the address hipGetSymbolAddress returns on that device.
constexpr size_t kNoallocCtlOff = 0;
constexpr size_t kNoallocGroupsOff = 256;
constexpr size_t kNoallocMaxTiles = (kMaxParticles + kTileRed - 1) / kTileRed;
constexpr size_t kNoallocPartOff = kNoallocGroupsOff + ((sizeof(GroupPartials) + 255) / 256) * 256;
constexpr size_t kNoallocPartBytes = kNoallocMaxTiles * sizeof(double);
constexpr size_t kNoallocBytes = kNoallocPartOff + 3 * kNoallocPartBytes;
static_assert(sizeof(RunCtl) <= kNoallocGroupsOff, "control block fits its slot");
static_assert(kNoallocPartBytes % 256 == 0, "partial arrays stay 256-byte aligned");

__device__ __align__(256) unsigned char scratch[kNoallocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Looks up this device's copy of the array once per device (the device must
// be current) and keeps its address.
smc_status scratch_address(int device, void** out)
{
    if (device < 0 || device >= kMaxDevices) return fail(SMC_ERR_INVALID, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(SMC_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return SMC_OK;
}

}  // namespace

struct smc_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    void* scratch = nullptr;  // this device's copy of the static scratch array
    smc_allocator alloc{};
    bool custom_alloc = false;

    void* allocate(size_t bytes)
    {
        if (bytes == 0) bytes = 8;
        if (custom_alloc) return alloc.alloc(alloc.ctx, bytes);
        void* p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
        return p;
    }
    void release(void* p)
    {
        if (!p) return;
        if (custom_alloc) alloc.free(alloc.ctx, p);
        else (void)hipFree(p);
    }
};

namespace {

// Device allocations owned by one object; released together.
struct DeviceArena {
    smc_ctx* ctx = nullptr;
    std::vector<void*> ptrs;
    void* get(size_t bytes)
    {
        void* p = ctx->allocate(bytes);
        if (p) ptrs.push_back(p);
        return p;
    }
    void release_all()
    {
        for (void* p : ptrs) ctx->release(p);
        ptrs.clear();
    }
};

int real_fields(int kind)
{
    switch (kind) {
    case SMC_MODEL_LGSSM: return 1;
    case SMC_MODEL_CRBD: return 2;
    case SMC_MODEL_CLADS: return 4;
    case SMC_MODEL_SEIR: return 6;
    case SMC_MODEL_CRBD_DS: return 4;
    default: return 0;
    }
}
int stored_int_fields(int kind)
{
    return (kind == SMC_MODEL_GEOMETRIC || kind == SMC_MODEL_PROGRAM) ? 1 : kind == SMC_MODEL_SEIR ? 9 : 0;
}
// Int fields as the model defines them (cursor-like ones follow the round and
// are not stored): geometric flips; LGSSM t; CRBD node; ClaDS node and stack
// size; SEIR nine counts and the day; delayed-sampling CRBD node; a compiled
// program's stack pointer.
int logical_int_fields(int kind) { return kind == SMC_MODEL_CLADS ? 2 : kind == SMC_MODEL_SEIR ? 10 : 1; }

// Static checks of a compiled program. Together with the kernel's run-time
// checks of sp, stored return blocks, return-value locations and data
// indices they keep every access of the interpreter inside its buffers:
// registers below kProgRegs; constants, arrays, distributions and blocks in
// range; frame offsets below the block's frame size; callee-frame stores only
// between CALLFRAME and its PUSH, with no jump into or out of that stretch
// (so the capacity check of CALLFRAME precedes them on every path); jumps
// forward inside the block; every block opened by FRAME and closed by a
// terminator.
smc_status check_program(const smc_program_desc* p)
{
    auto bad = [](const std::string& m) { return fail(SMC_ERR_INVALID, "program: " + m); };
    if (!p) return bad("description is NULL");
    if (p->n_blocks < 1 || p->n_blocks > kProgMaxBlocks) return bad("n_blocks must be in [1, 254]");
    if (!p->block_start || !p->code) return bad("block_start or code is NULL");
    if (p->n_code < 1 || p->n_code > kProgMaxCode) return bad("n_code must be in [1, 2^20]");
    if (p->stack_words < 1 || p->stack_words > kProgMaxStack) return bad("stack_words must be in [1, 4096]");
    if (p->n_consts > kProgMaxCode || (p->n_consts > 0 && !p->consts)) return bad("constants missing");
    if (p->n_data > (1u << 26) || (p->n_data > 0 && !p->data)) return bad("data missing");
    if (p->n_arrays > kProgMaxCode || (p->n_arrays > 0 && !p->array_start)) return bad("array_start missing");
    if (p->n_arrays > 0) {
        if (p->array_start[0] != 0 || p->array_start[p->n_arrays] != p->n_data)
            return bad("array_start must run from 0 to n_data");
        for (uint32_t a = 0; a < p->n_arrays; ++a)
            if (p->array_start[a + 1] < p->array_start[a]) return bad("array_start must not decrease");
    }
    if (p->block_start[0] != 0 || p->block_start[p->n_blocks] != p->n_code)
        return bad("block_start must run from 0 to n_code");
    std::vector<int> open_at;
    for (uint32_t b = 0; b < p->n_blocks; ++b) {
        const uint32_t start = p->block_start[b], end = p->block_start[b + 1];
        const std::string where = "block " + std::to_string(b);
        if (end <= start) return bad(where + " is empty");
        open_at.assign(end - start + 1, 0);
        uint32_t frame = 0;
        int64_t open = -1;  // words of the callee frame opened by CALLFRAME, -1 = none
        for (uint32_t pc = start; pc < end; ++pc) {
            const uint64_t w = p->code[pc];
            const uint32_t op = (uint32_t)(w & 255u), x = (uint32_t)(w >> 8) & 255u, y = (uint32_t)(w >> 16) & 255u,
                           z = (uint32_t)(w >> 24) & 255u, imm = (uint32_t)(w >> 32);
            const std::string at = where + " instruction " + std::to_string(pc) + ": ";
            open_at[pc - start] = open >= 0 ? 1 : 0;
            if (op < kOpFrame || op >= kOpCount) return bad(at + "unknown opcode");
            if (x >= (uint32_t)kProgRegs || y >= (uint32_t)kProgRegs || z >= (uint32_t)kProgRegs)
                return bad(at + "register out of range");
            if ((op == kOpFrame) != (pc == start)) return bad(at + "FRAME must open the block, and only there");
            switch (op) {
            case kOpFrame:
                if (imm > p->stack_words) return bad(at + "frame larger than the stack");
                frame = imm;
                break;
            case kOpConst:
                if (imm >= p->n_consts) return bad(at + "constant out of range");
                break;
            case kOpLdf:
            case kOpStf:
            case kOpAddr:
                if (imm >= frame) return bad(at + "frame offset out of range");
                break;
            case kOpData:
            case kOpLen:
                if (imm >= p->n_arrays) return bad(at + "data array out of range");
                break;
            case kOpSample:
                if (imm >= kDistCount) return bad(at + "unknown distribution");
                break;
            case kOpObserve:
                if (imm >= kDistCount || imm == kDistGamma || imm == kDistBeta)
                    return bad(at + "distribution cannot be observed");
                break;
            case kOpJz:
            case kOpJmp:
                if (!(imm > pc && imm < end)) return bad(at + "jump target must lie ahead in the same block");
                if (open >= 0) return bad(at + "jump inside an open callee frame");
                break;
            case kOpCallFrame:
                if (open >= 0) return bad(at + "callee frame already open");
                if (imm < 1 || imm > p->stack_words) return bad(at + "callee frame size out of range");
                open = imm;
                break;
            case kOpStn:
                if (open < 0 || imm >= (uint32_t)open) return bad(at + "STN outside the open callee frame");
                break;
            case kOpPush:
                if (open < 0 || imm != (uint32_t)open) return bad(at + "PUSH must close the open callee frame");
                open = -1;
                break;
            case kOpStret:
                if (frame < 2) return bad(at + "STRET needs a frame of at least 2 words");
                break;
            case kOpJret:
                if (frame < 2 || imm != frame) return bad(at + "JRET must pop the block's frame");
                break;
            case kOpGoto:
            case kOpCkpt:
                if (imm >= p->n_blocks) return bad(at + "block out of range");
                break;
            default: break;
            }
            const bool term = op == kOpGoto || op == kOpCkpt || op == kOpJret || op == kOpFault;
            if (term && open >= 0) return bad(at + "block transition with an open callee frame");
            if (pc + 1 == end && !term) return bad(where + " does not end with GOTO, CKPT, JRET or FAULT");
        }
        for (uint32_t pc = start; pc < end; ++pc) {
            const uint64_t w = p->code[pc];
            const uint32_t op = (uint32_t)(w & 255u), imm = (uint32_t)(w >> 32);
            if ((op == kOpJz || op == kOpJmp) && open_at[imm - start])
                return bad(where + " instruction " + std::to_string(pc) + ": jump into an open callee frame");
        }
    }
    return SMC_OK;
}

}  // namespace

struct smc_model {
    smc_ctx* ctx = nullptr;
    int kind = 0, precision = 64, checkpoint = 1, n_nodes = 0, T = 0;
    int stack_depth = 0;
    uint32_t ess_t = 0;              // ESS threshold numerator over 2^16 (0: resample every round)
    std::vector<int32_t> sp_before;  // ClaDS: stack size when node r is visited (index n_nodes = final)
    ModelDev host{};
    ModelDev* dev = nullptr;
    DeviceArena arena;
};

struct smc_run {
    smc_ctx* ctx = nullptr;
    smc_model* model = nullptr;
    uint64_t n = 0, seed = 0;
    RunDev host{};
    RunDev* dev = nullptr;
    uint32_t n_prop = 0, n_red = 0;
    bool expect_step = true;   // Alg. 1: step 2 and step 3 alternate
    bool owned = false;        // batched: one work-group advances it through a tick
    uint32_t rounds_issued = 0;
    int32_t known_status = SMC_OK;
    DeviceArena arena;
    // optional per-kernel timing: (kernel id, start event, end event)
    bool profiling = false;
    struct Timed {
        int kernel;
        hipEvent_t start, end;
    };
    std::vector<Timed> timed;
    std::vector<hipEvent_t> event_pool;
    size_t events_used = 0;
    // the whole lockstep run (rounds 0..R-1) captured once and replayed
    hipGraphExec_t graph = nullptr;
    uint32_t graph_rounds = 0;
    uint32_t* perm_buf = nullptr;  // block bucketing permutation (allocated on first use)
    uint32_t resets = 0;  // a reset run is replayed from a captured graph
    hipEvent_t next_event()
    {
        if (events_used == event_pool.size()) {
            hipEvent_t e = nullptr;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            event_pool.push_back(e);
        }
        return event_pool[events_used++];
    }
    ~smc_run()
    {
        for (hipEvent_t e : event_pool) (void)hipEventDestroy(e);
        if (graph) (void)hipGraphExecDestroy(graph);
    }
};

namespace {

smc_status read_ctl(smc_run* r, RunCtl* out)
{
    HIP_TRY(hipMemcpyAsync(out, r->host.ctl, sizeof(RunCtl), hipMemcpyDeviceToHost, r->ctx->stream));
    HIP_TRY(hipStreamSynchronize(r->ctx->stream));
    if (out->status != SMC_OK) r->known_status = out->status;
    return SMC_OK;
}

size_t real_bytes(const smc_model* m) { return m->precision == 32 ? 4 : 8; }

// Allocate and initialise a run's device state (Alg. 1 step 1).
void set_prop_tiles(RunDev& h, int lanes)
{
    h.lanes = (uint32_t)lanes;
    h.prop_tiles = (uint32_t)((h.n + lanes - 1) / lanes);
    h.fused = h.red_tiles <= kMaxFusedRedTiles ? 1u : 0u;
}

// The run's memory comes from ctx's allocator and its work goes to ctx's
// stream (a batch's runs use the batch's context, whatever context the model
// was registered on).
smc_status build_run(smc_model* m, uint64_t n, uint64_t seed, smc_run* r, smc_ctx* ctx)
{
    r->ctx = ctx;
    r->model = m;
    r->n = n;
    r->seed = seed;
    r->arena.ctx = ctx;
    RunDev& h = r->host;
    h.n = (uint32_t)n;
    h.red_tiles = (uint32_t)((n + kTileRed - 1) / kTileRed);
    h.model = m->dev;
    const size_t rb = real_bytes(m);
    auto get = [&](size_t bytes) { return r->arena.get(bytes); };
    h.ctl = (RunCtl*)get(sizeof(RunCtl));
    for (int b = 0; b < 2; ++b) {
        h.buf[b].blk = (uint8_t*)get(n);
        for (int f = 0; f < real_fields(m->kind); ++f) h.buf[b].real[f] = get(n * rb);
        for (int f = 0; f < stored_int_fields(m->kind); ++f) h.buf[b].ints[f] = (int32_t*)get(n * 4);
        if (m->kind == SMC_MODEL_CLADS || m->kind == SMC_MODEL_PROGRAM)
            h.buf[b].stack = get(n * rb * (size_t)m->stack_depth);
    }
    h.lw = (double*)get(n * 8);
    h.anc = (uint32_t*)get(n * 4);
    set_prop_tiles(h, prop_threads(m->kind));
    if (m->kind == SMC_MODEL_CLADS) h.side_stack = get((size_t)kMaxDepthCap * n * 17);
    h.groups = (GroupPartials*)get(sizeof(GroupPartials));
    h.part_q = (double*)get(h.red_tiles * 8);
    h.part_e = (double*)get(h.red_tiles * 8);
    h.prefix = (double*)get(h.red_tiles * 8);
    h.ess_t = m->ess_t;
    if (h.ess_t) h.part_q2 = (unsigned long long*)get(h.red_tiles * 16);
    r->dev = (RunDev*)get(sizeof(RunDev));
    r->n_prop = h.prop_tiles;
    r->n_red = h.red_tiles;
    bool ok = h.ctl && h.lw && h.anc && h.part_q && h.groups &&
              (h.side_stack || m->kind != SMC_MODEL_CLADS) && h.part_e && h.prefix && r->dev &&
              (h.part_q2 || !h.ess_t);
    for (int b = 0; b < 2; ++b) {
        ok = ok && h.buf[b].blk;
        for (int f = 0; f < real_fields(m->kind); ++f) ok = ok && h.buf[b].real[f];
        for (int f = 0; f < stored_int_fields(m->kind); ++f) ok = ok && h.buf[b].ints[f];
        if (m->kind == SMC_MODEL_CLADS || m->kind == SMC_MODEL_PROGRAM) ok = ok && h.buf[b].stack;
    }
    if (!ok) {
        r->arena.release_all();
        return fail(SMC_ERR_OOM, "device allocation failed for a run of " + std::to_string(n) + " particles");
    }
    hipStream_t st = ctx->stream;
    HIP_TRY(hipMemcpyAsync(r->dev, &r->host, sizeof(RunDev), hipMemcpyHostToDevice, st));
    HIP_TRY(launch_reset(r->dev, seed, st));  // control block: round 0, log Z 0, the seed
    return SMC_OK;
}

smc_status do_step(smc_run* r)
{
    if (!r->expect_step) return fail(SMC_ERR_STATE, "smc_step called twice without smc_resample");
    if (r->known_status != SMC_OK) return r->known_status;
    hipStream_t st = r->ctx->stream;
    const int kind = r->model->kind, prec = r->model->precision;
    if (r->host.perm) {
        if (r->profiling) {
            hipEvent_t a = r->next_event(), b = r->next_event();
            if (!a || !b) return fail(SMC_ERR_DEVICE, "event creation failed");
            HIP_TRY(hipEventRecord(a, st));
            HIP_TRY(launch_bucket(r->host, st));
            HIP_TRY(hipEventRecord(b, st));
            r->timed.push_back(smc_run::Timed{1, a, b});
        } else {
            HIP_TRY(launch_bucket(r->host, st));
        }
    }
    if (r->profiling) {
        hipEvent_t a = r->next_event(), b = r->next_event();
        if (!a || !b) return fail(SMC_ERR_DEVICE, "event creation failed");
        HIP_TRY(hipEventRecord(a, st));
        HIP_TRY(launch_propagate_one(kind, prec, r->host, st));
        HIP_TRY(hipEventRecord(b, st));
        r->timed.push_back(smc_run::Timed{0, a, b});
    } else {
        HIP_TRY(launch_propagate_one(kind, prec, r->host, st));
    }
    r->expect_step = false;
    return SMC_OK;
}

smc_status do_resample(smc_run* r)
{
    if (r->expect_step) return fail(SMC_ERR_STATE, "smc_resample called before smc_step");
    if (r->known_status != SMC_OK) return r->known_status;
    hipStream_t st = r->ctx->stream;
    if (r->profiling) {
        hipEvent_t a = r->next_event(), b = r->next_event(), c = r->next_event();
        if (!a || !b || !c) return fail(SMC_ERR_DEVICE, "event creation failed");
        HIP_TRY(hipEventRecord(a, st));
        HIP_TRY(launch_resample_one(r->host, r->dev, st, 1));
        HIP_TRY(hipEventRecord(b, st));
        HIP_TRY(launch_resample_one(r->host, r->dev, st, 2));
        HIP_TRY(hipEventRecord(c, st));
        r->timed.push_back(smc_run::Timed{2, a, b});
        r->timed.push_back(smc_run::Timed{3, b, c});
    } else {
        HIP_TRY(launch_resample_one(r->host, r->dev, st, 3));
    }
    r->expect_step = true;
    r->rounds_issued += 1;
    return SMC_OK;
}

// Rounds a model needs when every particle advances in lockstep (0 = unknown).
uint32_t lockstep_rounds(const smc_model* m)
{
    if (m->kind == SMC_MODEL_LGSSM || m->kind == SMC_MODEL_SEIR) return (uint32_t)m->T;
    if (m->kind == SMC_MODEL_CRBD || m->kind == SMC_MODEL_CLADS || m->kind == SMC_MODEL_CRBD_DS)
        return (uint32_t)m->n_nodes;
    return 0;
}

}  // namespace

// ===========================================================================
// C interface
// ===========================================================================
extern "C" {

const char* smc_last_error(void) { return g_error.c_str(); }
const char* smc_version(void) { return "pcfgsmc 0.1 gfx950"; }

smc_status smc_program_check(const smc_program_desc* program) { return check_program(program); }

smc_status smc_ctx_create(int32_t device, void* stream, const smc_allocator* allocator, smc_ctx** out)
{
    if (!out) return fail(SMC_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (allocator && (!allocator->alloc || !allocator->free))
        return fail(SMC_ERR_INVALID, "allocator needs both alloc and free");
    int count = 0;
    HIP_TRY(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) return fail(SMC_ERR_INVALID, "no such device");
    HIP_TRY(hipSetDevice(device));
    void* scratch_ptr = nullptr;
    const smc_status ss = scratch_address(device, &scratch_ptr);
    if (ss != SMC_OK) return ss;
    smc_ctx* c = new (std::nothrow) smc_ctx();
    if (!c) return fail(SMC_ERR_OOM, "host allocation failed");
    c->device = device;
    c->scratch = scratch_ptr;
    c->stream = (hipStream_t)stream;
    if (allocator) {
        c->alloc = *allocator;
        c->custom_alloc = true;
    }
    *out = c;
    return SMC_OK;
}

smc_status smc_ctx_destroy(smc_ctx* ctx)
{
    delete ctx;
    return SMC_OK;
}

smc_status smc_model_register(smc_ctx* ctx, const smc_model_desc* d, smc_model** out)
{
    if (!ctx || !d || !out) return fail(SMC_ERR_INVALID, "NULL argument");
    *out = nullptr;
    if (d->kind < SMC_MODEL_GEOMETRIC || d->kind > SMC_MODEL_PROGRAM) return fail(SMC_ERR_INVALID, "unknown model kind");
    if (d->precision != 32 && d->precision != 64) return fail(SMC_ERR_INVALID, "precision must be 32 or 64");
    if (d->kind == SMC_MODEL_PROGRAM) {
        if (d->precision != 64) return fail(SMC_ERR_INVALID, "compiled programs keep FP64 state: precision must be 64");
        const smc_status s = check_program(d->program);
        if (s != SMC_OK) return s;
    }
    const bool tree = d->kind == SMC_MODEL_CRBD || d->kind == SMC_MODEL_CLADS || d->kind == SMC_MODEL_CRBD_DS;
    if (tree) {
        if (d->n_nodes < 1 || d->n_nodes > 1 << 20 || !d->parent || !d->left || !d->age)
            return fail(SMC_ERR_INVALID, "tree arrays missing or empty");
        if (d->parent[0] != -1) return fail(SMC_ERR_INVALID, "node 0 must be the root");
        for (int i = 1; i < d->n_nodes; ++i)
            if (d->parent[i] < 0 || d->parent[i] >= i || !(d->age[d->parent[i]] >= d->age[i]))
                return fail(SMC_ERR_INVALID, "tree is not in preorder with ages decreasing from the root");
        const int ev = d->kind == SMC_MODEL_CLADS ? 7 : 5;
        if (!(d->params[ev + 1] >= 1.0 && d->params[ev + 1] <= 32.0))
            return fail(SMC_ERR_INVALID, "max depth must be in [1, 32]");
        if (!(d->params[ev] >= 0.0 && d->params[ev] <= 1e6)) return fail(SMC_ERR_INVALID, "max events must be in [0, 10^6]");
        if (!(d->params[0] > 0.0 && d->params[0] <= 1.0)) return fail(SMC_ERR_INVALID, "rho must be in (0, 1]");
        if (d->kind == SMC_MODEL_CRBD_DS && !(d->params[1] > 0.0 && d->params[2] > 0.0))
            return fail(SMC_ERR_INVALID, "prior scales must be positive");
    }
    if ((d->kind == SMC_MODEL_LGSSM || d->kind == SMC_MODEL_SEIR) && (d->T < 1 || d->T > (1 << 24) || !d->y))
        return fail(SMC_ERR_INVALID, "observations missing");
    if (d->kind == SMC_MODEL_SEIR) {
        const double* p = d->params;
        auto count = [](double v) { return v == std::floor(v) && v >= 0.0 && v <= 2147483647.0; };
        if (!(count(p[0]) && p[0] >= 1.0 && p[0] <= 1e7)) return fail(SMC_ERR_INVALID, "humans must be in [1, 10^7]");
        for (int i = 1; i <= 6; ++i)
            if (!(p[i] < 0.0 || p[i] <= 1.0)) return fail(SMC_ERR_INVALID, "fixed rates must lie in [0, 1]");
        for (int i = 7; i <= 10; ++i)
            if (!(p[i] < 0.0 || count(p[i]))) return fail(SMC_ERR_INVALID, "fixed initial counts must be integers");
        if (!(p[7] < 0.0 || p[8] < 0.0 || p[9] < 0.0 || p[7] + p[8] + p[9] <= p[0]))
            return fail(SMC_ERR_INVALID, "initial humans exceed the population");
        for (int t = 0; t < d->T; ++t)
            if (!(d->y[t] == -1.0 || count(d->y[t]))) return fail(SMC_ERR_INVALID, "observations must be counts or -1");
    }
    if (!(d->ess_threshold >= 0.0 && d->ess_threshold <= 1.0))
        return fail(SMC_ERR_INVALID, "ess_threshold must be in [0, 1]");
    smc_model* m = new (std::nothrow) smc_model();
    if (!m) return fail(SMC_ERR_OOM, "host allocation failed");
    m->ctx = ctx;
    m->arena.ctx = ctx;
    m->kind = d->kind;
    m->precision = d->precision;
    m->checkpoint = d->checkpoint;
    m->n_nodes = tree ? d->n_nodes : 0;
    m->T = (d->kind == SMC_MODEL_LGSSM || d->kind == SMC_MODEL_SEIR) ? d->T : 0;
    m->ess_t = (uint32_t)std::nearbyint(d->ess_threshold * 65536.0);
    ModelDev& h = m->host;
    h.kind = d->kind;
    h.precision = d->precision;
    h.checkpoint = d->checkpoint;
    h.n_nodes = m->n_nodes;
    h.T = m->T;
    for (int i = 0; i < 16; ++i) h.p[i] = d->params[i];
    hipStream_t st = ctx->stream;
    auto upload = [&](const void* src, size_t bytes) -> void* {
        void* p = m->arena.get(bytes);
        if (p && hipMemcpyAsync(p, src, bytes, hipMemcpyHostToDevice, st) != hipSuccess) return nullptr;
        return p;
    };
    bool ok = true;
    if (tree) {
        h.parent = (const int32_t*)upload(d->parent, sizeof(int32_t) * d->n_nodes);
        h.left = (const int32_t*)upload(d->left, sizeof(int32_t) * d->n_nodes);
        h.age = (const double*)upload(d->age, sizeof(double) * d->n_nodes);
        ok = h.parent && h.left && h.age;
        if (d->kind == SMC_MODEL_CLADS) {
            // pending right daughters along the preorder walk (same for every particle)
            m->sp_before.assign(d->n_nodes + 1, 0);
            int cur = 1, deepest = 1;
            for (int node = 1; node < d->n_nodes; ++node) {
                m->sp_before[node] = cur;
                cur = d->left[node] >= 0 ? cur + 1 : (cur > 0 ? cur - 1 : 0);
                if (cur > deepest) deepest = cur;
            }
            m->sp_before[d->n_nodes] = cur;
            m->stack_depth = deepest + 1;
            h.stack_depth = m->stack_depth;
            h.sp_before = (const int32_t*)upload(m->sp_before.data(), sizeof(int32_t) * m->sp_before.size());
            ok = ok && h.sp_before;
        }
    }
    if (d->kind == SMC_MODEL_LGSSM || d->kind == SMC_MODEL_SEIR) {
        h.y = (const double*)upload(d->y, sizeof(double) * d->T);
        ok = ok && h.y;
    }
    if (d->kind == SMC_MODEL_PROGRAM) {
        const smc_program_desc* p = d->program;
        static const double zero = 0.0;  // placeholders for empty tables (outlive the async copies)
        static const uint32_t start0 = 0;
        ProgramDev& g = h.prog;
        g.code = (const unsigned long long*)upload(p->code, sizeof(uint64_t) * p->n_code);
        g.block_start = (const uint32_t*)upload(p->block_start, sizeof(uint32_t) * (p->n_blocks + 1));
        g.consts = (const double*)(p->n_consts ? upload(p->consts, sizeof(double) * p->n_consts) : upload(&zero, 8));
        g.data = (const double*)(p->n_data ? upload(p->data, sizeof(double) * p->n_data) : upload(&zero, 8));
        g.array_start = (const uint32_t*)(p->n_arrays ? upload(p->array_start, sizeof(uint32_t) * (p->n_arrays + 1))
                                                      : upload(&start0, 4));
        g.n_blocks = p->n_blocks;
        g.n_arrays = p->n_arrays;
        g.stack_words = p->stack_words;
        g.n_consts = p->n_consts;
        m->stack_depth = (int)p->stack_words;
        h.stack_depth = m->stack_depth;
        ok = ok && g.code && g.block_start && g.consts && g.data && g.array_start;
    }
    m->dev = (ModelDev*)m->arena.get(sizeof(ModelDev));
    ok = ok && m->dev;
    if (!ok) {
        (void)hipStreamSynchronize(st);
        m->arena.release_all();
        delete m;
        return fail(SMC_ERR_OOM, "device allocation failed for model data");
    }
    if (hipMemcpyAsync(m->dev, &m->host, sizeof(ModelDev), hipMemcpyHostToDevice, st) != hipSuccess ||
        launch_model_setup(m->dev, st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
        m->arena.release_all();
        delete m;
        return fail(SMC_ERR_DEVICE, "model upload failed");
    }
    *out = m;
    return SMC_OK;
}

smc_status smc_model_destroy(smc_model* m)
{
    if (!m) return SMC_OK;
    (void)hipStreamSynchronize(m->ctx->stream);
    m->arena.release_all();
    delete m;
    return SMC_OK;
}

smc_status smc_init(smc_model* model, uint64_t n, uint64_t seed, smc_run** out)
{
    if (!model || !out) return fail(SMC_ERR_INVALID, "NULL argument");
    *out = nullptr;
    if (n == 0 || n > kMaxParticles) return fail(SMC_ERR_INVALID, "particle count must be in [1, 2^24]");
    smc_run* r = new (std::nothrow) smc_run();
    if (!r) return fail(SMC_ERR_OOM, "host allocation failed");
    smc_status s = build_run(model, n, seed, r, model->ctx);
    if (s != SMC_OK) {
        delete r;
        return s;
    }
    *out = r;
    return SMC_OK;
}

smc_status smc_step(smc_run* r)
{
    if (!r) return fail(SMC_ERR_INVALID, "NULL run");
    return do_step(r);
}

smc_status smc_resample(smc_run* r)
{
    if (!r) return fail(SMC_ERR_INVALID, "NULL run");
    return do_resample(r);
}

smc_status smc_done(smc_run* r, int32_t* done)
{
    if (!r || !done) return fail(SMC_ERR_INVALID, "NULL argument");
    RunCtl c;
    smc_status s = read_ctl(r, &c);
    if (s != SMC_OK) return s;
    *done = c.status != SMC_OK;
    return c.status;
}

smc_status smc_log_z(smc_run* r, double* out)
{
    if (!r || !out) return fail(SMC_ERR_INVALID, "NULL argument");
    RunCtl c;
    smc_status s = read_ctl(r, &c);
    if (s != SMC_OK) return s;
    *out = c.log_z;
    return c.status;
}

// Capture rounds 0..R-1 of a lockstep model (propagation, reduction, scan per
// round) as one graph. Capture needs a non-legacy stream, so it records on a
// private stream; the graph is then launched on the context's stream.
static smc_status capture_run(smc_run* r, uint32_t rounds)
{
    hipStream_t cap = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    for (uint32_t k = 0; k < rounds && e == hipSuccess; ++k) {
        if (r->host.perm) e = launch_bucket(r->host, cap);
        if (e == hipSuccess) e = launch_propagate_one(r->model->kind, r->model->precision, r->host, cap);
        if (e == hipSuccess) e = launch_resample_one(r->host, r->dev, cap, 3);
    }
    hipError_t e2 = hipStreamEndCapture(cap, &g);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&r->graph, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(cap);
    if (e != hipSuccess) {
        r->graph = nullptr;
        return fail(SMC_ERR_DEVICE, std::string("graph capture failed: ") + hipGetErrorString(e));
    }
    r->graph_rounds = rounds;
    return SMC_OK;
}

smc_status smc_run_to_end(smc_run* r)
{
    if (!r) return fail(SMC_ERR_INVALID, "NULL run");
    if (r->known_status != SMC_OK) return r->known_status;
    const uint32_t known = lockstep_rounds(r->model);
    if (known && r->rounds_issued == 0 && r->expect_step && !r->profiling && (r->graph || r->resets > 0)) {
        if (!r->graph) {
            smc_status s = capture_run(r, known);
            if (s != SMC_OK) return s;
        }
        HIP_TRY(hipGraphLaunch(r->graph, r->ctx->stream));
        r->rounds_issued = known;
        RunCtl c;
        smc_status s = read_ctl(r, &c);
        if (s != SMC_OK) return s;
        if (c.status != SMC_OK) return c.status;
    }
    if (!r->expect_step) {
        smc_status s = do_resample(r);
        if (s != SMC_OK) return s;
    }
    uint32_t chunk = 16;
    if (known && r->rounds_issued < known) chunk = known - r->rounds_issued;
    for (;;) {
        for (uint32_t k = 0; k < chunk; ++k) {
            smc_status s = do_step(r);
            if (s != SMC_OK) return s;
            s = do_resample(r);
            if (s != SMC_OK) return s;
        }
        RunCtl c;
        smc_status s = read_ctl(r, &c);
        if (s != SMC_OK) return s;
        if (c.status != SMC_OK) return c.status;
        chunk = 16;
    }
}

// Device regions holding a run's state between calls: the control block, both
// particle buffers, log-weights, ancestors, ClaDS side stacks and the group
// slots the next propagation folds into (cleared by the previous scan).
// Reduction partials are rewritten before every read, so they are not state.
static std::vector<std::pair<void*, size_t>> state_regions(const smc_run* r)
{
    const smc_model* m = r->model;
    const RunDev& h = r->host;
    const size_t n = r->n, rb = real_bytes(m);
    std::vector<std::pair<void*, size_t>> out;
    out.push_back({h.ctl, sizeof(RunCtl)});
    for (int b = 0; b < 2; ++b) {
        out.push_back({h.buf[b].blk, n});
        for (int f = 0; f < real_fields(m->kind); ++f) out.push_back({h.buf[b].real[f], n * rb});
        for (int f = 0; f < stored_int_fields(m->kind); ++f) out.push_back({h.buf[b].ints[f], n * 4});
        if (h.buf[b].stack) out.push_back({h.buf[b].stack, n * rb * (size_t)m->stack_depth});
    }
    out.push_back({h.lw, n * 8});
    out.push_back({h.anc, n * 4});
    if (h.side_stack) out.push_back({h.side_stack, (size_t)kMaxDepthCap * n * 17});
    out.push_back({h.groups, sizeof(GroupPartials)});
    return out;
}

struct SnapshotHeader {
    uint64_t magic, bytes, n;
    int32_t kind, precision, stack_depth, known_status;
    uint32_t rounds_issued, expect_step;
};
constexpr uint64_t kSnapshotMagic = 0x31746e7370636d73ull;  // "smcpsnt1"

smc_status smc_snapshot(smc_run* r, void* host_dst, size_t* bytes)
{
    if (!r || !bytes) return fail(SMC_ERR_INVALID, "NULL argument");
    const auto regions = state_regions(r);
    size_t need = sizeof(SnapshotHeader);
    for (const auto& g : regions) need += g.second;
    if (!host_dst) {
        *bytes = need;
        return SMC_OK;
    }
    if (*bytes < need) return fail(SMC_ERR_INVALID, "snapshot buffer too small");
    SnapshotHeader hd{kSnapshotMagic, need, r->n, r->model->kind, r->model->precision, r->model->stack_depth,
                      r->known_status, r->rounds_issued, r->expect_step ? 1u : 0u};
    std::memcpy(host_dst, &hd, sizeof hd);
    char* p = static_cast<char*>(host_dst) + sizeof hd;
    hipStream_t st = r->ctx->stream;
    for (const auto& g : regions) {
        HIP_TRY(hipMemcpyAsync(p, g.first, g.second, hipMemcpyDeviceToHost, st));
        p += g.second;
    }
    HIP_TRY(hipStreamSynchronize(st));
    *bytes = need;
    return SMC_OK;
}

smc_status smc_restore(smc_run* r, const void* host_src, size_t bytes)
{
    if (!r || !host_src) return fail(SMC_ERR_INVALID, "NULL argument");
    if (bytes < sizeof(SnapshotHeader)) return fail(SMC_ERR_INVALID, "not a snapshot");
    SnapshotHeader hd;
    std::memcpy(&hd, host_src, sizeof hd);
    const auto regions = state_regions(r);
    size_t need = sizeof(SnapshotHeader);
    for (const auto& g : regions) need += g.second;
    if (hd.magic != kSnapshotMagic || hd.bytes != need || bytes < need)
        return fail(SMC_ERR_INVALID, "not a snapshot of a run of this size");
    if (hd.n != r->n || hd.kind != r->model->kind || hd.precision != r->model->precision ||
        hd.stack_depth != r->model->stack_depth)
        return fail(SMC_ERR_INVALID, "snapshot taken from a run of another model or particle count");
    const char* p = static_cast<const char*>(host_src) + sizeof hd;
    hipStream_t st = r->ctx->stream;
    for (const auto& g : regions) {
        HIP_TRY(hipMemcpyAsync(g.first, p, g.second, hipMemcpyHostToDevice, st));
        p += g.second;
    }
    HIP_TRY(hipStreamSynchronize(st));
    r->rounds_issued = hd.rounds_issued;
    r->expect_step = hd.expect_step != 0;
    r->known_status = hd.known_status;
    return SMC_OK;
}

smc_status smc_set_workgroup(smc_run* r, int32_t lanes)
{
    if (!r) return fail(SMC_ERR_INVALID, "NULL run");
    if (lanes != 128 && lanes != 256) return fail(SMC_ERR_INVALID, "lanes must be 128 or 256");
    if (r->host.lanes == (uint32_t)lanes) return SMC_OK;
    set_prop_tiles(r->host, lanes);
    r->n_prop = r->host.prop_tiles;
    HIP_TRY(hipMemcpyAsync(r->dev, &r->host, sizeof(RunDev), hipMemcpyHostToDevice, r->ctx->stream));
    HIP_TRY(hipStreamSynchronize(r->ctx->stream));
    if (r->graph) {  // the captured launches have the old shape
        (void)hipGraphExecDestroy(r->graph);
        r->graph = nullptr;
    }
    return SMC_OK;
}

smc_status smc_set_bucketing(smc_run* r, int32_t enable)
{
    if (!r) return fail(SMC_ERR_INVALID, "NULL run");
    RunDev& h = r->host;
    const bool on = enable != 0;
    if (on && !r->perm_buf) {
        h.bucket_hist = (uint32_t*)r->arena.get((size_t)kBuckets * h.red_tiles * sizeof(uint32_t));
        h.bucket_total = (uint32_t*)r->arena.get((size_t)kBuckets * sizeof(uint32_t));
        r->perm_buf = (uint32_t*)r->arena.get((size_t)r->n * sizeof(uint32_t));
        if (!h.bucket_hist || !h.bucket_total || !r->perm_buf) {
            h.bucket_hist = nullptr;
            h.bucket_total = nullptr;
            r->perm_buf = nullptr;
            return fail(SMC_ERR_OOM, "device allocation failed for the bucketing buffers");
        }
    }
    if ((h.perm != nullptr) == on) return SMC_OK;
    h.perm = on ? r->perm_buf : nullptr;
    HIP_TRY(hipMemcpyAsync(r->dev, &r->host, sizeof(RunDev), hipMemcpyHostToDevice, r->ctx->stream));
    HIP_TRY(hipStreamSynchronize(r->ctx->stream));
    if (r->graph) {  // the captured launch sequence changes: capture again when next needed
        (void)hipGraphExecDestroy(r->graph);
        r->graph = nullptr;
    }
    return SMC_OK;
}

smc_status smc_reset(smc_run* r, uint64_t seed)
{
    if (!r) return fail(SMC_ERR_INVALID, "NULL run");
    HIP_TRY(launch_reset(r->dev, seed, r->ctx->stream));
    r->seed = seed;
    r->expect_step = true;
    r->rounds_issued = 0;
    r->known_status = SMC_OK;
    r->resets += 1;
    return SMC_OK;
}

smc_status smc_read(smc_run* r, int32_t what, void* dst, size_t bytes)
{
    if (!r || !dst) return fail(SMC_ERR_INVALID, "NULL argument");
    RunCtl c;
    smc_status s = read_ctl(r, &c);
    if (s != SMC_OK) return s;
    const smc_model* m = r->model;
    const uint64_t n = r->n;
    hipStream_t st = r->ctx->stream;
    if (r->rounds_issued == 0 && r->expect_step) return fail(SMC_ERR_STATE, "nothing propagated yet");
    // Where the newest state lives, and whether it still waits for its gather
    // (a round that kept its weights under the ESS rule has nothing to gather).
    const bool resampled_pending = r->expect_step && c.status == SMC_OK;
    const bool pending_gather = resampled_pending && !c.carry;
    const uint32_t last_round = resampled_pending ? c.round - 1 : c.round;
    const ParticleBuf& b = r->host.buf[last_round & 1u];
    const uint32_t* anc = pending_gather ? r->host.anc : nullptr;
    auto fetch = [&](const void* src, int elem, uint64_t levels) -> smc_status {
        const size_t need = (size_t)elem * n * levels;
        if (bytes < need) return fail(SMC_ERR_INVALID, "destination too small");
        void* tmp = r->ctx->allocate(need);
        if (!tmp) return fail(SMC_ERR_OOM, "temporary allocation failed");
        hipError_t e = launch_gather(elem, src, anc, tmp, n, levels, n, st);
        if (e == hipSuccess) e = hipMemcpyAsync(dst, tmp, need, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        r->ctx->release(tmp);
        if (e != hipSuccess) return fail(SMC_ERR_DEVICE, hipGetErrorString(e));
        return SMC_OK;
    };
    if (what == SMC_READ_BLK) return fetch(b.blk, 1, 1);
    if (what == SMC_READ_LW) {
        if (bytes < n * 8) return fail(SMC_ERR_INVALID, "destination too small");
        if (pending_gather) {
            std::memset(dst, 0, n * 8);  // weights are reset by resampling
            return SMC_OK;
        }
        HIP_TRY(hipMemcpyAsync(dst, r->host.lw, n * 8, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        return SMC_OK;
    }
    if (what == SMC_READ_ANC) {
        if (bytes < n * 4) return fail(SMC_ERR_INVALID, "destination too small");
        if (c.carry) {  // the last smc_resample kept the weights: identity ancestors
            uint32_t* o = (uint32_t*)dst;
            for (uint64_t i = 0; i < n; ++i) o[i] = (uint32_t)i;
            return SMC_OK;
        }
        HIP_TRY(hipMemcpyAsync(dst, r->host.anc, n * 4, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        return SMC_OK;
    }
    int f = what - SMC_READ_FIELD0;
    const int nr = real_fields(m->kind);
    const int elem = (int)real_bytes(m);
    if (f >= 0 && f < nr) return fetch(b.real[f], elem, 1);
    f -= nr;
    if (f >= 0 && f < logical_int_fields(m->kind)) {
        if (bytes < n * 4) return fail(SMC_ERR_INVALID, "destination too small");
        if (f < stored_int_fields(m->kind)) return fetch(b.ints[f], 4, 1);
        // cursor-like fields advance once per round for every particle
        int32_t v = (int32_t)last_round + 1;
        if (m->kind == SMC_MODEL_CLADS && f == 1) {
            const int node = (int)last_round;
            if (node == 0) v = 1;
            else v = m->sp_before[node + 1 <= m->n_nodes ? node + 1 : m->n_nodes];
        }
        int32_t* o = (int32_t*)dst;
        for (uint64_t i = 0; i < n; ++i) o[i] = v;
        return SMC_OK;
    }
    f -= logical_int_fields(m->kind);
    if (f == 0 && (m->kind == SMC_MODEL_CLADS || m->kind == SMC_MODEL_PROGRAM)) {
        const uint64_t depth = (uint64_t)m->stack_depth;
        const size_t need = (size_t)elem * n * depth;
        if (bytes < need) return fail(SMC_ERR_INVALID, "destination too small");
        std::vector<char> level_major(need);
        s = fetch(b.stack, elem, depth);
        if (s != SMC_OK) return s;
        // fetch wrote level-major into dst; transpose to [particle][level]
        std::memcpy(level_major.data(), dst, need);
        char* o = (char*)dst;
        for (uint64_t i = 0; i < n; ++i)
            for (uint64_t k = 0; k < depth; ++k)
                std::memcpy(o + (i * depth + k) * elem, level_major.data() + (k * n + i) * elem, elem);
        return SMC_OK;
    }
    return fail(SMC_ERR_INVALID, "unknown read selector");
}

smc_status smc_run_stats(smc_run* r, smc_stats* out)
{
    if (!r || !out) return fail(SMC_ERR_INVALID, "NULL argument");
    RunCtl c;
    smc_status s = read_ctl(r, &c);
    if (s != SMC_OK) return s;
    out->round = c.round;
    out->status = c.status;
    out->block_steps = c.block_steps;
    out->log_z = c.log_z;
    out->stack_depth = r->model->stack_depth;
    out->resamples = c.resamples;
    return SMC_OK;
}

smc_status smc_profile(smc_run* r, int32_t enable)
{
    if (!r) return fail(SMC_ERR_INVALID, "NULL run");
    HIP_TRY(hipStreamSynchronize(r->ctx->stream));
    r->profiling = enable != 0;
    r->timed.clear();
    r->events_used = 0;
    return SMC_OK;
}

smc_status smc_profile_read(smc_run* r, smc_kernel_times* out)
{
    if (!r || !out) return fail(SMC_ERR_INVALID, "NULL argument");
    HIP_TRY(hipStreamSynchronize(r->ctx->stream));
    std::memset(out, 0, sizeof(*out));
    for (const auto& t : r->timed) {
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, t.start, t.end));
        out->ms[t.kernel] += ms;
        out->launches[t.kernel] += 1;
    }
    return SMC_OK;
}

smc_status smc_run_destroy(smc_run* r)
{
    if (!r) return SMC_OK;
    (void)hipStreamSynchronize(r->ctx->stream);
    r->arena.release_all();
    delete r;
    return SMC_OK;
}

smc_status smc_resample_weights(smc_ctx* ctx, const double* lw, uint64_t n, uint64_t seed, uint32_t round,
                                uint32_t* anc, double* logz_inc)
{
    if (!ctx || !lw || !anc || !logz_inc) return fail(SMC_ERR_INVALID, "NULL argument");
    if (n == 0 || n > kMaxParticles) return fail(SMC_ERR_INVALID, "n must be in [1, 2^24]");
    DeviceArena arena;
    arena.ctx = ctx;
    RunDev h{};
    h.n = (uint32_t)n;
    h.red_tiles = (uint32_t)((n + kTileRed - 1) / kTileRed);
    set_prop_tiles(h, kMaxkeyThreads);
    h.lw = const_cast<double*>(lw);
    h.anc = anc;
    h.ctl = (RunCtl*)arena.get(sizeof(RunCtl));
    h.groups = (GroupPartials*)arena.get(sizeof(GroupPartials));
    h.part_q = (double*)arena.get(h.red_tiles * 8);
    h.part_e = (double*)arena.get(h.red_tiles * 8);
    h.prefix = (double*)arena.get(h.red_tiles * 8);
    RunDev* dev = (RunDev*)arena.get(sizeof(RunDev));
    TileRef* tiles = (TileRef*)arena.get(sizeof(TileRef) * h.red_tiles);
    TileRef* ptiles = (TileRef*)arena.get(sizeof(TileRef) * h.prop_tiles);
    if (!h.ctl || !h.groups || !h.part_q || !h.part_e || !h.prefix || !dev ||
        !tiles || !ptiles) {
        arena.release_all();
        return fail(SMC_ERR_OOM, "device allocation failed");
    }
    std::vector<TileRef> th(h.red_tiles), ph(h.prop_tiles);
    for (uint32_t t = 0; t < h.red_tiles; ++t) th[t] = TileRef{0, t};
    for (uint32_t t = 0; t < h.prop_tiles; ++t) ph[t] = TileRef{0, t};
    RunCtl c0{};
    c0.round = round;
    c0.seed = seed;
    hipStream_t st = ctx->stream;
    hipError_t e = hipMemcpyAsync(h.ctl, &c0, sizeof(RunCtl), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(dev, &h, sizeof(RunDev), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(tiles, th.data(), sizeof(TileRef) * th.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(ptiles, ph.data(), sizeof(TileRef) * ph.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemsetAsync(h.groups, 0, sizeof(GroupPartials), st);
    if (e == hipSuccess) e = launch_maxkey(dev, ptiles, h.prop_tiles, st);
    if (e == hipSuccess) e = launch_reduce(dev, tiles, h.red_tiles, 1, !h.fused, st);
    if (e == hipSuccess) e = launch_scan_anc(dev, tiles, h.red_tiles, st);
    if (e == hipSuccess) e = hipMemcpyAsync(logz_inc, &h.ctl->log_z, sizeof(double), hipMemcpyDeviceToDevice, st);
    RunCtl c{};
    if (e == hipSuccess) e = hipMemcpyAsync(&c, h.ctl, sizeof(RunCtl), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    arena.release_all();
    if (e != hipSuccess) return fail(SMC_ERR_DEVICE, hipGetErrorString(e));
    return c.status;
}

smc_status smc_resample_weights_noalloc(smc_ctx* ctx, const double* lw, uint64_t n, uint64_t seed, uint32_t round,
                                        uint32_t* anc, double* logz_inc)
{
    if (!ctx || !lw || !anc || !logz_inc) return fail(SMC_ERR_INVALID, "NULL argument");
    if (n == 0 || n > kMaxParticles) return fail(SMC_ERR_INVALID, "n must be in [1, 2^24]");
    if (!ctx->scratch) return fail(SMC_ERR_STATE, "context has no scratch address");
    unsigned char* base = static_cast<unsigned char*>(ctx->scratch);
    RunDev h{};
    h.n = (uint32_t)n;
    h.red_tiles = (uint32_t)((n + kTileRed - 1) / kTileRed);
    if (h.red_tiles > kNoallocMaxTiles) return fail(SMC_ERR_INVALID, "n beyond the scratch capacity");
    set_prop_tiles(h, kMaxkeyThreads);
    h.lw = const_cast<double*>(lw);
    h.anc = anc;
    h.ctl = reinterpret_cast<RunCtl*>(base + kNoallocCtlOff);
    h.groups = reinterpret_cast<GroupPartials*>(base + kNoallocGroupsOff);
    h.part_q = reinterpret_cast<double*>(base + kNoallocPartOff);
    h.part_e = reinterpret_cast<double*>(base + kNoallocPartOff + kNoallocPartBytes);
    h.prefix = reinterpret_cast<double*>(base + kNoallocPartOff + 2 * kNoallocPartBytes);
    hipStream_t st = ctx->stream;
    hipError_t e = launch_resample_weights_one(h, round, seed, logz_inc, st);
    int32_t status = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&status, &h.ctl->status, sizeof(status), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(SMC_ERR_DEVICE, hipGetErrorString(e));
    return status;
}

// ---------------------------------------------------------------------------
// Batches: the same round kernels over a combined (run, tile) table.
// ---------------------------------------------------------------------------
}  // extern "C"

struct smc_batch {
    smc_ctx* ctx = nullptr;
    std::vector<smc_run*> slots;  // nullptr = free slot
    bool dirty = true;
    DeviceArena tables;
    RunDev* runs = nullptr;
    struct Group {
        int kind, precision, lanes;
        TileRef* tiles;
        uint32_t n;
    };
    std::vector<Group> groups;
    struct Owned {  // runs owned by one work-group each, one launch per tick
        int kind, precision;
        uint32_t* ids;
        uint32_t n;
    };
    std::vector<Owned> owned;
    std::vector<std::vector<uint32_t>> owned_ids_h;
    TileRef* red_tiles = nullptr;
    uint32_t n_red = 0;
    std::vector<RunDev> runs_h;
    bool any_unfused = false;
    std::vector<std::vector<TileRef>> group_tiles_h;
    std::vector<TileRef> red_tiles_h;
    // A tick of an unchanged batch is a fixed launch sequence: from the second
    // such tick on it is captured once and replayed.
    hipGraphExec_t graph = nullptr;
    int32_t graph_rounds = 0;
    uint32_t same_ticks = 0;
    ~smc_batch()
    {
        if (graph) (void)hipGraphExecDestroy(graph);
    }
};

namespace {

// Drops the device tables and the host lists they were built from; the next
// tick rebuilds them (dirty stays set).
void clear_tables(smc_batch* b)
{
    b->tables.release_all();
    b->runs = nullptr;
    b->red_tiles = nullptr;
    b->n_red = 0;
    b->groups.clear();
    b->owned.clear();
    b->owned_ids_h.clear();
    b->runs_h.clear();
    b->group_tiles_h.clear();
    b->red_tiles_h.clear();
    b->any_unfused = false;
    b->dirty = true;
}

// Rebuilds the (run, tile) tables of the live runs. The batch counts as
// rebuilt (dirty cleared) only once every table is on the device: after a
// failed allocation or copy the tables are released and the next tick
// rebuilds them from scratch, so no kernel ever sees a partial table.
smc_status rebuild_tables(smc_batch* b)
{
    hipStream_t st = b->ctx->stream;
    HIP_TRY(hipStreamSynchronize(st));  // old tables may still be in use
    if (b->graph) {  // it launches over the old tables
        (void)hipGraphExecDestroy(b->graph);
        b->graph = nullptr;
    }
    b->same_ticks = 0;
    clear_tables(b);
    struct Key {
        int kind, precision, lanes;
    };
    std::vector<Key> keys;
    std::vector<Key> owned_keys;
    for (smc_run* r : b->slots) {
        if (!r) continue;
        const uint32_t idx = (uint32_t)b->runs_h.size();
        b->runs_h.push_back(r->host);
        if (!r->host.fused) b->any_unfused = true;
        if (r->owned) {
            size_t g = 0;
            for (; g < owned_keys.size(); ++g)
                if (owned_keys[g].kind == r->model->kind && owned_keys[g].precision == r->model->precision) break;
            if (g == owned_keys.size()) {
                owned_keys.push_back(Key{r->model->kind, r->model->precision, 0});
                b->owned_ids_h.emplace_back();
            }
            b->owned_ids_h[g].push_back(idx);
            continue;
        }
        size_t g = 0;
        const int lanes = (int)r->host.lanes;
        for (; g < keys.size(); ++g)
            if (keys[g].kind == r->model->kind && keys[g].precision == r->model->precision && keys[g].lanes == lanes)
                break;
        if (g == keys.size()) {
            keys.push_back(Key{r->model->kind, r->model->precision, lanes});
            b->group_tiles_h.emplace_back();
        }
        for (uint32_t t = 0; t < r->n_prop; ++t) b->group_tiles_h[g].push_back(TileRef{idx, t});
        for (uint32_t t = 0; t < r->n_red; ++t) b->red_tiles_h.push_back(TileRef{idx, t});
    }
    if (b->runs_h.empty()) {
        b->dirty = false;
        return SMC_OK;
    }
    auto undo = [&](smc_status s) {
        clear_tables(b);
        return s;
    };
    b->runs = (RunDev*)b->tables.get(sizeof(RunDev) * b->runs_h.size());
    // every run may be owned by a work-group: then there are no tile tables
    const bool any_tiles = !b->red_tiles_h.empty();
    b->red_tiles = any_tiles ? (TileRef*)b->tables.get(sizeof(TileRef) * b->red_tiles_h.size()) : nullptr;
    if (!b->runs || (any_tiles && !b->red_tiles)) return undo(fail(SMC_ERR_OOM, "batch table allocation failed"));
    hipError_t e = hipMemcpyAsync(b->runs, b->runs_h.data(), sizeof(RunDev) * b->runs_h.size(),
                                  hipMemcpyHostToDevice, st);
    if (e == hipSuccess && any_tiles)
        e = hipMemcpyAsync(b->red_tiles, b->red_tiles_h.data(), sizeof(TileRef) * b->red_tiles_h.size(),
                           hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return undo(fail(SMC_ERR_DEVICE, std::string("batch tables: ") + hipGetErrorString(e)));
    for (size_t g = 0; g < owned_keys.size(); ++g) {
        const size_t bytes = sizeof(uint32_t) * b->owned_ids_h[g].size();
        uint32_t* ids = (uint32_t*)b->tables.get(bytes);
        if (!ids) return undo(fail(SMC_ERR_OOM, "batch table allocation failed"));
        e = hipMemcpyAsync(ids, b->owned_ids_h[g].data(), bytes, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return undo(fail(SMC_ERR_DEVICE, std::string("batch tables: ") + hipGetErrorString(e)));
        b->owned.push_back(smc_batch::Owned{owned_keys[g].kind, owned_keys[g].precision, ids,
                                            (uint32_t)b->owned_ids_h[g].size()});
    }
    for (size_t g = 0; g < keys.size(); ++g) {
        TileRef* t = (TileRef*)b->tables.get(sizeof(TileRef) * b->group_tiles_h[g].size());
        if (!t) return undo(fail(SMC_ERR_OOM, "batch table allocation failed"));
        e = hipMemcpyAsync(t, b->group_tiles_h[g].data(), sizeof(TileRef) * b->group_tiles_h[g].size(),
                           hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return undo(fail(SMC_ERR_DEVICE, std::string("batch tables: ") + hipGetErrorString(e)));
        b->groups.push_back(smc_batch::Group{keys[g].kind, keys[g].precision, keys[g].lanes, t,
                                             (uint32_t)b->group_tiles_h[g].size()});
    }
    b->n_red = (uint32_t)b->red_tiles_h.size();
    b->dirty = false;
    return SMC_OK;
}

}  // namespace

extern "C" {

smc_status smc_batch_create(smc_ctx* ctx, smc_batch** out)
{
    if (!ctx || !out) return fail(SMC_ERR_INVALID, "NULL argument");
    smc_batch* b = new (std::nothrow) smc_batch();
    if (!b) return fail(SMC_ERR_OOM, "host allocation failed");
    b->ctx = ctx;
    b->tables.ctx = ctx;
    *out = b;
    return SMC_OK;
}

smc_status smc_batch_add(smc_batch* b, smc_model* model, uint64_t n, uint64_t seed, int32_t* slot)
{
    if (!b || !model || !slot) return fail(SMC_ERR_INVALID, "NULL argument");
    // a model registered on another context of the same device will do (its
    // registration has completed; its memory is the device's)
    if (model->ctx->device != b->ctx->device) return fail(SMC_ERR_INVALID, "model belongs to another device");
    if (n == 0 || n > kMaxParticles) return fail(SMC_ERR_INVALID, "particle count must be in [1, 2^24]");
    smc_run* r = new (std::nothrow) smc_run();
    if (!r) return fail(SMC_ERR_OOM, "host allocation failed");
    const smc_status s = build_run(model, n, seed, r, b->ctx);
    if (s != SMC_OK) {
        delete r;
        return s;
    }
    int32_t idx = -1;
    for (size_t i = 0; i < b->slots.size(); ++i)
        if (!b->slots[i]) {
            idx = (int32_t)i;
            break;
        }
    if (idx < 0) {
        idx = (int32_t)b->slots.size();
        b->slots.push_back(nullptr);
    }
    b->slots[idx] = r;
    b->dirty = true;
    *slot = idx;
    return SMC_OK;
}

smc_status smc_batch_set_workgroup(smc_batch* b, int32_t slot, int32_t lanes)
{
    if (!b) return fail(SMC_ERR_INVALID, "NULL batch");
    if (slot < 0 || (size_t)slot >= b->slots.size() || !b->slots[slot]) return fail(SMC_ERR_INVALID, "no such slot");
    if (lanes != 128 && lanes != 256) return fail(SMC_ERR_INVALID, "lanes must be 128 or 256");
    smc_run* r = b->slots[slot];
    if (r->host.lanes == (uint32_t)lanes) return SMC_OK;
    const smc_status s = smc_set_workgroup(r, lanes);
    if (s != SMC_OK) return s;
    b->dirty = true;  // its tiles move to the group of that size
    return SMC_OK;
}

smc_status smc_batch_set_owned(smc_batch* b, int32_t slot, int32_t owned)
{
    if (!b) return fail(SMC_ERR_INVALID, "NULL batch");
    if (slot < 0 || (size_t)slot >= b->slots.size() || !b->slots[slot]) return fail(SMC_ERR_INVALID, "no such slot");
    smc_run* r = b->slots[slot];
    if (owned && (r->model->kind == SMC_MODEL_PROGRAM || r->n > kOwnedMaxParticles))
        return fail(SMC_ERR_INVALID, "a work-group owns only built-in models of at most 4096 particles");
    if (r->owned == (owned != 0)) return SMC_OK;
    r->owned = owned != 0;
    b->dirty = true;
    return SMC_OK;
}

smc_status smc_batch_tick(smc_batch* b, int32_t rounds)
{
    if (!b || rounds < 0) return fail(SMC_ERR_INVALID, "bad argument");
    if (b->dirty) {
        smc_status s = rebuild_tables(b);
        if (s != SMC_OK) return s;
    }
    if (b->runs_h.empty()) return SMC_OK;
    hipStream_t st = b->ctx->stream;
    auto enqueue = [&](hipStream_t s) -> hipError_t {
        const uint32_t n_runs = (uint32_t)b->runs_h.size();
        for (const auto& o : b->owned) {  // every round of the tick in one launch
            const hipError_t e = launch_owned(o.kind, o.precision, b->runs, o.ids, o.n, (uint32_t)rounds, s);
            if (e != hipSuccess) return e;
        }
        if (b->groups.empty() && b->n_red == 0) return hipSuccess;  // no segmented runs
        for (int32_t k = 0; k < rounds; ++k) {
            for (const auto& g : b->groups) {
                const hipError_t e = launch_propagate(g.kind, g.precision, g.lanes, b->runs, g.tiles, g.n, s);
                if (e != hipSuccess) return e;
            }
            hipError_t e = launch_reduce(b->runs, b->red_tiles, b->n_red, n_runs, b->any_unfused, s);
            if (e == hipSuccess) e = launch_scan_anc(b->runs, b->red_tiles, b->n_red, s);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    if (b->graph && b->graph_rounds != rounds) {
        (void)hipGraphExecDestroy(b->graph);
        b->graph = nullptr;
    }
    if (!b->graph && b->same_ticks >= 1 && rounds > 0) {
        // Capture on a private stream (capture needs a non-legacy stream); if
        // it fails the tick simply runs eagerly.
        hipStream_t cap = nullptr;
        if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) == hipSuccess) {
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) e = enqueue(cap);
            const hipError_t e2 = hipStreamEndCapture(cap, &g);
            if (e == hipSuccess) e = e2;
            if (e == hipSuccess) e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
            if (e != hipSuccess) b->graph = nullptr;
            if (g) (void)hipGraphDestroy(g);
            (void)hipStreamDestroy(cap);
            (void)hipGetLastError();
            if (b->graph) b->graph_rounds = rounds;
        }
    }
    if (b->graph) {
        HIP_TRY(hipGraphLaunch(b->graph, st));
    } else {
        HIP_TRY(enqueue(st));
    }
    b->same_ticks += 1;
    for (smc_run* r : b->slots)
        if (r) r->rounds_issued += (uint32_t)rounds;
    return SMC_OK;
}

smc_status smc_batch_poll(smc_batch* b, int32_t slots, int32_t* done, double* log_z, int32_t* status,
                          uint64_t* block_steps)
{
    if (!b || slots < 0) return fail(SMC_ERR_INVALID, "bad argument");
    const int32_t m = slots < (int32_t)b->slots.size() ? slots : (int32_t)b->slots.size();
    std::vector<RunCtl> c(m);
    hipStream_t st = b->ctx->stream;
    for (int32_t i = 0; i < m; ++i)
        if (b->slots[i]) HIP_TRY(hipMemcpyAsync(&c[i], b->slots[i]->host.ctl, sizeof(RunCtl), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int32_t i = 0; i < slots; ++i) {
        const bool live = i < m && b->slots[i];
        if (done) done[i] = live ? (c[i].status != SMC_OK) : 1;
        if (log_z) log_z[i] = live ? c[i].log_z : 0.0;
        if (status) status[i] = live ? c[i].status : SMC_ERR_STATE;
        if (block_steps) block_steps[i] = live ? c[i].block_steps : 0;
    }
    return SMC_OK;
}

smc_status smc_batch_retire(smc_batch* b, int32_t slot)
{
    if (!b || slot < 0 || slot >= (int32_t)b->slots.size() || !b->slots[slot])
        return fail(SMC_ERR_INVALID, "no such slot");
    smc_run_destroy(b->slots[slot]);
    b->slots[slot] = nullptr;
    b->dirty = true;
    return SMC_OK;
}

smc_status smc_batch_destroy(smc_batch* b)
{
    if (!b) return SMC_OK;
    (void)hipStreamSynchronize(b->ctx->stream);
    for (smc_run* r : b->slots) smc_run_destroy(r);
    b->tables.release_all();
    delete b;
    return SMC_OK;
}

smc_status smc_selftest_math(smc_ctx* ctx, int32_t op, const double* in, double* out, uint64_t n)
{
    if (!ctx || !in || !out) return fail(SMC_ERR_INVALID, "NULL argument");
    if (op < 0 || op > 15) return fail(SMC_ERR_INVALID, "unknown op");
    if (n == 0) return SMC_OK;
    HIP_TRY(launch_selftest_math(op, in, out, n, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return SMC_OK;
}

smc_status smc_selftest_philox(smc_ctx* ctx, const uint32_t* ctr, const uint32_t* key, uint32_t* out, uint64_t n)
{
    if (!ctx || !ctr || !key || !out) return fail(SMC_ERR_INVALID, "NULL argument");
    if (n == 0) return SMC_OK;
    HIP_TRY(launch_selftest_philox(ctr, key, out, n, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return SMC_OK;
}

}  // extern "C"
