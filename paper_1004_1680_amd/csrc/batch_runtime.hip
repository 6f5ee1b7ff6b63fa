// Batched ensembles of uneven periodic boxes (C ABI part of mhd.h).
//
// All boxes live in one pair of device buffers; box b holds its 8 fields
// contiguously at an element offset.  A step is the per-box CFL (segmented
// FP64 max-reduction, each box its own dt and relaxation speed) followed by
// the 12 operators, each ONE persistent launch over the (box, tile) work
// items of its direction, and the per-box time advance.  Every field is
// written 6 times per step, so after a full step the state is back in the
// buffer it started in, and the captured HIP graph of one step can be
// replayed for any number of steps.  With the middle M_z M_z F_z in one
// launch the face fields are written 5 times per step: they alternate
// between the buffers (cur), and the captured graph holds two steps.
#include <hip/hip_runtime.h>

#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "../../include/mhd.h"
#include "mhd_kernels.h"
#include "runtime_common.h"

using namespace mhd;
#define HIP_TRY MHD_HIP_TRY

struct mhd_batch {
    int nbox;
    std::vector<BoxDesc> boxes;
    BoxDesc* d_boxes;
    double gamma;
    int prec;
    size_t esize;
    hipStream_t stream;
    bool own_stream;
    int device;
    size_t total;                 // elements per buffer
    void* buf[2];
    int cur[8];
    double* scal;                 // nbox x SCAL_COUNT
    int* flag;                    // nbox x FLAG_COUNT
    int2* d_items[3];
    int nitems[3];
    int2* d_pitems[3];            // work lists of the fused pairs along y, z (x: d_items[0])
    int npitems[3];
    int2* d_cfl_items;
    int n_cfl_items;
    int* d_item_first;
    double* partial;
    int* partial_bad;
    int grid[3];
    int chunk_target;
    int pair_chunk_target;
    int rev_mode;           // reverse-half pairs M_d F_d: 0 built-in, 1 one launch each, 2 two
    int mid_mode;           // M_z M_z F_z: 0 built-in, 1 one launch, 2 M_z and the z pair
    int limiter;            // slope limiter of the operators (MHD_LIMITER_*)
    // fused CFL: the last launch of a step leaves each box's FP64 maximum
    // signal speed in cfl_acc (CFL_ACC_SLOTS + 1 words per box); acc_valid
    // while the state is the one those maxima describe
    unsigned long long* cfl_acc;
    bool acc_valid;
    bool wide;              // 64-bit addressing in the marches even where 32-bit offsets fit
    hipGraph_t graph;
    hipGraphExec_t exec;
    double graph_cfl;
    bool graph_valid;
    int graph_steps;        // steps in the captured graph (1, or 2 with the fused middle)
    int graph_bpar;         // buffer of the face fields when the graph starts
    bool failed;
};

static int pick_chunk(int n, int target)
{
    int best = 0;
    for (int c = 8; c <= n; ++c)
        if (n % c == 0 && c <= target) best = c;
    if (!best)
        for (int c = 8; c <= n; ++c)
            if (n % c == 0) { best = c; break; }
    return best;
}

static void free_lists(mhd_batch* b)
{
    for (int d = 0; d < 3; ++d) {
        if (b->d_items[d]) { (void)hipFree(b->d_items[d]); b->d_items[d] = nullptr; }
        if (b->d_pitems[d]) { (void)hipFree(b->d_pitems[d]); b->d_pitems[d] = nullptr; }
    }
    if (b->d_boxes) { (void)hipFree(b->d_boxes); b->d_boxes = nullptr; }
}

static void drop_graph(mhd_batch* b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_valid = false;
}

// (re)build box shapes and the work lists of the three directions
static int build_lists(mhd_batch* b)
{
    free_lists(b);
    drop_graph(b);
    std::vector<int2> items[3], pitems[3];
    for (int i = 0; i < b->nbox; ++i) {
        BoxDesc& bd = b->boxes[i];
        bd.chunk[0] = bd.pchunk[0] = 0;
        bd.chunk[1] = pick_chunk(bd.n[1], b->chunk_target);
        bd.chunk[2] = pick_chunk(bd.n[2], b->chunk_target);
        bd.pchunk[1] = pick_chunk(bd.n[1], b->pair_chunk_target);
        bd.pchunk[2] = pick_chunk(bd.n[2], b->pair_chunk_target);
        bd.tpr = bd.n[0] / 4;
        bd.rpw = std::max(1, 256 / bd.tpr);
        bd.ntile[0] = (bd.n[1] * bd.n[2] + bd.rpw - 1) / bd.rpw;
        for (int d = 1; d < 3; ++d) {
            const long lanes = (long)bd.n[0] * (d == 1 ? bd.n[2] : bd.n[1]) * (bd.n[d] / bd.chunk[d]);
            bd.ntile[d] = (int)((lanes + 255) / 256);
        }
        // x tiles in the single-grid visit order (groups of rows along y, one
        // group per z in turn), so the rows z +- 1 a tile reads were read a
        // few items earlier on the same XCD
        const int st = row_group_tiles(bd.n[1], bd.rpw, 0);
        const int ty = bd.n[1] / bd.rpw;
        for (int t = 0; t < bd.ntile[0]; ++t) items[0].push_back(make_int2(i, row_tile(t, st, ty, bd.n[2])));
        for (int d = 1; d < 3; ++d)
            for (int t = 0; t < bd.ntile[d]; ++t) items[d].push_back(make_int2(i, t));
        for (int d = 1; d < 3; ++d) {
            const long lanes = (long)bd.n[0] * (d == 1 ? bd.n[2] : bd.n[1]) * (bd.n[d] / bd.pchunk[d]);
            const int nt = (int)((lanes + 255) / 256);
            for (int t = 0; t < nt; ++t) pitems[d].push_back(make_int2(i, t));
        }
    }
    HIP_TRY(b, hipMalloc(&b->d_boxes, sizeof(BoxDesc) * b->nbox));
    HIP_TRY(b, hipMemcpy(b->d_boxes, b->boxes.data(), sizeof(BoxDesc) * b->nbox,
                         hipMemcpyHostToDevice));
    for (int d = 0; d < 3; ++d) {
        b->nitems[d] = (int)items[d].size();
        HIP_TRY(b, hipMalloc(&b->d_items[d], sizeof(int2) * items[d].size()));
        HIP_TRY(b, hipMemcpy(b->d_items[d], items[d].data(), sizeof(int2) * items[d].size(),
                             hipMemcpyHostToDevice));
    }
    for (int d = 1; d < 3; ++d) {
        b->npitems[d] = (int)pitems[d].size();
        HIP_TRY(b, hipMalloc(&b->d_pitems[d], sizeof(int2) * pitems[d].size()));
        HIP_TRY(b, hipMemcpy(b->d_pitems[d], pitems[d].data(), sizeof(int2) * pitems[d].size(),
                             hipMemcpyHostToDevice));
    }
    return MHD_OK;
}

extern "C" void mhd_batch_destroy(mhd_batch* b)
{
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    drop_graph(b);
    free_lists(b);
    void* ptrs[] = { b->buf[0], b->buf[1], b->scal, b->flag, b->d_cfl_items, b->d_item_first,
                     b->partial, b->partial_bad, b->cfl_acc };
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

extern "C" mhd_batch* mhd_batch_create(int nbox, const int* dims, double gamma, int prec,
                                       void* hip_stream)
{
    if (nbox < 1 || !dims) {
        mhd_fail(MHD_EINVAL, "need nbox >= 1 and a dims array of 3*nbox ints");
        return nullptr;
    }
    if (!(gamma > 1.0) || !isfinite(gamma)) {
        mhd_fail(MHD_EINVAL, "gamma must be > 1 (got %g)", gamma);
        return nullptr;
    }
    if (prec != MHD_F32 && prec != MHD_F64) {
        mhd_fail(MHD_EINVAL, "precision must be MHD_F32 or MHD_F64");
        return nullptr;
    }
    for (int i = 0; i < nbox; ++i) {
        for (int d = 0; d < 3; ++d)
            if (dims[3 * i + d] < 8 || dims[3 * i + d] % 4) {
                mhd_fail(MHD_EINVAL, "box %d dimension %d = %d: must be >= 8 and a multiple of 4", i,
                         d, dims[3 * i + d]);
                return nullptr;
            }
        if (dims[3 * i] > 1024 || dims[3 * i + 1] > 4096 || dims[3 * i + 2] > 4096 ||
            (long long)dims[3 * i] * dims[3 * i + 1] * dims[3 * i + 2] >= (1LL << 31)) {
            mhd_fail(MHD_EINVAL, "box %d above the size limit", i);
            return nullptr;
        }
    }
    mhd_batch* b = new mhd_batch();
    b->nbox = nbox;
    b->gamma = gamma;
    b->prec = prec;
    b->esize = prec == MHD_F64 ? sizeof(double) : sizeof(float);
    b->chunk_target = 64;
    b->pair_chunk_target = 128;
    b->rev_mode = 0;
    b->mid_mode = 0;
    b->limiter = MHD_LIMITER_VANLEER;
    b->wide = false;
    b->d_boxes = nullptr;
    for (int d = 0; d < 3; ++d) {
        b->d_items[d] = b->d_pitems[d] = nullptr;
        b->nitems[d] = b->npitems[d] = 0;
        b->grid[d] = 1024;
    }
    b->buf[0] = b->buf[1] = nullptr;
    b->scal = nullptr; b->flag = nullptr;
    b->d_cfl_items = nullptr; b->d_item_first = nullptr;
    b->partial = nullptr; b->partial_bad = nullptr;
    b->graph = nullptr; b->exec = nullptr; b->graph_valid = false;
    b->graph_steps = 1; b->graph_bpar = 0;
    b->failed = false;
    for (int q = 0; q < 8; ++q) b->cur[q] = 0;
    if (hipGetDevice(&b->device) != hipSuccess) {
        mhd_fail(MHD_EDEVICE, "no HIP device");
        delete b;
        return nullptr;
    }
    if (hip_stream) {
        b->stream = (hipStream_t)hip_stream;
        b->own_stream = false;
    } else {
        // graph capture needs a stream other than the legacy default one
        if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
            mhd_fail(MHD_EDEVICE, "stream creation failed");
            delete b;
            return nullptr;
        }
        b->own_stream = true;
    }
    b->boxes.resize(nbox);
    size_t off = 0;
    std::vector<int2> cfl_items;
    std::vector<int> first(nbox + 1);
    for (int i = 0; i < nbox; ++i) {
        BoxDesc& bd = b->boxes[i];
        memset(&bd, 0, sizeof bd);
        for (int d = 0; d < 3; ++d) bd.n[d] = dims[3 * i + d];
        bd.ncell = (unsigned)((size_t)bd.n[0] * bd.n[1] * bd.n[2]);
        bd.off = off;
        off += 8 * (size_t)bd.ncell;
        first[i] = (int)cfl_items.size();
        const int nblk = (int)((bd.ncell + CFL_CELLS - 1) / CFL_CELLS);
        for (int k = 0; k < nblk; ++k) cfl_items.push_back(make_int2(i, k));
    }
    first[nbox] = (int)cfl_items.size();
    b->total = off;
    b->n_cfl_items = (int)cfl_items.size();
    const size_t bytes = off * b->esize;
    bool ok = hipMalloc(&b->buf[0], bytes) == hipSuccess && hipMalloc(&b->buf[1], bytes) == hipSuccess &&
              hipMalloc(&b->scal, sizeof(double) * SCAL_COUNT * nbox) == hipSuccess &&
              hipMalloc(&b->flag, sizeof(int) * FLAG_COUNT * nbox) == hipSuccess &&
              hipMalloc(&b->d_cfl_items, sizeof(int2) * cfl_items.size()) == hipSuccess &&
              hipMalloc(&b->d_item_first, sizeof(int) * (nbox + 1)) == hipSuccess &&
              hipMalloc(&b->partial, sizeof(double) * cfl_items.size()) == hipSuccess &&
              hipMalloc(&b->partial_bad, sizeof(int) * cfl_items.size()) == hipSuccess &&
              hipMalloc(&b->cfl_acc, sizeof(unsigned long long) * (CFL_ACC_SLOTS + 1) * nbox) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        mhd_fail(MHD_ENOMEM, "device allocation of 2 x %zu bytes failed", bytes);
        mhd_batch_destroy(b);
        return nullptr;
    }
    ok = hipMemcpy(b->d_cfl_items, cfl_items.data(), sizeof(int2) * cfl_items.size(),
                   hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(b->d_item_first, first.data(), sizeof(int) * (nbox + 1),
                   hipMemcpyHostToDevice) == hipSuccess &&
         hipMemset(b->buf[0], 0, bytes) == hipSuccess && hipMemset(b->buf[1], 0, bytes) == hipSuccess &&
         hipMemset(b->scal, 0, sizeof(double) * SCAL_COUNT * nbox) == hipSuccess &&
         hipMemset(b->flag, 0, sizeof(int) * FLAG_COUNT * nbox) == hipSuccess &&
         hipMemset(b->cfl_acc, 0, sizeof(unsigned long long) * (CFL_ACC_SLOTS + 1) * nbox) == hipSuccess;
    b->acc_valid = false;
    if (!ok || build_lists(b) != MHD_OK) {
        mhd_fail(MHD_EDEVICE, "batch initialisation failed");
        mhd_batch_destroy(b);
        return nullptr;
    }
    return b;
}

static int check_batch(const mhd_batch* b)
{
    if (!b) return mhd_fail(MHD_EINVAL, "null batch handle");
    if (b->failed) return mhd_fail(MHD_ESTATE, "batch handle failed earlier (HIP error)");
    return MHD_OK;
}

extern "C" int mhd_batch_info(const mhd_batch* b, int* nbox, long long* ncell)
{
    if (!b) return mhd_fail(MHD_EINVAL, "null batch handle");
    long long n = 0;
    for (const BoxDesc& bd : b->boxes) n += bd.ncell;
    if (nbox) *nbox = b->nbox;
    if (ncell) *ncell = n;
    return MHD_OK;
}

template <typename T>
static T* box_field(mhd_batch* b, int box, int f, int which)
{
    const BoxDesc& bd = b->boxes[box];
    return reinterpret_cast<T*>(b->buf[which]) + bd.off + (size_t)f * bd.ncell;
}

extern "C" int mhd_batch_set_state(mhd_batch* b, int box, const double* host, size_t n)
{
    int r = check_batch(b);
    if (r) return r;
    if (box < 0 || box >= b->nbox) return mhd_fail(MHD_EINVAL, "box index %d out of range", box);
    if (!host) return mhd_fail(MHD_EINVAL, "null host pointer");
    const BoxDesc& bd = b->boxes[box];
    if (n != 8 * (size_t)bd.ncell) return mhd_fail(MHD_EINVAL, "state size %zu != 8 * cells of box", n);
    HIP_TRY(b, hipSetDevice(b->device));
    b->acc_valid = false;         // the fused CFL maxima describe the old state
    const size_t N = bd.ncell;
    // the fluid fields (0-4) and the face fields (5-7) each lie contiguously
    // in the buffer that holds them now
    const int bu = b->cur[0], bf = b->cur[5];
    if (b->prec == MHD_F64) {
        HIP_TRY(b, hipMemcpyAsync(box_field<double>(b, box, 0, bu), host, 5 * N * sizeof(double),
                                  hipMemcpyHostToDevice, b->stream));
        HIP_TRY(b, hipMemcpyAsync(box_field<double>(b, box, 5, bf), host + 5 * N, 3 * N * sizeof(double),
                                  hipMemcpyHostToDevice, b->stream));
    } else {
        double* stage = nullptr;
        if (hipMalloc(&stage, 8 * N * sizeof(double)) != hipSuccess) {
            (void)hipGetLastError();
            return mhd_fail(MHD_ENOMEM, "staging allocation failed");
        }
        hipError_t e = hipMemcpyAsync(stage, host, 8 * N * sizeof(double), hipMemcpyHostToDevice, b->stream);
        if (e == hipSuccess)
            e = launch_convert_in<float>(stage, box_field<float>(b, box, 0, bu), 5 * N, b->stream);
        if (e == hipSuccess)
            e = launch_convert_in<float>(stage + 5 * N, box_field<float>(b, box, 5, bf), 3 * N, b->stream);
        const hipError_t e2 = hipStreamSynchronize(b->stream);
        (void)hipFree(stage);
        HIP_TRY(b, e);
        HIP_TRY(b, e2);
    }
    // this box starts afresh: time 0, no record
    HIP_TRY(b, hipMemsetAsync(b->scal + (size_t)box * SCAL_COUNT, 0, sizeof(double) * SCAL_COUNT, b->stream));
    HIP_TRY(b, hipMemsetAsync(b->flag + (size_t)box * FLAG_COUNT, 0, sizeof(int) * FLAG_COUNT, b->stream));
    HIP_TRY(b, hipStreamSynchronize(b->stream));
    return MHD_OK;
}

extern "C" int mhd_batch_get_state(mhd_batch* b, int box, double* host, size_t n)
{
    int r = check_batch(b);
    if (r) return r;
    if (box < 0 || box >= b->nbox) return mhd_fail(MHD_EINVAL, "box index %d out of range", box);
    if (!host) return mhd_fail(MHD_EINVAL, "null host pointer");
    const BoxDesc& bd = b->boxes[box];
    if (n != 8 * (size_t)bd.ncell) return mhd_fail(MHD_EINVAL, "state size %zu != 8 * cells of box", n);
    HIP_TRY(b, hipSetDevice(b->device));
    const size_t N = bd.ncell;
    const int bu = b->cur[0], bf = b->cur[5];
    if (b->prec == MHD_F64) {
        HIP_TRY(b, hipMemcpyAsync(host, box_field<double>(b, box, 0, bu), 5 * N * sizeof(double),
                                  hipMemcpyDeviceToHost, b->stream));
        HIP_TRY(b, hipMemcpyAsync(host + 5 * N, box_field<double>(b, box, 5, bf), 3 * N * sizeof(double),
                                  hipMemcpyDeviceToHost, b->stream));
        HIP_TRY(b, hipStreamSynchronize(b->stream));
        return MHD_OK;
    }
    double* stage = nullptr;
    if (hipMalloc(&stage, 8 * N * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        return mhd_fail(MHD_ENOMEM, "staging allocation failed");
    }
    hipError_t e = launch_convert_out<float>(box_field<float>(b, box, 0, bu), stage, 5 * N, b->stream);
    if (e == hipSuccess) e = launch_convert_out<float>(box_field<float>(b, box, 5, bf), stage + 5 * N, 3 * N, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(host, stage, 8 * N * sizeof(double), hipMemcpyDeviceToHost, b->stream);
    const hipError_t e2 = hipStreamSynchronize(b->stream);
    (void)hipFree(stage);
    HIP_TRY(b, e);
    HIP_TRY(b, e2);
    return MHD_OK;
}

// reverse-half pairs in one launch each: asked for, or the built-in choice
// (FP32 with van Leer's or minmod, as for a single grid)
static bool batch_pairs_fused(const mhd_batch* b)
{
    return b->rev_mode == 1 ||
           (b->rev_mode == 0 && b->prec == MHD_F32 &&
            (b->limiter == MHD_LIMITER_VANLEER || b->limiter == MHD_LIMITER_MINMOD));
}

// the middle of a step M_z M_z F_z in one launch: with fused pairs, FP32 and
// van Leer's limiter, as for a single grid; built in from 128^3 cells per box
// on average
static bool batch_mid_fused(const mhd_batch* b)
{
    if (!batch_pairs_fused(b) || b->prec != MHD_F32 || b->limiter != MHD_LIMITER_VANLEER) return false;
    if (b->mid_mode == 0) {
        unsigned long long cells = 0;
        for (const BoxDesc& bd : b->boxes) cells += bd.ncell;
        return cells >= (unsigned long long)b->boxes.size() * 128ull * 128 * 128;
    }
    return b->mid_mode == 1;
}

template <typename T>
static int enqueue_batch_step(mhd_batch* b, double cfl)
{
    const T* base[8];
    for (int q = 0; q < 8; ++q) base[q] = reinterpret_cast<const T*>(b->buf[b->cur[q]]);
    if (b->acc_valid) {
        // the previous step's last launch found every box's maximum already
        HIP_TRY(b, launch_batch_cfl_from_acc(b->cfl_acc, b->d_boxes, b->nbox, cfl, b->scal, b->flag,
                                             b->stream));
    } else {
        HIP_TRY(b, launch_batch_cfl<T>(base, b->d_boxes, b->d_cfl_items, b->n_cfl_items,
                                       b->d_item_first, b->nbox, b->gamma, cfl, b->partial,
                                       b->partial_bad, b->scal, b->flag, b->stream));
        HIP_TRY(b, launch_batch_clear_acc(b->cfl_acc, b->nbox, b->stream));
    }
    b->acc_valid = false;
    // (op, d): op 0 fluid, 1 magnetic, 2 the reverse-half pair in one launch
    static const int separate[12][2] = { { 0, 0 }, { 1, 0 }, { 0, 1 }, { 1, 1 }, { 0, 2 }, { 1, 2 },
                                         { 1, 2 }, { 0, 2 }, { 1, 1 }, { 0, 1 }, { 1, 0 }, { 0, 0 } };
    static const int fused[9][2] = { { 0, 0 }, { 1, 0 }, { 0, 1 }, { 1, 1 }, { 0, 2 }, { 1, 2 },
                                     { 2, 2 }, { 2, 1 }, { 2, 0 } };
    // op 3: the middle M_z M_z F_z in one launch
    static const int middle[8][2] = { { 0, 0 }, { 1, 0 }, { 0, 1 }, { 1, 1 }, { 0, 2 }, { 3, 2 }, { 2, 1 }, { 2, 0 } };
    const bool fz = batch_pairs_fused(b), mid = fz && batch_mid_fused(b);
    const int nops = mid ? 8 : fz ? 9 : 12;
    for (int k = 0; k < nops; ++k) {
        const int op = mid ? middle[k][0] : fz ? fused[k][0] : separate[k][0];
        const int d = mid ? middle[k][1] : fz ? fused[k][1] : separate[k][1];
        BatchParams<T> P;
        for (int q = 0; q < 8; ++q) {
            P.in_base[q] = reinterpret_cast<const T*>(b->buf[b->cur[q]]);
            P.out_base[q] = reinterpret_cast<T*>(b->buf[1 - b->cur[q]]);
        }
        P.boxes = b->d_boxes;
        // the fused pairs along y and z (and the middle) have work lists of
        // their own chunks
        const bool pl = (op == 2 || op == 3) && d > 0;
        P.items = pl ? b->d_pitems[d] : b->d_items[d];
        P.nitems = pl ? b->npitems[d] : b->nitems[d];
        P.gamma = (T)b->gamma;
        P.scal = b->scal;
        P.flag = b->flag;
        P.offsets32 = !b->wide;
        P.limiter = b->limiter;
        // the last launch (F_x or the x pair) also finds the next step's CFL
        P.cfl_acc = k == nops - 1 ? b->cfl_acc : nullptr;
        P.gamma64 = b->gamma;
        for (const BoxDesc& bd : b->boxes)
            if ((unsigned long long)bd.ncell * (b->prec == MHD_F64 ? 8 : 4) > (1ull << 32)) P.offsets32 = false;
        const int grid = std::max(8, std::min(b->grid[d], (P.nitems + 7) / 8 * 8));
        HIP_TRY(b, launch_batch_op<T>(P, op, d, grid, b->stream));
        if (op != 1)
            for (int q = 0; q < 5; ++q) b->cur[q] = 1 - b->cur[q];
        if (op != 0)
            for (int q = 5; q < 8; ++q) b->cur[q] = 1 - b->cur[q];
    }
    HIP_TRY(b, launch_batch_advance(b->scal, b->flag, b->nbox, b->stream));
    b->acc_valid = true;
    return MHD_OK;
}

static int enqueue_step(mhd_batch* b, double cfl)
{
    return b->prec == MHD_F64 ? enqueue_batch_step<double>(b, cfl) : enqueue_batch_step<float>(b, cfl);
}

extern "C" int mhd_batch_step_auto(mhd_batch* b, double cfl)
{
    int r = check_batch(b);
    if (r) return r;
    if (!(cfl > 0.0) || !isfinite(cfl)) return mhd_fail(MHD_EINVAL, "cfl must be > 0");
    HIP_TRY(b, hipSetDevice(b->device));
    return enqueue_step(b, cfl);
}

extern "C" int mhd_batch_run(mhd_batch* b, double cfl, int nsteps, int use_graph)
{
    int r = check_batch(b);
    if (r) return r;
    if (!(cfl > 0.0) || !isfinite(cfl)) return mhd_fail(MHD_EINVAL, "cfl must be > 0");
    if (nsteps < 0) return mhd_fail(MHD_EINVAL, "nsteps must be >= 0");
    HIP_TRY(b, hipSetDevice(b->device));
    if (!use_graph) {
        for (int s = 0; s < nsteps; ++s)
            if ((r = enqueue_step(b, cfl))) return r;
        return MHD_OK;
    }
    // the captured step takes its CFL from the maxima the previous step left:
    // a step without them (after a new state) runs eagerly first
    if (!b->acc_valid && nsteps > 0) {
        if ((r = enqueue_step(b, cfl))) return r;
        --nsteps;
    }
    if (nsteps == 0) return MHD_OK;
    // with the fused middle a step moves the face fields to the other
    // buffer: the graph holds two steps and starts from one buffer of them
    const int gs = batch_mid_fused(b) ? 2 : 1;
    if (b->graph_valid && (b->graph_cfl != cfl || b->graph_steps != gs)) drop_graph(b);
    if (gs == 2 && b->graph_valid && b->cur[5] != b->graph_bpar) {
        if ((r = enqueue_step(b, cfl))) return r;
        if (--nsteps == 0) return MHD_OK;
    }
    if (!b->graph_valid) {
        const int bpar = b->cur[5];
        HIP_TRY(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        r = enqueue_step(b, cfl);
        if (!r && gs == 2) r = enqueue_step(b, cfl);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(b->stream, &g);
        if (r) {
            if (g) (void)hipGraphDestroy(g);
            return r;
        }
        HIP_TRY(b, e);
        b->graph = g;
        HIP_TRY(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
        b->graph_cfl = cfl;
        b->graph_steps = gs;
        b->graph_bpar = bpar;
        b->graph_valid = true;
    }
    for (; nsteps >= gs; nsteps -= gs) HIP_TRY(b, hipGraphLaunch(b->exec, b->stream));
    if (nsteps > 0 && (r = enqueue_step(b, cfl))) return r;       // the odd last step
    return MHD_OK;
}

// steps[b] (if not null) = steps box b completed; nonphys[b] (if not null) =
// its record (0 none, 1 non-physical, 2 zero signal speed).  Returns
// MHD_ENONPHYS if any box has a record; records are then cleared.
extern "C" int mhd_batch_status(mhd_batch* b, long long* steps, int* nonphys)
{
    int r = check_batch(b);
    if (r) return r;
    HIP_TRY(b, hipSetDevice(b->device));
    std::vector<int> fl((size_t)FLAG_COUNT * b->nbox);
    HIP_TRY(b, hipMemcpyAsync(fl.data(), b->flag, sizeof(int) * fl.size(), hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(b, hipStreamSynchronize(b->stream));
    int any = 0;
    for (int i = 0; i < b->nbox; ++i) {
        if (steps) steps[i] = fl[(size_t)i * FLAG_COUNT + FLAG_STEPS];
        const int np = fl[(size_t)i * FLAG_COUNT + FLAG_NONPHYS];
        if (nonphys) nonphys[i] = np;
        if (np) {
            any = 1;
            HIP_TRY(b, hipMemsetAsync(b->flag + (size_t)i * FLAG_COUNT + FLAG_NONPHYS, 0, sizeof(int), b->stream));
        }
    }
    HIP_TRY(b, hipStreamSynchronize(b->stream));
    if (any) return mhd_fail(MHD_ENONPHYS, "a box reached a non-physical state; its steps were skipped");
    return MHD_OK;
}

extern "C" int mhd_batch_time(mhd_batch* b, double* times)
{
    int r = check_batch(b);
    if (r) return r;
    if (!times) return mhd_fail(MHD_EINVAL, "null output");
    HIP_TRY(b, hipSetDevice(b->device));
    std::vector<double> sc((size_t)SCAL_COUNT * b->nbox);
    HIP_TRY(b, hipMemcpyAsync(sc.data(), b->scal, sizeof(double) * sc.size(), hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(b, hipStreamSynchronize(b->stream));
    for (int i = 0; i < b->nbox; ++i) times[i] = sc[(size_t)i * SCAL_COUNT + SCAL_TIME];
    return MHD_OK;
}

extern "C" int mhd_batch_set_launch(mhd_batch* b, int key, int value)
{
    int r = check_batch(b);
    if (r) return r;
    HIP_TRY(b, hipSetDevice(b->device));
    HIP_TRY(b, hipStreamSynchronize(b->stream));
    if (key == MHD_BATCH_GRID_X || key == MHD_BATCH_GRID_Y || key == MHD_BATCH_GRID_Z) {
        if (value < 8 || value % 8) return mhd_fail(MHD_EINVAL, "persistent grid must be a positive multiple of 8");
        b->grid[key - MHD_BATCH_GRID_X] = value;
        drop_graph(b);
        return MHD_OK;
    }
    if (key == MHD_BATCH_CHUNK || key == MHD_BATCH_PAIR_CHUNK) {
        if (value < 8) return mhd_fail(MHD_EINVAL, "chunk target must be >= 8");
        (key == MHD_BATCH_CHUNK ? b->chunk_target : b->pair_chunk_target) = value;
        return build_lists(b);
    }
    if (key == MHD_BATCH_WIDE_OFFSETS) {
        if (value < 0 || value > 1) return mhd_fail(MHD_EINVAL, "wide-offset switch must be 0 or 1 (got %d)", value);
        b->wide = value == 1;
        drop_graph(b);
        return MHD_OK;
    }
    if (key == MHD_BATCH_REVERSE) {
        if (value < 0 || value > 2)
            return mhd_fail(MHD_EINVAL, "reverse-half choice must be 0, 1 or 2 (got %d)", value);
        b->rev_mode = value;
        drop_graph(b);
        return MHD_OK;
    }
    if (key == MHD_BATCH_MIDDLE) {
        if (value < 0 || value > 2)
            return mhd_fail(MHD_EINVAL, "middle-of-step choice must be 0, 1 or 2 (got %d)", value);
        b->mid_mode = value;
        drop_graph(b);
        return MHD_OK;
    }
    return mhd_fail(MHD_EINVAL, "unknown launch key %d", key);
}

extern "C" int mhd_batch_set_limiter(mhd_batch* b, int limiter)
{
    int r = check_batch(b);
    if (r) return r;
    if (limiter < MHD_LIMITER_VANLEER || limiter > MHD_LIMITER_SUPERBEE)
        return mhd_fail(MHD_EINVAL, "limiter must be 0..3 (got %d)", limiter);
    HIP_TRY(b, hipSetDevice(b->device));
    HIP_TRY(b, hipStreamSynchronize(b->stream));
    b->limiter = limiter;
    drop_graph(b);          // a captured step holds the kernels of the old limiter
    return MHD_OK;
}

extern "C" int mhd_batch_get_limiter(const mhd_batch* b, int* limiter)
{
    if (!b || !limiter) return mhd_fail(MHD_EINVAL, "null argument");
    *limiter = b->limiter;
    return MHD_OK;
}

extern "C" int mhd_batch_get_launch(const mhd_batch* b, int key, int* value)
{
    if (!b || !value) return mhd_fail(MHD_EINVAL, "null argument");
    if (key == MHD_BATCH_GRID_X || key == MHD_BATCH_GRID_Y || key == MHD_BATCH_GRID_Z)
        *value = b->grid[key - MHD_BATCH_GRID_X];
    else if (key == MHD_BATCH_CHUNK)
        *value = b->chunk_target;
    else if (key == MHD_BATCH_PAIR_CHUNK)
        *value = b->pair_chunk_target;
    else if (key == MHD_BATCH_REVERSE)
        *value = batch_pairs_fused(b) ? 1 : 2;
    else if (key == MHD_BATCH_WIDE_OFFSETS)
        *value = b->wide ? 1 : 0;
    else if (key == MHD_BATCH_MIDDLE)
        *value = batch_mid_fused(b) ? 1 : 2;
    else
        return mhd_fail(MHD_EINVAL, "unknown launch key %d", key);
    return MHD_OK;
}
