// lbsq_noalloc.hip -- lb_read_fields_noalloc: the field readout of
// lb_read_fields for callers that cannot allocate device memory.
//
// The FP64 fields pass through one fixed device array per GPU, `scratch`,
// in chunks of NOALLOC_CHUNK cells: rho[chunk] | u[3][chunk] | owner[chunk].
// The array is a file-scope __device__ variable, so each GPU the library
// runs on holds its own copy until the process ends.  Host code never
// passes the array's name to a kernel or a copy (in host code that name is
// a host-side stand-in, not a device address): the device address is looked
// up once per device with hipGetSymbolAddress, with that device current, and
// kept in g_scratch[device].
#include <mutex>

#include "lbsq_sim.h"

using namespace lbsq;

namespace {

constexpr size_t NOALLOC_BYTES = size_t(16) << 20;  // 16 MiB per GPU
constexpr size_t CELL_BYTES = sizeof(double) * 4 + 1;
// cells per chunk: whole blocks of 256 that fit the array
constexpr uint32_t NOALLOC_CHUNK = uint32_t(NOALLOC_BYTES / CELL_BYTES / 256 * 256);
static_assert(size_t(NOALLOC_CHUNK) * CELL_BYTES <= NOALLOC_BYTES, "chunk exceeds the scratch array");

constexpr int MAX_DEVICES = 64;
std::mutex g_lock[MAX_DEVICES];  // one call at a time per GPU within the process
void *g_scratch[MAX_DEVICES];     // device address of scratch on each GPU

}  // namespace

static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

int lbsq_noalloc_init(int device)
{
    if (device < 0 || device >= MAX_DEVICES) return LB_EDEVICE;
    std::lock_guard<std::mutex> lk(g_lock[device]);
    if (g_scratch[device]) return LB_OK;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != device) return LB_EDEVICE;
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return LB_EDEVICE;
    g_scratch[device] = p;
    return LB_OK;
}

extern "C" int lb_read_fields_noalloc(lb_sim *s, double *rho, double *u, uint8_t *owner)
{
    if (!s || !rho || !u) return LB_EINVAL;
    const TraceRange tr("lb_read_fields_noalloc");
    if (hipSetDevice(s->device) != hipSuccess) return LB_EDEVICE;
    int rc = lbsq_noalloc_init(s->device);
    if (rc != LB_OK) return rc;
    rc = lbsq_sync_check(s);
    if (rc != LB_OK) return rc;
    // the array is shared by every call on this GPU: calls are serialised,
    // and each returns only after its last copy out of the array has ended
    std::lock_guard<std::mutex> lk(g_lock[s->device]);
    unsigned char *base = static_cast<unsigned char *>(g_scratch[s->device]);
    double *d_rho = reinterpret_cast<double *>(base);
    double *d_u = d_rho + NOALLOC_CHUNK;
    uint8_t *d_o = reinterpret_cast<uint8_t *>(d_u + 3 * size_t(NOALLOC_CHUNK));
    const uint32_t n = s->args.box.n;
    const void *A = lbsq_pop_buf(s);
    const int lay = lbsq_pop_lay(s);
    // every slot a chunk copies out is written by that chunk's kernel first,
    // so nothing left from an earlier call is read and nothing needs clearing
    for (uint32_t c0 = 0; c0 < n && rc == LB_OK; c0 += NOALLOC_CHUNK) {
        const uint32_t cnt = n - c0 < NOALLOC_CHUNK ? n - c0 : NOALLOC_CHUNK;
        if (launch_fields(s->p.storage, s->args, A, s->own[s->cur], lay, c0, cnt, d_rho, d_u, d_o, s->stream) !=
            hipSuccess) {
            rc = LB_EDEVICE;
            break;
        }
        hipError_t e = hipMemcpyAsync(rho + c0, d_rho, size_t(cnt) * sizeof(double), hipMemcpyDeviceToHost,
                                      s->stream);
        for (int k = 0; k < 3 && e == hipSuccess; ++k)
            e = hipMemcpyAsync(u + size_t(k) * n + c0, d_u + size_t(k) * cnt, size_t(cnt) * sizeof(double),
                               hipMemcpyDeviceToHost, s->stream);
        if (e == hipSuccess && owner) e = hipMemcpyAsync(owner + c0, d_o, cnt, hipMemcpyDeviceToHost, s->stream);
        // the next chunk's kernel reuses the array: it waits for these copies
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) rc = LB_EDEVICE;
    }
    return rc;
}
