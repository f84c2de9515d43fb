/* Host-only stand-in for the HIP runtime, for CPU tests of the library's
 * host logic (argument checks, planning, job and busy bookkeeping, byte
 * accounting): "device" memory is host memory, copies are memmove, kernel
 * launches and events do nothing.  No numerical result is meaningful under
 * it.  Exports the runtime symbols the library imports, versioned hip_4.2
 * (graphs and stream capture hip_4.3, the stream-ordered allocator hip_5.1,
 * the device properties hip_6.0). */
#include <stdlib.h>
#include <string.h>
#include <stddef.h>
typedef int hipError_t;
typedef struct { unsigned x, y, z; } dim3;
static char dummy[64];
hipError_t hipMalloc(void **p, size_t n) { *p = calloc(1, n ? n : 1); return *p ? 0 : 2; }
hipError_t hipFree(void *p) { free(p); return 0; }
hipError_t hipMallocAsync(void **p, size_t n, void *st) { return hipMalloc(p, n); }
hipError_t hipFreeAsync(void *p, void *st) { free(p); return 0; }
hipError_t hipDeviceGetDefaultMemPool(void **pool, int dev) { *pool = (void *)dummy; return 0; }
hipError_t hipMemPoolSetAttribute(void *pool, int attr, void *value) { return 0; }
hipError_t hipMemcpy(void *d, const void *s, size_t n, int k) { memmove(d, s, n); return 0; }
hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, int k, void *st) { memmove(d, s, n); return 0; }
hipError_t hipMemsetAsync(void *d, int v, size_t n, void *st) { memset(d, v, n); return 0; }
hipError_t hipStreamSynchronize(void *s) { return 0; }
hipError_t hipGetLastError(void) { return 0; }
hipError_t hipSetDevice(int d) { return 0; }
hipError_t hipGetDevice(int *d) { *d = 0; return 0; }
/* a __device__ variable's host shadow has the variable's size: use it */
hipError_t hipGetSymbolAddress(void **p, const void *sym) { *p = (void *)sym; return 0; }
void __hipRegisterVar(void **m, void *var, char *hv, const char *dv, int ext, size_t size, int constant,
                      int global) {}
hipError_t hipFuncSetAttribute(const void *f, int a, int v) { return 0; }
const char *hipGetErrorString(hipError_t e) { return "stub"; }
hipError_t hipLaunchKernel(const void *f, dim3 g, dim3 b, void **a, size_t sh, void *st) { return 0; }
hipError_t __hipPushCallConfiguration(dim3 g, dim3 b, size_t sh, void *st) { return 0; }
hipError_t __hipPopCallConfiguration(dim3 *g, dim3 *b, size_t *sh, void **st) {
  g->x = g->y = g->z = 1; b->x = b->y = b->z = 1; *sh = 0; *st = 0; return 0; }
void **__hipRegisterFatBinary(const void *d) { return (void **)dummy; }
void __hipRegisterFunction(void **m, const void *hf, char *df, const char *dn, int t, void *a, void *b, void *c, void *d, int *e) {}
void __hipUnregisterFatBinary(void **m) {}
hipError_t hipEventCreateWithFlags(void **e, unsigned f) { *e = (void *)dummy; return 0; }
hipError_t hipEventRecord(void *e, void *s) { return 0; }
hipError_t hipEventQuery(void *e) { return 0; }
hipError_t hipEventSynchronize(void *e) { return 0; }
hipError_t hipEventDestroy(void *e) { return 0; }
hipError_t hipEventCreate(void **e) { *e = (void *)dummy; return 0; }
hipError_t hipStreamCreateWithFlags(void **s, unsigned f) { *s = (void *)dummy; return 0; }
hipError_t hipStreamDestroy(void *s) { return 0; }
hipError_t hipStreamBeginCapture(void *s, int mode) { return 0; }
hipError_t hipStreamEndCapture(void *s, void **g) { *g = (void *)dummy; return 0; }
hipError_t hipGraphInstantiate(void **x, void *g, void *node, char *log, size_t n) { *x = (void *)dummy; return 0; }
hipError_t hipGraphLaunch(void *x, void *s) { return 0; }
hipError_t hipGraphExecDestroy(void *x) { return 0; }
hipError_t hipGraphDestroy(void *g) { return 0; }
hipError_t hipEventElapsedTime(float *ms, void *a, void *b) { *ms = 1.0f; return 0; }
/* the properties structure (1472 bytes in this runtime) is only written */
hipError_t hipGetDevicePropertiesR0600(void *prop, int dev) { memset(prop, 0, 1472); return 0; }
