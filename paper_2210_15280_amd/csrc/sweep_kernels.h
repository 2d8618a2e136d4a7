// Launchers of the per-sweep kernels.
#pragma once

#include "ctx.h"

namespace ilu {

void launch_residual(const Ctx& c, const double* x, const double* b, void* r, bool f32, int subtract, double* partial,
                     hipStream_t st);
// r = b - A x (assembled A) as tagged entries (XEnt words, tag *tagp) for a
// forward sweep consuming them while this kernel runs; res_tag_partials
// partial sums of ||r||^2
int64_t res_tag_partials(const Ctx& c);
void launch_residual_tagged(const Ctx& c, const double* x, const double* b, uint64_t* rt, bool f32,
                            const int32_t* tagp, uint64_t* rflag, double* partial, hipStream_t st);
void launch_sumsq(const Ctx& c, const double* v, double* partial, hipStream_t st);
// number of partial sums the residual and norm kernels write
int64_t res_partials(const Ctx& c);
void launch_reduce(const double* partial, int64_t count, double* out, int slot, hipStream_t st);
void launch_fwd_plane(const Ctx& c, int variant, int t, hipStream_t st);
void launch_bwd_plane(const Ctx& c, int variant, int t, double* x, hipStream_t st);
// surrogate weights of one tetrahedron in lexicographic order: L_out [N][7], Dinv_out [N]
void launch_export_surrogate(const Ctx& c, bool f32, int tet, double* L_out, double* Dinv_out, hipStream_t st);

// persistent dataflow schedule (dataflow_kernels.hip)
struct Flow {
    const int32_t* order_fwd = nullptr;  // block ids in a topological order of the forward sweep
    const int32_t* order_bwd = nullptr;  // ... and of the backward sweep
    uint64_t* xch = nullptr;             // tagged boundary values of every block and hyperplane
    int32_t* ticket = nullptr;           // [4] work counters (fwd, bwd) and the launch tag
    int32_t* flags = nullptr;            // [4] error flags (flags[2]: wait limit hit)
    int grid = 0;                        // resident workgroups
    // overlapped residual (forward sweep only; null: read the plain residual
    // stream): tagged residual entries and the x, b streams to compute a
    // missing one from
    const uint64_t* rt = nullptr;
    const double* xo = nullptr;
    const double* bo = nullptr;
    int rspin = 0;                       // polls of a missing entry before computing it
    const uint64_t* rflag = nullptr;     // per (block, 64-lane group, band): the tag once the residual kernel
    int nbands = 0;                      // finished that band (bands of RES_T absolute hyperplanes)
};
void launch_flow_reset(const Flow& f, hipStream_t st);
void launch_fwd_flow(const Ctx& c, const Flow& f, int variant, hipStream_t st);
void launch_bwd_flow(const Ctx& c, const Flow& f, int variant, double* x, hipStream_t st);
int flow_max_resident(int variant, int NC, bool v1, int bv, int bw);
bool flow_shape_supported(int bv, int bw);

}  // namespace ilu
