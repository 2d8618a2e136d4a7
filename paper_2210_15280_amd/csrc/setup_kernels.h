// Launchers of the setup kernels.
#pragma once

#include "ctx.h"

namespace ilu {

struct QrJob {
    int64_t in_off;   // level 0: offset of the samples; later levels: row offset in the input
    int64_t in_rows;  // rows of this problem at this level
    int64_t out_off;  // row offset of this problem's R factors in the output
    int32_t tet, fit; // problem = (tetrahedron, fitted direction)
    int64_t run_rows; // rows per run
    int32_t chunk0;   // first global run id of this problem
    int32_t nchunk;   // runs of this problem
};

void launch_assemble(const Ctx& c, double* A8, double* Afull, hipStream_t st);
void launch_factor_plane(const Ctx& c, int t, double* Lf, double* Df, int* flags, hipStream_t st);
// Alg. 1 for hyperplane t into a ring of four hyperplanes (ring: [8][4][nring]
// FP64, nring = lanes + 1, zeroed once), with the samples (may be null) and,
// variant V1, the boundary records F (FP32 if f32, may be null) of the points
// factored.  With c.A8 null the stencil rows are computed on the fly and their
// samples written to asamples (may be null).
void launch_factor_ring(const Ctx& c, int t, double* ring, int64_t nring, double* samples, double* asamples,
                        void* F, bool f32, int* flags, hipStream_t st);
void launch_transpose(const Ctx& c, const double* Lf, const double* Df, double* Lb, hipStream_t st);
// One TSQR level: every run of QrJob.run_rows rows of a problem (level 0: the
// samples, later levels: the stacked R factors in `in`) is reduced to its
// m x m triangular factor, written to `out` at row J.out_off + run * m;
// QrJob.nchunk counts the runs, m <= 512
void launch_qr_stream(const Ctx& c, const QrJob* jobs, int njobs, int level0, int m, const double* samples,
                      const double* in, double* out, int grid, int nruns, hipStream_t st);
void launch_qr_solve(const QrJob* jobs, int njobs, int m, const double* R, double* coef, int* flags, hipStream_t st);
void launch_row_tables(const Ctx& c, int nslots, const double* coef, int NC, double* tab, float* tab32, hipStream_t st);
// variant V1: backward weights of set B from F and the FP64 row tables
void launch_build_v1b(const Ctx& c, const double* tab, const void* F, void* Bw, bool f32, hipStream_t st);
// mode 0: stream -> lexicographic, mode 1: lexicographic -> stream
void launch_permute(const Ctx& c, int mode, int count, const double* src, double* dst, int64_t sstride, int lmul,
                    int only_tet, hipStream_t st);
// x and b (interface order, all tetrahedra) into the stream layout xs and bs, one launch
void launch_permute_in2(const Ctx& c, const double* x, double* xs, const double* b, double* bs, hipStream_t st);


}  // namespace ilu
