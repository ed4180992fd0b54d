// Kernel launch interfaces shared between the HIP sources.
#pragma once

#include "wcl_internal.h"

enum { DS_PLAIN = 0, DS_AXPY = 1, DS_DOT = 2 };

struct DslashArgs {
    Geom g;
    const void* gauge;
    const void* clover;
    const void* in;
    void* out;
    const void* y;       // DS_AXPY source
    const void* a;       // DS_DOT left vector
    size_t in_stride, out_stride, y_stride, a_stride;  // bytes per rhs
    double kappa, csw;
    int nrhs;
    double* partial;     // DS_DOT: [nrhs][tiles][3]
};

int launch_pack_spinor(const Geom& g, int prec, int nrhs, const double* aos, void* soa, size_t stride,
                       hipStream_t st);
int launch_unpack_spinor(const Geom& g, int prec, int nrhs, const void* soa, size_t stride, double* aos,
                         hipStream_t st);
int launch_pack_gauge(const Geom& g, const double* aos, void* g64, void* g32, void* g16, hipStream_t st);
int launch_clover_build(const Geom& g, const void* g64, void* c64, void* c32, void* c16, hipStream_t st);
int launch_pack_clover(const Geom& g, const double* host_dev, void* c64, void* c32, void* c16, hipStream_t st);
int launch_unpack_clover(const Geom& g, const void* c64, double* host_dev, hipStream_t st);

int dslash_partials_per_rhs(int V);
int launch_dslash(const DslashArgs& a, int gp, int spi, int spo, int epi, int spy, hipStream_t st);
