// lgf_ensemble.hpp -- device-visible descriptors of the ensemble work list and
// the launchers of the persistent ensemble kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "lgf_device.hpp"

namespace lgf {

constexpr int kEnsTile = 128;     // default sites per tile (one workgroup of one lane per site)
constexpr int kEnsMinTile = 64;   // smallest tile width (sizes the work-list buffers)
constexpr int kEnsMaxTile = 256;  // largest tile width (the kernels' launch bound)

struct EnsCfg {         // one configuration as the kernels see it
    Geom g;
    void *field;        // links in the current storage format
    void *gf;           // fixed-link form: the gauge transformation (site field, same format), else NULL
    const void *rec;    // fixed-link form: the links' per-site records (launch_record_links), else NULL
    int fmt;            // current storage format
    uint32_t instance;  // the configuration's index: third word of the SR counter
};

// lanes per site of the fixed-link ensemble kernels: a tile of `tile` lanes
// covers tile / kEnsFixedLanes sites
constexpr int kEnsFixedLanes = 2;

struct EnsTile {        // `tile` consecutive half indices of one configuration
    uint32_t cfg;
    uint32_t h0;
};

struct EnsSpan {        // the tiles [first, first + count) of configuration cfg
    uint32_t cfg;
    uint32_t first;
    uint32_t count;
    double V;
};

struct EnsRelax {       // relaxation parameters shared by the whole launch
    double omega;
    int overrelax;
    uint64_t sr_threshold;
    uint32_t key0, key1;
};

struct EnsLaunch {      // device pointers of one ensemble's work list
    const EnsCfg *cfgs;
    const EnsTile *tiles;
    const uint32_t *n_tiles;
    const uint64_t *sweep_base;
    uint32_t grid;      // persistent workgroups
    uint32_t tile;      // sites per tile = lanes per workgroup (64, 128 or 256)
};

// meas (optional): the fused reunitarization + measurement, its per-tile
// partial sums written to the second-pass slots of the measurement layout
hipError_t launch_ensemble_sweep(int fa, int fb, const EnsLaunch &L, int parity, const EnsRelax &r,
                                 uint32_t sweep_offset, bool sr, bool nt, hipStream_t s, double *meas = nullptr);
hipError_t launch_ensemble_measure(int fa, int fb, const EnsLaunch &L, uint32_t n_tiles, int parity,
                                   bool reunit_fwd, bool reunit_bwd, double *partials, hipStream_t s);
hipError_t launch_ensemble_finish(const double *partials, uint32_t n_tiles, const EnsSpan *spans,
                                  uint32_t n_spans, double *out, hipStream_t s);
// workgroups of `tile` lanes that fill every CU for the sweep kernel of a
// format pair, times grid_mult
int ensemble_persistent_grid(int fa, int fb, bool sr, bool nt, int tile, int grid_mult);

// The fixed-link form of the persistent sweep (links read only, cfgs[].gf
// updated; post as launch_fixed_sweep: 0 plain, 1 g reunitarized as stored,
// 2 also the per-tile (F, theta) sums in the second-pass slots of meas) and
// its read-only measurement pass (one workgroup per listed tile).  Format
// pairs: ensemble_fixed_pair.  rec: every listed configuration reads its
// links from cfgs[].rec (pairs of ensemble_fixed_records_pair only).
bool ensemble_fixed_pair(int fa, int fb);
bool ensemble_fixed_records_pair(int fa, int fb);
hipError_t launch_ensemble_fixed_sweep(int fa, int fb, const EnsLaunch &L, int parity, const EnsRelax &r,
                                       uint32_t sweep_offset, bool sr, int post, double *meas, hipStream_t s,
                                       bool rec);
hipError_t launch_ensemble_fixed_measure(int fa, int fb, const EnsLaunch &L, uint32_t n_tiles, int parity,
                                         double *partials, hipStream_t s, bool rec);
int ensemble_fixed_grid(int fa, int fb, bool sr, int tile, int grid_mult, bool rec);
// *p = v, as a one-lane kernel on the stream (safe inside a captured graph)
hipError_t launch_set_u64(uint64_t *p, uint64_t v, hipStream_t s);

}  // namespace lgf
