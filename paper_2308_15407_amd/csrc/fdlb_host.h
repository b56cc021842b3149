// fdlb_host.h -- host-side structures of the FDLB solver (not part of the C ABI).
#pragma once
#include <string>
#include <vector>

#include "../../include/fdlb.h"
#include "fdlb_common.h"

namespace fdlb {

// Host copy of one case: parameters, lattice constants, grid and wall tables.
struct CaseHost {
  fdlb_params p;
  int nx, qh, qy, qz, K;
  int nxp;                          // slots per population row (fslots(nx))
  double sigma, R, Lc, chi0, deta, dt;
  LatOff lo;
  std::vector<double> lat;          // lattice constants (see LatOff)
  std::vector<double> wx, wy, wz;   // 1D weights
  std::vector<double> x, jac, invdx;
  std::vector<double> gw[2];        // wall Maxwellians (n = 1) [K]
  double wallD[2];
  int kxc, nchunk;                  // kx per velocity chunk, number of chunks
  size_t ws_off[32];                // workspace offsets of this case's arrays
  int prec;                         // active storage precision
  bool wide;                        // x tables on the NB_WIDE base rule (qx_half > MAXQH or full-range x)
  bool active;
  long steps;
  double last_resid;
};

int validate(const fdlb_params &p, std::string &why, double *sigma, double *R);
// records msg as the library's last error and returns code
int api_fail(int code, const std::string &msg);
int build_case(const fdlb_params &p, CaseHost &c, std::string &why);

// table-pass mode bits
enum {
  TM_PARTIALS = 1,  // moments from the partial raw sums
  TM_FIELDS = 2,    // moments from the staged Grad-13 fields (initial state)
  TM_WRITE_MOM = 4, // store the moments of owned cells
  TM_RESID = 8,     // residual against the stored moments
  TM_TABLES = 16,   // projection tables for the update pass
  TM_WALLS = 32     // wall densities (wall blocks)
};

// kernel launchers (fdlb_kernels.hip); map arrays are int4 {case, tile, chunk, 0}
// e0/e1 (optional): events recorded at the kernel's own start and end (timing)
// reduced models: nsteps TVD-RK3 steps of every case, launched per group of
// cases (at most 256 rows, more than 256), each with its own map (int2
// {case, tile} per block of `tile` = r1_tile(rmax, group cells) cells) and
// rmax, the largest row count of its cases; dim: 1 or 2, the same for every
// case; and the moments of case c into its mom array
struct R1Group {
  const int *map;
  int nblocks, rmax, tile;
};
int r1_tile(int rmax, int total_cells);
// (map_n: int2 {case, tile} per NBAR_TILE cells of the chi_mode 1 cases, with
// lds_n the bytes of the largest window of a tile; nblocks_n = 0 if none)
hipError_t launch_r1_step(const R1Dev *cases, const R1Group *groups, int ngroups, int dim, const int *map_n,
                          int nblocks_n, size_t lds_n, long nsteps, hipStream_t s);
hipError_t launch_r1_moments(const R1Dev *cases, int c, int nx, hipStream_t s);
// wide: the map may hold cases with qx_half > MAXQH (adds the wide pass);
// tile: the cells per block the map was built with (CTILE or CTILE_SMALL)
hipError_t launch_table(int prec, const CaseDev *cases, const int *map, int nblocks, int mode, int gin,
                        bool wide, int tile, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// averaged density of the revised Enskog contact value (chi_mode 1 cases):
// one block per NBAR_TILE cells; lds = bytes of the largest window of a tile
constexpr int NBAR_TILE = 16;
constexpr size_t NBAR_LDS_MAX = 65536;
hipError_t launch_nbar(int prec, const CaseDev *cases, const int *map, int nblocks, size_t lds, hipStream_t s);
// dynamic LDS of an update launch: partial sums of the waves, or the staged
// projection tables of a tile when tlds (at most UPDATE_LDS_MAX bytes)
constexpr size_t UPDATE_LDS_MAX = 65536;
// fewest velocity rows per wave for which an update block stages its tables in LDS
#ifndef FDLB_TLDS_MIN_ROWS
#define FDLB_TLDS_MIN_ROWS 8
#endif
constexpr int TLDS_MIN_ROWS = FDLB_TLDS_MIN_ROWS;
size_t update_lds_bytes(int prec, int qyz, int kxc, int waves, bool tlds);
// force: 0 force-free; otherwise the largest Q_y of the launch's (body-force)
// cases, which selects the kernel instance (Q_y <= 4 or <= 8)
hipError_t launch_update(int prec, int stage, const CaseDev *cases, const int *map, int nblocks, int waves,
                         int force, size_t lds, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_fill(int prec, const CaseDev *cases, const int *map, int nblocks, int waves, int use_noise,
                       hipStream_t s);
hipError_t launch_partials(int prec, const CaseDev *cases, const int *map, int nblocks, int waves,
                           hipStream_t s);
hipError_t launch_zero_resid(const CaseDev *cases, int ncases, hipStream_t s);
hipError_t launch_convert(int dir, const void *src, void *dst, size_t n, hipStream_t s);
hipError_t launch_copy_probe(const void *src, void *dst, size_t bytes, hipStream_t s);
hipError_t launch_scale(void *x, double a, size_t n, hipStream_t s);
// FP32 deviation storage of case c -> FP64 populations (adds the background)
hipError_t launch_promote(const CaseDev *cases, int c, size_t n, hipStream_t s);

}  // namespace fdlb
