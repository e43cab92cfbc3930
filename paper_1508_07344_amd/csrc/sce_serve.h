// Internal declarations of the batched serving path: many independent small
// simulations advanced together, one launch per phase of the step for all of
// them.  Shared by the batched kernels (kernels_serve.hip) and the server
// runtime (sce_server.hip).
//
// Per-request state lives in one device arena at byte offsets held in the
// request's descriptor; every kernel finds its request through a work item
// (slot, index) and the descriptor table.  Each tick runs one "pass" of every
// resident request: force at the current positions, then kick and drift.
// With S steps a request takes S + 1 passes (leapfrog with merged kicks):
//   pass 0       F(x0),  v += (h/2) F / m,  x += h v
//   pass 0<p<S   F(xp),  v += h F / m,      x += h v
//   pass S       F(xS),  v += (h/2) F / m   (no drift)
// which is the kick-drift-kick step with its end force reused by the next
// step, carried out S times.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sce {

// Largest n_max the batched kernels hold in registers; requests beyond it
// belong on a context of their own.
constexpr int kServeMaxN = 16;
// Particles per deposit segment (one partial sum per segment and row tile).
// 256 gave 2-3% more saturated capacity than 512 (shorter items at the end
// of a tick); 128 and 1,024 gave less.
constexpr int kServeSeg = 256;
// Doubles per force work item in the diagnostics partials.
constexpr int kServeFDiag = 12;
// Doubles per request of the diagnostics record: first pass [0..7], last pass [8..15]:
// K, W, sum q Phi, P_x, P_y, P_z, sum m|v|, max|rho|.
constexpr int kServeDiag = 16;

// n_z slots of a request's tables: n + 1 rounded to a kernel class (5, 9 or 17).
__host__ __device__ inline int serve_nz(int n) { return n <= 4 ? 5 : (n <= 8 ? 9 : 17); }

struct ReqDesc {
    int64_t N;
    int n, R, Rp, nzs;       // n_max, rows, rows rounded up to 64, n_z slots (serve_nz)
    int segs, rblocks, fblocks, shape;
    int dim;                 // 3, or 2: the n_x = 0 slice (rows 0..n), area L^2
    double L, invL, a, eps0, dt;
    int64_t pass, n_steps;   // pass: passes done (device-incremented at tick end)
    // byte offsets into the arena
    int64_t o_pos, o_vel, o_q, o_m, o_F, o_part, o_ftab, o_psi0, o_rpart, o_fpart, o_diag;
};

// Work item: x = slot, y = index within the request (see each kernel).
struct ServeItem {
    int slot, idx;
};

// Arena bytes a request needs; fills the offsets (relative to its base) and counts.
size_t serve_layout(ReqDesc &d, int elem_bytes);

// One tick: deposit, reduce + solve, force + kick + drift, diagnostics.
// elem_bytes 4 or 8 selects the working precision of phases and sums.  The
// grids have gdep, gred, gfrc and gslots blocks; counts (device, 4 ints)
// holds the numbers of valid items of each list, blocks beyond return.
hipError_t launch_serve_tick(hipStream_t s, int elem_bytes, const ReqDesc *desc, char *arena,
                             const ServeItem *dep, int gdep, const ServeItem *red, int gred,
                             const ServeItem *frc, int gfrc, const int *slots, int gslots,
                             const int *counts);

}  // namespace sce
