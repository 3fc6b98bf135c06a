// Batches of independent trajectories (td_batch_* in tddftb.h): the probe
// trajectories of the pump-probe protocol (Sec. 5.1) stepped together.
//
// Each member is a full one-trajectory context (same buffers, ground
// state, kick and checkpoint code) on the batch's stream. A step of the
// batch runs every kernel of the density step (Sec. 2.3: charges,
// potential, H, the products S^-1 H and (S^-1 H)[Re rho | Im rho], the
// leapfrog update) once for all members, over device tables of work items
// (rows, atoms, product tiles, tile pairs). The two density buffers of each
// member alternate roles step by step, so the steps after the Euler start
// are two fixed launch sequences (even and odd parity), captured once as
// HIP graphs (one step, and runs of 16 steps) and replayed; a device step
// counter indexes the field and the dipole record, so the graphs need no
// per-step arguments.
//
// Product tiles: members are grouped in size buckets (padded n / 128); a
// bucket's products run as 128 x 128 or 64 x 64 tiles, chosen by timing
// both on that bucket's members at creation. 64 x 64 tiles cover only
// round_up(n, 64) rows and columns, and every product's K stops at
// round_up(n, 16): the padding is zero, so both give the solo result.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "../../include/tddftb.h"
#include "common.hpp"
#include "ctx.hpp"

using td::round_up;
using tdi::Fail;
using tdi::guarded;
using tdi::set_err;

struct td_batch {
  std::string err;
  int nm = 0;
  td_options opt{};
  uint32_t flags = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::vector<td_ctx*> mem;
  std::vector<double*> buf[2];    // the two density buffers of each member
  int parity = 0;                 // R[parity] holds the current density
  bool has_prev = false;
  int64_t step = 0;
  int last_n = 0;
  // device tables
  std::vector<td::BatchMember> mem_h;   // host copy of the member table
  td::BatchMember* mem_d = nullptr;
  td::BatchItem* rows_d = nullptr;
  td::BatchItem* atoms_d = nullptr;
  td::BatchPair* pairs_d = nullptr;
  int nrows = 0, natoms = 0, npairs = 0;
  // grouped products per tile variant v (0: 128, 1: 64) and parity p
  td::GemmProblem* g1_d[2] = {nullptr, nullptr};
  td::GemmProblem* g2_d[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  int g1_n[2] = {0, 0}, g1_tiles[2] = {0, 0};
  int g2_n[2] = {0, 0}, g2_tiles[2] = {0, 0};
  std::vector<int> bucket;        // per member
  int bucket_tile[TD_BATCH_BUCKETS] = {0};
  int bucket_members[TD_BATCH_BUCKETS] = {0};
  double bucket_ms[TD_BATCH_BUCKETS][2] = {{0}};
  // step inputs and outputs
  double* field = nullptr;
  double* dip = nullptr;
  int* kstep = nullptr;
  int cap = 0;
  hipGraphExec_t graph[2] = {nullptr, nullptr};       // one leapfrog step, by parity
  hipGraphExec_t graph_run[2] = {nullptr, nullptr};   // kGraphRun steps, by parity
  // moving nuclei: members of one system, grouped products per step phase
  bool ehr = false;
  tdi::EhrGroup eg;
};

namespace {

constexpr int kTiles[2] = {128, 64};
// Steps captured in one graph for long runs: one graph launch costs tens of
// microseconds, about a whole small-batch step, so runs of steps share it.
// Even, so a run returns the density buffers to the parity it started from.
constexpr int kGraphRun = 16;

template <class T>
void upload(td_batch* b, T** dst, const std::vector<T>& src) {
  if (*dst) HIPCHK(b, hipFree(*dst));
  *dst = nullptr;
  HIPCHK(b, hipMalloc((void**)dst, sizeof(T) * std::max<size_t>(src.size(), 1)));
  if (!src.empty())
    HIPCHK(b, hipMemcpyAsync(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice,
                             b->stream));
}

void drop_graphs(td_batch* b) {
  for (hipGraphExec_t* set : {b->graph, b->graph_run})
    for (int p = 0; p < 2; ++p) {
      if (set[p]) (void)hipGraphExecDestroy(set[p]);
      set[p] = nullptr;
    }
}

// Problems of the two products of member m for tile edge T and parity p.
void member_problems(td_batch* b, int m, int T, int p, std::vector<td::GemmProblem>* g1,
                     std::vector<td::GemmProblem>* g2) {
  const td_ctx* c = b->mem[m];
  const int np = c->np;
  const int mt = T == 128 ? np : std::min(np, round_up(c->n, T));
  const int K = round_up(c->n, 16);
  const int tiles = mt / T;
  if (g1) {
    td::GemmProblem q{};
    q.A = c->Sinv;
    q.B = c->H;
    q.C = c->A;
    q.lda = q.ldb = q.ldc = np;
    q.K = K;
    q.tiles_m = q.tiles_n = tiles;
    g1->push_back(q);
  }
  if (g2) {
    for (int half = 0; half < 2; ++half) {   // real columns, then imaginary columns
      td::GemmProblem q{};
      q.A = c->A;
      q.B = b->buf[p][m] + (size_t)half * np;
      q.C = c->X + (size_t)half * np;
      q.lda = np;
      q.ldb = q.ldc = 2 * np;
      q.K = K;
      q.tiles_m = q.tiles_n = tiles;
      g2->push_back(q);
    }
  }
}

int number_tiles(std::vector<td::GemmProblem>& v) {
  int t = 0;
  for (auto& q : v) {
    q.tile0 = t;
    t += q.tiles_m * q.tiles_n;
  }
  return t;
}

// Device tables of the products for the current bucket -> tile choice,
// and the columns of H each member's S^-1 H product reads.
void build_products(td_batch* b) {
  for (int m = 0; m < b->nm; ++m) {
    const td_ctx* c = b->mem[m];
    const int T = b->bucket_tile[b->bucket[m]];
    b->mem_h[m].hw = T == 128 ? c->np : std::min(c->np, round_up(c->n, T));
  }
  HIPCHK(b, hipMemcpyAsync(b->mem_d, b->mem_h.data(), sizeof(td::BatchMember) * b->mem_h.size(),
                           hipMemcpyHostToDevice, b->stream));
  for (int v = 0; v < 2; ++v) {
    std::vector<td::GemmProblem> g1, g2[2];
    for (int m = 0; m < b->nm; ++m) {
      if (b->bucket_tile[b->bucket[m]] != kTiles[v]) continue;
      member_problems(b, m, kTiles[v], 0, &g1, &g2[0]);
      member_problems(b, m, kTiles[v], 1, nullptr, &g2[1]);
    }
    b->g1_n[v] = (int)g1.size();
    b->g1_tiles[v] = number_tiles(g1);
    upload(b, &b->g1_d[v], g1);
    b->g2_n[v] = (int)g2[0].size();
    for (int p = 0; p < 2; ++p) {
      b->g2_tiles[v] = number_tiles(g2[p]);
      upload(b, &b->g2_d[v][p], g2[p]);
    }
  }
}

// Times the second product of each bucket's members with both tiles.
void tune_tiles(td_batch* b) {
  hipEvent_t e0, e1;
  HIPCHK(b, hipEventCreate(&e0));
  HIPCHK(b, hipEventCreate(&e1));
  struct Ev {
    hipEvent_t a, b;
    ~Ev() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } guard{e0, e1};
  td::GemmProblem* tmp = nullptr;
  struct Tmp {
    td::GemmProblem** p;
    ~Tmp() {
      if (*p) (void)hipFree(*p);
    }
  } tguard{&tmp};
  for (int k = 0; k < TD_BATCH_BUCKETS; ++k) {
    if (!b->bucket_members[k]) continue;
    double best = INFINITY;
    for (int v = 0; v < 2; ++v) {
      std::vector<td::GemmProblem> g2;
      for (int m = 0; m < b->nm; ++m)
        if (b->bucket[m] == k) member_problems(b, m, kTiles[v], b->parity, nullptr, &g2);
      const int tiles = number_tiles(g2);
      upload(b, &tmp, g2);
      HIPCHK(b, td::dgemm_grouped(b->stream, kTiles[v], tmp, (int)g2.size(), tiles));
      HIPCHK(b, hipEventRecord(e0, b->stream));
      constexpr int reps = 3;
      for (int r = 0; r < reps; ++r)
        HIPCHK(b, td::dgemm_grouped(b->stream, kTiles[v], tmp, (int)g2.size(), tiles));
      HIPCHK(b, hipEventRecord(e1, b->stream));
      HIPCHK(b, hipEventSynchronize(e1));
      float ms = 0.f;
      HIPCHK(b, hipEventElapsedTime(&ms, e0, e1));
      b->bucket_ms[k][v] = ms / reps;
      if (ms < best) {
        best = ms;
        b->bucket_tile[k] = kTiles[v];
      }
    }
  }
}

// One step of every member: density R[cur] -> R[cur ^ 1]. Euler start
// (base R[cur], dt) or leapfrog (base R[cur ^ 1], 2 dt).
void step_body(td_batch* b, int cur, bool euler) {
  hipStream_t s = b->stream;
  const int nxt = cur ^ 1;
  HIPCHK(b, td::batch_rowdot(s, b->mem_d, b->rows_d, b->nrows, cur));
  HIPCHK(b, td::batch_charges(s, b->mem_d, b->nm, b->kstep, b->dip, b->cap));
  HIPCHK(b, td::batch_potential(s, b->mem_d, b->atoms_d, b->natoms, b->field, b->kstep));
  HIPCHK(b, td::batch_assemble(s, b->mem_d, b->rows_d, b->nrows));
  for (int v = 0; v < 2; ++v)
    if (b->g1_n[v]) HIPCHK(b, td::dgemm_grouped(s, kTiles[v], b->g1_d[v], b->g1_n[v], b->g1_tiles[v]));
  for (int v = 0; v < 2; ++v)
    if (b->g2_n[v])
      HIPCHK(b, td::dgemm_grouped(s, kTiles[v], b->g2_d[v][cur], b->g2_n[v], b->g2_tiles[v]));
  HIPCHK(b, td::batch_leapfrog(s, b->mem_d, b->pairs_d, b->npairs, euler ? cur : nxt, nxt,
                               euler ? b->opt.dt : 2.0 * b->opt.dt));
  HIPCHK(b, td::batch_tick(s, b->kstep, 0));
}

// Captures `steps` leapfrog steps starting from parity `cur` into *out.
void capture(td_batch* b, int cur, int steps, hipGraphExec_t* out) {
  hipGraph_t g = nullptr;
  HIPCHK(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  try {
    for (int k = 0; k < steps; ++k) step_body(b, cur ^ (k & 1), false);
  } catch (...) {
    (void)hipStreamEndCapture(b->stream, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  HIPCHK(b, hipStreamEndCapture(b->stream, &g));
  hipError_t e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  HIPCHK(b, e);
}

// Member contexts mirror the batch state (current buffer, history, step).
void sync_members(td_batch* b) {
  for (int m = 0; m < b->nm; ++m) {
    td_ctx* c = b->mem[m];
    c->rho_cur = b->buf[b->parity][m];
    c->rho_prev = b->buf[b->parity ^ 1][m];
    c->has_prev = b->has_prev;
    c->step = b->step;
    c->last_n = 0;
  }
}

void refresh_members(td_batch* b) {
  HIPCHK(b, hipStreamSynchronize(b->stream));
  for (int m = 0; m < b->nm; ++m) {
    td_ctx* c = b->mem[m];
    try {
      tdi::refresh_ctx(c);
    } catch (const Fail& f) {
      b->err = "member " + std::to_string(m) + ": " + c->err;
      throw;
    }
  }
}

void free_batch(td_batch* b) {
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  drop_graphs(b);
  tdi::ehr_group_free(b->eg);
  void* bufs[] = {b->mem_d, b->rows_d, b->atoms_d, b->pairs_d, b->g1_d[0], b->g1_d[1],
                  b->g2_d[0][0], b->g2_d[0][1], b->g2_d[1][0], b->g2_d[1][1], b->field,
                  b->dip, b->kstep};
  for (void* p : bufs)
    if (p) (void)hipFree(p);
  for (td_ctx* c : b->mem) td_destroy(c);
  b->mem.clear();
  if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
  b->stream = nullptr;
}

void create_impl(td_batch* b, int n, const td_system* systems, const td_options* opt,
                 uint32_t flags) {
  REQUIRE(b, n >= 1 && systems && opt, TD_EINVAL, "need n >= 1, systems and options");
  REQUIRE(b, (flags & ~(TD_BATCH_NO_GRAPH | TD_BATCH_TILE_128 | TD_BATCH_TILE_64)) == 0,
          TD_EINVAL, "unknown batch flags");
  REQUIRE(b, !((flags & TD_BATCH_TILE_128) && (flags & TD_BATCH_TILE_64)), TD_EINVAL,
          "TD_BATCH_TILE_128 and TD_BATCH_TILE_64 exclude each other");
  REQUIRE(b, opt->precision == TD_FP64, TD_ENOTSUP, "batches run in TD_FP64 precision only");
  REQUIRE(b, opt->dt > 0 && std::isfinite(opt->dt), TD_EINVAL, "dt must be positive");
  for (int m = 0; m < n; ++m)
    REQUIRE(b, systems[m].plus_u == TD_PLUS_U_NONE, TD_ENOTSUP,
            "member " + std::to_string(m) + ": batches have no on-site corrections (plus_u)");
  b->nm = n;
  b->opt = *opt;
  b->flags = flags;
  if (opt->hip_stream) {
    b->stream = (hipStream_t)opt->hip_stream;
  } else {
    HIPCHK(b, hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
    b->own_stream = true;
  }
  td_options mo = *opt;
  mo.hip_stream = b->stream;
  mo.profile = 0;
  b->mem.reserve(n);
  for (int m = 0; m < n; ++m) {
    td_ctx* c = nullptr;
    char msg[512];
    const td_status st = td_create(&systems[m], &mo, &c, msg, sizeof(msg));
    if (st != TD_OK) {
      b->err = "member " + std::to_string(m) + ": " + msg;
      throw Fail{st};
    }
    b->mem.push_back(c);
    b->buf[0].push_back(c->rho_cur);
    b->buf[1].push_back(c->rho_prev);
  }
  // work tables
  std::vector<td::BatchMember> bm(n);
  std::vector<td::BatchItem> rows, atoms;
  std::vector<td::BatchPair> pairs;
  b->bucket.resize(n);
  for (int m = 0; m < n; ++m) {
    const td_ctx* c = b->mem[m];
    td::BatchMember& M = bm[m];
    M.S = c->S;
    M.H0 = c->H0;
    M.H = c->H;
    M.A = c->A;
    M.X = c->X;
    M.R[0] = b->buf[0][m];
    M.R[1] = b->buf[1][m];
    M.gamma = c->gamma;
    M.pos = c->pos;
    M.q0 = c->q0;
    M.orb_off = c->orb_off;
    M.q_orb = c->q_orb;
    M.dq = c->dq;
    M.v = c->v;
    M.vorb = c->vorb;
    M.np = c->np;
    M.na = c->na;
    M.kw = round_up(c->n, 16);
    M.hw = c->np;            // narrowed to the product's tile span once tiles are chosen
    // rows of the charges and of H: the products read H rows below K =
    // round_up(n, 16) only, and the charges use the rows of real orbitals
    for (int r = 0; r < M.kw; ++r) rows.push_back({m, r});
    for (int a = 0; a < c->na; ++a) atoms.push_back({m, a});
    const int nt = round_up(c->n, 32) / 32;   // tiles beyond n stay zero
    for (int i = 0; i < nt; ++i)
      for (int j = i; j < nt; ++j) pairs.push_back({m, i, j, 0});
    b->bucket[m] = std::min(c->np / 128 - 1, TD_BATCH_BUCKETS - 1);
    b->bucket_members[b->bucket[m]] += 1;
  }
  b->nrows = (int)rows.size();
  b->natoms = (int)atoms.size();
  b->npairs = (int)pairs.size();
  b->mem_h = bm;
  upload(b, &b->mem_d, bm);
  upload(b, &b->rows_d, rows);
  upload(b, &b->atoms_d, atoms);
  upload(b, &b->pairs_d, pairs);
  HIPCHK(b, hipMalloc((void**)&b->kstep, sizeof(int)));
  HIPCHK(b, td::batch_tick(b->stream, b->kstep, 1));
  if (flags & (TD_BATCH_TILE_128 | TD_BATCH_TILE_64)) {
    const int t = (flags & TD_BATCH_TILE_64) ? 64 : 128;
    for (int k = 0; k < TD_BATCH_BUCKETS; ++k) b->bucket_tile[k] = b->bucket_members[k] ? t : 0;
  } else {
    tune_tiles(b);
  }
  build_products(b);
  HIPCHK(b, hipStreamSynchronize(b->stream));
}

void ehr_step_impl(td_batch* b, int n, const double* field) {
  if (field) {
    if (b->cap < n) {
      if (b->field) HIPCHK(b, hipFree(b->field));
      b->field = nullptr;
      b->cap = 0;
      HIPCHK(b, hipMalloc((void**)&b->field, sizeof(double) * 3 * (size_t)n));
      b->cap = n;
    }
    HIPCHK(b, hipMemcpyAsync(b->field, field, sizeof(double) * 3 * n, hipMemcpyHostToDevice,
                             b->stream));
  }
  for (int m = 0; m < b->nm; ++m) {
    try {
      tdi::ensure_series_ctx(b->mem[m], n);
    } catch (const Fail&) {
      b->err = "member " + std::to_string(m) + ": " + b->mem[m]->err;
      throw;
    }
  }
  b->last_n = 0;
  tdi::ehr_batch_steps(b->mem, b->eg, n, field ? b->field : nullptr, b->err);
  b->step += n;
  b->has_prev = true;
  b->last_n = n;
}

void step_impl(td_batch* b, int n, const double* field) {
  REQUIRE(b, n >= 0, TD_EINVAL, "n must be >= 0");
  // the leapfrog limit of each member (Sec. 2.3, Eq. 19), as a solo td_step checks it
  for (int m = 0; m < b->nm; ++m) {
    const td_ctx* c = b->mem[m];
    if (!(c->info.stability < 1.0)) {
      b->err = "member " + std::to_string(m) + ": time step " + std::to_string(c->opt.dt) +
               " too large for the leapfrog: dt times the width of the spectrum of S^-1 H is " +
               std::to_string(c->info.stability) + " (must be below 1)";
      throw Fail{TD_EUNSTABLE};
    }
  }
  if (n == 0) {
    b->last_n = 0;     // an empty call records no dipoles
    return;
  }
  if (field) {
    for (size_t i = 0; i < 3 * (size_t)n; ++i)
      REQUIRE(b, std::isfinite(field[i]), TD_EINVAL, "non-finite field");
    // with the spread of the field's potential over each member's atoms
    for (int m = 0; m < b->nm; ++m) {
      const td_ctx* c = b->mem[m];
      const double spread = tdi::field_spread(c, field, n);
      const double st = c->opt.dt * (c->info.width_estimate + spread);
      if (!(st < 1.0)) {
        b->err = "member " + std::to_string(m) + ": time step " + std::to_string(c->opt.dt) +
                 " too large for the leapfrog under this field: dt times the width of the "
                 "spectrum of S^-1 H plus the spread of R . E over the atoms is " +
                 std::to_string(st) + " (must be below 1)";
        throw Fail{TD_EUNSTABLE};
      }
    }
  }
  if (b->ehr) {
    ehr_step_impl(b, n, field);
    return;
  }
  if (b->cap < n) {
    drop_graphs(b);   // the graphs hold the old buffers
    if (b->field) HIPCHK(b, hipFree(b->field));
    if (b->dip) HIPCHK(b, hipFree(b->dip));
    b->field = b->dip = nullptr;
    b->cap = 0;
    HIPCHK(b, hipMalloc((void**)&b->field, sizeof(double) * 3 * (size_t)n));
    HIPCHK(b, hipMalloc((void**)&b->dip, sizeof(double) * 3 * (size_t)n * b->nm));
    b->cap = n;
  }
  if (field)
    HIPCHK(b, hipMemcpyAsync(b->field, field, sizeof(double) * 3 * n, hipMemcpyHostToDevice,
                             b->stream));
  else
    HIPCHK(b, hipMemsetAsync(b->field, 0, sizeof(double) * 3 * n, b->stream));
  HIPCHK(b, td::batch_tick(b->stream, b->kstep, 1));
  const bool use_graph = !(b->flags & TD_BATCH_NO_GRAPH);
  b->last_n = 0;
  for (int k = 0; k < n;) {
    if (!b->has_prev) {
      step_body(b, b->parity, true);
      b->has_prev = true;
    } else if (use_graph && n - k >= kGraphRun) {
      if (!b->graph_run[b->parity]) capture(b, b->parity, kGraphRun, &b->graph_run[b->parity]);
      HIPCHK(b, hipGraphLaunch(b->graph_run[b->parity], b->stream));
      b->step += kGraphRun;        // even: the parity is unchanged
      k += kGraphRun;
      continue;
    } else if (use_graph) {
      if (!b->graph[b->parity]) capture(b, b->parity, 1, &b->graph[b->parity]);
      HIPCHK(b, hipGraphLaunch(b->graph[b->parity], b->stream));
    } else {
      step_body(b, b->parity, false);
    }
    b->parity ^= 1;
    b->step += 1;
    ++k;
  }
  b->last_n = n;
  sync_members(b);
  refresh_members(b);
}

void kick_impl(td_batch* b, const double* e0, const double* dir) {
  REQUIRE(b, e0 && dir, TD_EINVAL, "e0 and dir must not be null");
  if (!b->ehr) sync_members(b);
  for (int m = 0; m < b->nm; ++m) {
    const td_status st = td_kick(b->mem[m], e0[m], dir + 3 * (size_t)m);
    if (st != TD_OK) {
      b->err = "member " + std::to_string(m) + ": " + td_last_error(b->mem[m]);
      throw Fail{st};
    }
  }
  b->has_prev = false;
  if (!b->ehr) sync_members(b);
}

// Members of one system with their own nuclear velocities: member 0 solves
// the ground state (unless sys->rho0 is given), the others start from its
// density; all run on the batch's stream.
void create_ehr_impl(td_batch* b, int n, const td_system* sys, const td_model* model,
                     const double* velocities, const td_options* opt) {
  REQUIRE(b, n >= 1 && sys && model && opt, TD_EINVAL, "need n >= 1, system, model and options");
  REQUIRE(b, opt->dt > 0 && std::isfinite(opt->dt), TD_EINVAL, "dt must be positive");
  b->nm = n;
  b->opt = *opt;
  b->ehr = true;
  b->flags = TD_BATCH_NO_GRAPH;
  if (opt->hip_stream) {
    b->stream = (hipStream_t)opt->hip_stream;
  } else {
    HIPCHK(b, hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
    b->own_stream = true;
  }
  td_options mo = *opt;
  mo.hip_stream = b->stream;
  mo.profile = 0;
  const size_t na3 = 3 * (size_t)sys->n_atoms;
  std::vector<double> rho0;
  td_system s = *sys;
  b->mem.reserve(n);
  for (int m = 0; m < n; ++m) {
    td_ctx* c = nullptr;
    char msg[512];
    const td_status st = td_create_ehrenfest(&s, model, velocities ? velocities + m * na3 : nullptr,
                                             &mo, &c, msg, sizeof(msg));
    if (st != TD_OK) {
      b->err = "member " + std::to_string(m) + ": " + msg;
      throw Fail{st};
    }
    b->mem.push_back(c);
    if (m == 0 && !sys->rho0) {
      const size_t n2 = (size_t)sys->n_orb * sys->n_orb;
      rho0.resize(2 * n2);
      int64_t step = 0;
      int32_t hp = 0;
      const td_status g = td_get_rho(c, rho0.data(), nullptr, &step, &hp);
      if (g != TD_OK) {
        b->err = std::string("member 0: ") + td_last_error(c);
        throw Fail{g};
      }
      s.rho0 = rho0.data();
    }
  }
  tdi::ehr_group_alloc(b->mem[0], b->eg, n);
  HIPCHK(b, hipStreamSynchronize(b->stream));
}

void check_member(td_batch* b, int m) {
  REQUIRE(b, m >= 0 && m < b->nm, TD_EINVAL, "member index out of range");
}

td_status member_call(td_batch* b, int m, td_status st) {
  if (st != TD_OK) b->err = "member " + std::to_string(m) + ": " + td_last_error(b->mem[m]);
  return st;
}

}  // namespace

extern "C" {

td_status td_batch_create(int32_t n, const td_system* systems, const td_options* opt,
                          uint32_t flags, td_batch** out, char* err, int32_t errlen) {
  if (!out) {
    set_err(err, errlen, "out must not be null");
    return TD_EINVAL;
  }
  *out = nullptr;
  td_batch* b = new (std::nothrow) td_batch();
  if (!b) {
    set_err(err, errlen, "host allocation failed");
    return TD_ENOMEM;
  }
  const td_status st = guarded(b, [&] { create_impl(b, n, systems, opt, flags); });
  if (st != TD_OK) {
    set_err(err, errlen, b->err);
    free_batch(b);
    delete b;
    return st;
  }
  set_err(err, errlen, "");
  *out = b;
  return TD_OK;
}

td_status td_batch_kick(td_batch* b, const double* e0, const double* dir) {
  return guarded(b, [&] { kick_impl(b, e0, dir); });
}

td_status td_batch_step(td_batch* b, int32_t n, const double* field) {
  return guarded(b, [&] { step_impl(b, n, field); });
}

td_status td_batch_get_dipole_series(td_batch* b, int32_t member, double* mu, int32_t cap,
                                     int32_t* n_out) {
  return guarded(b, [&] {
    check_member(b, member);
    REQUIRE(b, n_out && cap >= 0 && (mu || cap == 0), TD_EINVAL, "invalid output");
    if (b->ehr) {
      const td_status st = td_get_dipole_series(b->mem[member], mu, cap, n_out);
      if (st != TD_OK) {
        b->err = "member " + std::to_string(member) + ": " + td_last_error(b->mem[member]);
        throw Fail{st};
      }
      return;
    }
    const int k = std::min(cap, b->last_n);
    if (k > 0)
      HIPCHK(b, hipMemcpyAsync(mu, b->dip + (size_t)member * b->cap * 3, sizeof(double) * 3 * k,
                               hipMemcpyDeviceToHost, b->stream));
    HIPCHK(b, hipStreamSynchronize(b->stream));
    *n_out = b->last_n;
  });
}

td_status td_batch_get_charges(td_batch* b, int32_t member, double* dq) {
  td_status st = guarded(b, [&] { check_member(b, member); });
  if (st != TD_OK) return st;
  return member_call(b, member, td_get_charges(b->mem[member], dq));
}

td_status td_batch_get_rho(td_batch* b, int32_t member, double* rho, double* rho_prev,
                           int64_t* step, int32_t* has_prev) {
  td_status st = guarded(b, [&] {
    check_member(b, member);
    if (!b->ehr) sync_members(b);
  });
  if (st != TD_OK) return st;
  return member_call(b, member, td_get_rho(b->mem[member], rho, rho_prev, step, has_prev));
}

td_status td_batch_get_info(td_batch* b, td_batch_info* info) {
  return guarded(b, [&] {
    REQUIRE(b, info, TD_EINVAL, "null output");
    *info = td_batch_info{};
    info->n_members = b->nm;
    info->step = b->step;
    info->has_prev = b->has_prev ? 1 : 0;
    info->graph = (b->flags & TD_BATCH_NO_GRAPH) ? 0 : 1;
    for (int k = 0; k < TD_BATCH_BUCKETS; ++k) {
      info->bucket_members[k] = b->bucket_members[k];
      info->bucket_tile[k] = b->bucket_tile[k];
      info->bucket_ms[k][0] = b->bucket_ms[k][0];
      info->bucket_ms[k][1] = b->bucket_ms[k][1];
    }
  });
}

td_status td_batch_create_ehrenfest(int32_t n, const td_system* sys, const td_model* model,
                                    const double* velocities, const td_options* opt,
                                    td_batch** out, char* err, int32_t errlen) {
  if (!out) {
    set_err(err, errlen, "out must not be null");
    return TD_EINVAL;
  }
  *out = nullptr;
  td_batch* b = new (std::nothrow) td_batch();
  if (!b) {
    set_err(err, errlen, "host allocation failed");
    return TD_ENOMEM;
  }
  const td_status st = guarded(b, [&] { create_ehr_impl(b, n, sys, model, velocities, opt); });
  if (st != TD_OK) {
    set_err(err, errlen, b->err);
    free_batch(b);
    delete b;
    return st;
  }
  set_err(err, errlen, "");
  *out = b;
  return TD_OK;
}

td_status td_batch_get_nuclei(td_batch* b, int32_t member, double* positions, double* velocities) {
  td_status st = guarded(b, [&] {
    check_member(b, member);
    REQUIRE(b, b->ehr, TD_ENOTSUP, "clamped-nuclei batch: no nuclear state");
  });
  if (st != TD_OK) return st;
  return member_call(b, member, td_get_nuclei(b->mem[member], positions, velocities));
}

td_status td_batch_get_energy_series(td_batch* b, int32_t member, double* e_el, double* e_kin,
                                     int32_t cap, int32_t* n_out) {
  td_status st = guarded(b, [&] {
    check_member(b, member);
    REQUIRE(b, b->ehr, TD_ENOTSUP, "clamped-nuclei batch: no energy series");
  });
  if (st != TD_OK) return st;
  return member_call(b, member, td_get_energy_series(b->mem[member], e_el, e_kin, cap, n_out));
}

const char* td_batch_last_error(const td_batch* b) { return b ? b->err.c_str() : "null batch"; }

void td_batch_destroy(td_batch* b) {
  if (!b) return;
  free_batch(b);
  delete b;
}

}  // extern "C"
