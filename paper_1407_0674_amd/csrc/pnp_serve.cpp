// Serving layer of the cDFT excess-chemical-potential library: resident
// sessions in a caller-owned device pool, admitted under its byte budget and
// stepped together through the batched evaluation.
//
// A session is one PNP-style state: densities rho_i(r) that stay on the
// device, their beta mu_ex and Slotboom factors, and the evaluation's
// workspace.  One step evaluates beta mu_ex of every listed session (equal
// grid sizes share every launch, see pnp_batch_mu_ex) and then moves each
// session's densities by the relaxation of Sec. 3.2 toward the equilibrium
// of the new mu_ex (pnp_relax_densities).
//
// The pool sub-allocates sessions first-fit from one device range and
// coalesces free blocks on release; admission fails with PNP_E_BUDGET when
// no free block is large enough.  With captured steps switched on
// (pnp_pool_graphs) a step whose id list was seen before replays the graph
// captured for it (pnp_plan_*).  Only host bookkeeping lives here: every
// device operation goes through the public entry points or a stream-ordered
// copy.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstring>
#include <list>
#include <map>
#include <string>
#include <vector>

#include "pnp_cdft.h"

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Session {
  pnp_grid grid{};
  int32_t S = 0;
  std::vector<pnp_species> species;
  double T = 0;
  pnp_params params{};
  std::vector<double> sw_eps, sw_rout;  // owned copies behind params' pointers
  std::vector<double> mu_bulk;
  double lambda = 0, clip = 0;
  size_t offset = 0, bytes = 0;
  double *rho = nullptr, *mu = nullptr, *slot = nullptr;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  int64_t steps = 0;
  int32_t status = PNP_OK;
};

}  // namespace

struct pnp_pool_s {
  pnp_ctx ctx = nullptr;
  char* base = nullptr;
  size_t bytes = 0;
  std::map<size_t, size_t> free_blocks;  // offset -> length, disjoint, coalesced
  std::map<int64_t, Session> sessions;
  int64_t next_id = 1;
  size_t used = 0;
  // captured steps, keyed by the exact id list, least recently used first
  int32_t max_plans = 0;
  std::list<std::pair<std::vector<int64_t>, pnp_plan>> plans;

  void drop_plans_with(int64_t id) {
    for (auto it = plans.begin(); it != plans.end();) {
      if (std::find(it->first.begin(), it->first.end(), id) != it->first.end()) {
        pnp_plan_destroy(it->second);
        it = plans.erase(it);
      } else {
        ++it;
      }
    }
  }
  void drop_all_plans() {
    for (auto& kv : plans) pnp_plan_destroy(kv.second);
    plans.clear();
  }

  bool take(size_t need, size_t& off) {
    for (auto it = free_blocks.begin(); it != free_blocks.end(); ++it) {
      if (it->second >= need) {
        off = it->first;
        const size_t rest = it->second - need;
        free_blocks.erase(it);
        if (rest) free_blocks[off + need] = rest;
        used += need;
        return true;
      }
    }
    return false;
  }
  void give(size_t off, size_t len) {
    used -= len;
    auto it = free_blocks.emplace(off, len).first;
    auto nx = std::next(it);
    if (nx != free_blocks.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_blocks.erase(nx);
    }
    if (it != free_blocks.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_blocks.erase(it);
      }
    }
  }
};

namespace {

pnp_status session_layout(pnp_ctx ctx, const pnp_grid* g, int32_t S, const pnp_params* p, size_t* field_bytes,
                          size_t* ws_bytes, size_t* total) {
  if (!g || !p) return PNP_E_ARG;
  pnp_params q = *p;
  q.per_term = 0;
  size_t ws = 0;
  const pnp_status st = pnp_workspace_bytes(ctx, g, S, &q, &ws);
  if (st != PNP_OK) return st;
  const size_t n3 = (size_t)g->nx * g->ny * g->nz;
  const size_t fb = align_up(sizeof(double) * (size_t)S * n3);
  *field_bytes = fb;
  *ws_bytes = align_up(ws);
  *total = 3 * fb + *ws_bytes;
  return PNP_OK;
}

}  // namespace

extern "C" {

pnp_status pnp_session_bytes(pnp_ctx ctx, const pnp_grid* grid, int32_t S, const pnp_params* params,
                             size_t* bytes) {
  if (!ctx || !bytes) return PNP_E_ARG;
  size_t fb, wb;
  return session_layout(ctx, grid, S, params, &fb, &wb, bytes);
}

pnp_status pnp_pool_create(pnp_ctx ctx, void* arena, size_t arena_bytes, pnp_pool* out) {
  if (!ctx || !out || !arena || arena_bytes < kAlign || ((uintptr_t)arena % kAlign)) return PNP_E_ARG;
  pnp_pool p = new pnp_pool_s();
  p->ctx = ctx;
  p->base = (char*)arena;
  p->bytes = arena_bytes / kAlign * kAlign;
  p->free_blocks[0] = p->bytes;
  *out = p;
  return PNP_OK;
}

void pnp_pool_destroy(pnp_pool pool) {
  if (!pool) return;
  pool->drop_all_plans();
  delete pool;
}

pnp_status pnp_pool_graphs(pnp_pool pool, int32_t max_plans) {
  if (!pool || max_plans < 0) return PNP_E_ARG;
  pool->max_plans = max_plans;
  while ((int32_t)pool->plans.size() > max_plans) {
    pnp_plan_destroy(pool->plans.front().second);
    pool->plans.pop_front();
  }
  return PNP_OK;
}

pnp_status pnp_pool_usage(pnp_pool pool, size_t* used, size_t* largest_free, int32_t* sessions) {
  if (!pool) return PNP_E_ARG;
  size_t big = 0;
  for (const auto& kv : pool->free_blocks) big = kv.second > big ? kv.second : big;
  if (used) *used = pool->used;
  if (largest_free) *largest_free = big;
  if (sessions) *sessions = (int32_t)pool->sessions.size();
  return PNP_OK;
}

pnp_status pnp_session_open(pnp_pool pool, const pnp_grid* grid, int32_t S, const pnp_species* species,
                            double T, const pnp_params* params, const double* rho0, const double* mu_bulk,
                            double lambda, double clip, void* stream, int64_t* id) {
  if (!pool || !grid || !species || !params || !rho0 || !id) return PNP_E_ARG;
  if (S < 1 || S > 8 || !(lambda >= 0.0 && lambda <= 1.0) || clip != clip) return PNP_E_ARG;
  if (params->per_term) return PNP_E_ARG;
  size_t fb, wb, total;
  pnp_status st = session_layout(pool->ctx, grid, S, params, &fb, &wb, &total);
  if (st != PNP_OK) return st;
  Session s;
  s.grid = *grid;
  s.S = S;
  s.species.assign(species, species + S);
  s.T = T;
  s.params = *params;
  s.params.flags = 0;
  if (params->sw_eps) {
    s.sw_eps.assign(params->sw_eps, params->sw_eps + (size_t)S * S);
    s.params.sw_eps = s.sw_eps.data();
  }
  if (params->sw_rout) {
    s.sw_rout.assign(params->sw_rout, params->sw_rout + (size_t)S * S);
    s.params.sw_rout = s.sw_rout.data();
  }
  s.mu_bulk.resize(S);
  if (mu_bulk) {
    s.mu_bulk.assign(mu_bulk, mu_bulk + S);
  } else {
    st = pnp_bulk_mu_ex(pool->ctx, S, species, T, &s.params, s.mu_bulk.data());
    if (st != PNP_OK) return st;
  }
  s.lambda = lambda;
  s.clip = clip;
  size_t off;
  if (!pool->take(total, off)) return PNP_E_BUDGET;
  s.offset = off;
  s.bytes = total;
  char* b = pool->base + off;
  s.rho = (double*)b;
  s.mu = (double*)(b + fb);
  s.slot = (double*)(b + 2 * fb);
  s.ws = b + 3 * fb;
  s.ws_bytes = wb;
  const size_t n3 = (size_t)grid->nx * grid->ny * grid->nz;
  if (hipMemcpyAsync(s.rho, rho0, sizeof(double) * (size_t)S * n3, hipMemcpyDeviceToDevice,
                     (hipStream_t)stream) != hipSuccess) {
    pool->give(off, total);
    return PNP_E_DEVICE;
  }
  const int64_t sid = pool->next_id++;
  pool->sessions.emplace(sid, std::move(s));
  *id = sid;
  return PNP_OK;
}

pnp_status pnp_session_step(pnp_pool pool, int32_t count, const int64_t* ids, int32_t* status, void* stream) {
  if (!pool || count < 0 || (count > 0 && (!ids || !status))) return PNP_E_ARG;
  std::vector<Session*> ss(count);
  for (int32_t k = 0; k < count; ++k) {
    auto it = pool->sessions.find(ids[k]);
    if (it == pool->sessions.end()) return PNP_E_ARG;
    ss[k] = &it->second;
  }
  std::vector<pnp_request> reqs(count);
  for (int32_t k = 0; k < count; ++k) {
    Session& s = *ss[k];
    pnp_request& r = reqs[k];
    std::memset(&r, 0, sizeof(r));
    r.grid = s.grid;
    r.S = s.S;
    r.species = s.species.data();
    r.rho = s.rho;
    r.T = s.T;
    r.params = &s.params;
    r.mu_ex = s.mu;
    r.slotboom = s.slot;
    r.workspace = s.ws;
    r.workspace_bytes = s.ws_bytes;
  }
  if (pool->max_plans > 0 && count > 0) {
    // captured step: evaluation and update replayed as one graph
    const std::vector<int64_t> key(ids, ids + count);
    auto hit = pool->plans.end();
    for (auto it = pool->plans.begin(); it != pool->plans.end(); ++it)
      if (it->first == key) hit = it;
    pnp_plan plan = nullptr;
    if (hit != pool->plans.end()) {
      plan = hit->second;
      pool->plans.splice(pool->plans.end(), pool->plans, hit);  // most recently used
    } else {
      std::vector<pnp_relax_spec> rx(count);
      for (int32_t k = 0; k < count; ++k) rx[k] = pnp_relax_spec{ss[k]->mu_bulk.data(), ss[k]->lambda, ss[k]->clip};
      pnp_status st = pnp_plan_create(pool->ctx, count, reqs.data(), rx.data(), &plan);
      if (st != PNP_OK) return st;
      if ((int32_t)pool->plans.size() >= pool->max_plans) {
        pnp_plan_destroy(pool->plans.front().second);
        pool->plans.pop_front();
      }
      pool->plans.emplace_back(key, plan);
    }
    pnp_status st = pnp_plan_launch(plan, stream);
    if (st == PNP_OK) st = pnp_plan_status(plan, stream, status);
    if (st != PNP_OK) return st;
    for (int32_t k = 0; k < count; ++k) {
      ss[k]->status = status[k];
      if (status[k] == PNP_OK) ++ss[k]->steps;
    }
    return PNP_OK;
  }
  pnp_status st = pnp_batch_mu_ex(pool->ctx, count, reqs.data(), stream);
  if (st != PNP_OK) return st;
  for (int32_t k = 0; k < count; ++k) {
    Session& s = *ss[k];
    status[k] = reqs[k].status;
    s.status = reqs[k].status;
    if (reqs[k].status != PNP_OK) continue;
    st = pnp_relax_densities(pool->ctx, &s.grid, s.S, s.species.data(), s.rho, s.mu, s.mu_bulk.data(), s.lambda,
                             s.clip, stream);
    if (st != PNP_OK) return st;
    ++s.steps;
  }
  return PNP_OK;
}

pnp_status pnp_session_view(pnp_pool pool, int64_t id, double** rho, double** mu_ex, double** slotboom,
                            int64_t* steps) {
  if (!pool) return PNP_E_ARG;
  auto it = pool->sessions.find(id);
  if (it == pool->sessions.end()) return PNP_E_ARG;
  if (rho) *rho = it->second.rho;
  if (mu_ex) *mu_ex = it->second.mu;
  if (slotboom) *slotboom = it->second.slot;
  if (steps) *steps = it->second.steps;
  return PNP_OK;
}

pnp_status pnp_session_close(pnp_pool pool, int64_t id) {
  if (!pool) return PNP_E_ARG;
  auto it = pool->sessions.find(id);
  if (it == pool->sessions.end()) return PNP_E_ARG;
  pool->drop_plans_with(id);
  pool->give(it->second.offset, it->second.bytes);
  pool->sessions.erase(it);
  return PNP_OK;
}

}  // extern "C"
