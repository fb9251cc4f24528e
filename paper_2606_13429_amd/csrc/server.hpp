// Serving engine (continuous batching of solves that share a mesh); the
// opaque dcg_server of the C ABI.
#pragma once
#include <memory>
#include <string>

#include "runtime.hpp"

namespace dcg {

class Server {
 public:
  explicit Server(const dcg_options& opt);
  ~Server();
  Server(const Server&) = delete;
  Server& operator=(const Server&) = delete;

  // Builds (or finds) the mesh context of ``mesh`` on the server's device.
  void prepare(const dcg_mesh& mesh);
  // Queues a request; throws Error(DCG_EAGAIN) when max_pending requests are
  // unfinished.
  dcg_status submit(const dcg_mesh& mesh, double dt, double nu, const double* b, double* x,
                    double tol, uint64_t* ticket);
  // DCG_PENDING, or the terminal status (the ticket is then forgotten).
  dcg_status poll(uint64_t ticket, dcg_stats* st, std::string* err);
  void counters(int64_t* steps, int64_t* slot_steps) const;
  // Device bytes of one group of mesh size n (context + 16-slot workspace).
  static int64_t group_bytes(int n, bool fp32);

  struct Impl;

 private:
  std::unique_ptr<Impl> impl;
};

}  // namespace dcg

struct dcg_srv {
  std::unique_ptr<dcg::Server> server;
};
