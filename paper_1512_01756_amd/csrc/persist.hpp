// Saving and loading the host tables of a handle.
#pragma once
#include <cstdint>
#include <vector>

#include "host.hpp"

namespace smpm {

struct TableHeader {
  int32_t nsys = 0;
  int32_t zlabel = 0;   // deflation space the tables were built for
  int32_t my = 0;       // > 0: a Fourier handle over m_y planes of length ly
  int32_t pad = 0;
  double ly = 0.0;
};

// Throw std::runtime_error / std::invalid_argument with a message on failure.
void save_tables(const char *path, const TableHeader &h, const std::vector<System> &sys);
void load_tables(const char *path, TableHeader &h, std::vector<System> &sys);

}  // namespace smpm
