// Device back end of the dense setup steps (rocSOLVER / rocBLAS); see
// DenseBackend in host.hpp for what each step computes.
#pragma once
#include "host.hpp"

namespace smpm {

struct DeviceDense;
// always: take the device path for every supported step whatever its size
// (the default takes it from a few GFLOP of work on).
DeviceDense *device_dense_create(bool always);
void device_dense_destroy(DeviceDense *dd);
const DenseBackend *device_dense_backend(const DeviceDense *dd);

}  // namespace smpm
