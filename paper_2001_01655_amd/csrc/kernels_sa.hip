// Setup kernels of smoothed aggregation (strength, aggregation, prolongators).
#include "tm_device.h"

namespace tmi {}  // namespace tmi
