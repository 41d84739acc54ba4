// Host-only mock of hip_ext.h: the extension launch is declared with the rest of the mock.
#pragma once
#include "hip_runtime.h"
