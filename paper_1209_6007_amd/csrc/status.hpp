// Status codes shared by the host modules (values fixed by the public header).
#pragma once
#include "shatterbc.h"
