// RAII bracket of one kernel launch for the opt-in per-kernel timer.
#pragma once
#include <hip/hip_runtime.h>

#include <string>

namespace sj {

class ProfRange {
public:
    ProfRange(const char* name, hipStream_t s);
    ~ProfRange();
    ProfRange(const ProfRange&) = delete;
    ProfRange& operator=(const ProfRange&) = delete;

private:
    std::string name_;
    hipStream_t s_;
    void* a_;
};

}  // namespace sj
