// Optional library log on stderr, switched on by SP_LOG=1 in the
// environment: the launch configuration each entry point chooses, and the
// shot queue's admissions, compositions and retirements.  Off by default;
// the switch is read once per process.
#pragma once

namespace sp {

bool log_on();
void log_line(const char *fmt, ...) __attribute__((format(printf, 1, 2)));

}  // namespace sp
