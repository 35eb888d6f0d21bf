#!/bin/bash
# The CPU test suite against the host-side AddressSanitizer + UndefinedBehaviorSanitizer
# build of the library (device code uninstrumented; no GPU needed):
#   python paper_2310_16668_amd/_build.py --sanitize && bash tests/run_sanitized.sh
set -e
cd "$(dirname "$0")/.."
ASAN_RT=$(/opt/rocm/bin/hipcc -print-file-name=libclang_rt.asan-x86_64.so)
export SKELFMM_LIB="$PWD/paper_2310_16668_amd/libskelfmm_san.so"
# python itself is not instrumented: leaks at exit are not the library's; any
# other report aborts the run
export ASAN_OPTIONS=detect_leaks=0:abort_on_error=1:halt_on_error=1
export UBSAN_OPTIONS=halt_on_error=1:print_stacktrace=1
LD_PRELOAD="$ASAN_RT" python -m pytest tests -x -q -m "not gpu" -p no:cacheprovider "$@"
