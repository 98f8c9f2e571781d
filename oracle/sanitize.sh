#!/bin/bash
# Runs the oracle's CPU pins against a build of the oracle with AddressSanitizer and
# UndefinedBehaviorSanitizer (host code only; the sanitizer runtimes are preloaded into the
# Python process that loads the library).
set -e
cd "$(dirname "$0")/.."
export LF_ORACLE_SANITIZE=1
export ASAN_OPTIONS=detect_leaks=0:abort_on_error=1
export UBSAN_OPTIONS=print_stacktrace=1:halt_on_error=1
export LD_PRELOAD="$(gcc -print-file-name=libasan.so):$(gcc -print-file-name=libubsan.so)"
exec python -m pytest tests/test_oracle_*.py -q -p no:cacheprovider "$@"
