#!/bin/bash
# The oracle's CPU pins against an AddressSanitizer + UndefinedBehaviorSanitizer
# build of the oracle (a separate library in $TMPDIR; the in-tree one is not
# touched).  Usage: bash oracle/sanitize.sh [extra pytest arguments]
set -euo pipefail
here=$(cd "$(dirname "$0")" && pwd)
out="${TMPDIR:-/tmp}/liboracle_asan_ubsan.so"
gcc -O1 -g -fno-omit-frame-pointer -fsanitize=address,undefined -fno-sanitize-recover=undefined \
    -std=c11 -ffp-contract=off -D_DEFAULT_SOURCE -fopenmp -fPIC -shared -Wall -o "$out" "$here/dartray_oracle.c" -lm
cd "$here/.."
LD_PRELOAD="$(gcc -print-file-name=libasan.so) $(gcc -print-file-name=libubsan.so)" \
ASAN_OPTIONS=detect_leaks=0:abort_on_error=1 UBSAN_OPTIONS=print_stacktrace=1:halt_on_error=1 \
DARTRAY_ORACLE_LIB="$out" python -m pytest tests -m "not gpu" -q -p no:cacheprovider -k oracle "$@"
