#!/bin/bash
# The library's host code (argument and grid validation, table set-up, the
# C ABI) under AddressSanitizer + UndefinedBehaviorSanitizer: a separate build
# in $TMPDIR with the sanitizers on the host side only (the gfx950 device code
# is built as usual), driven by the ABI tests, which need no GPU.
# Usage: bash paper_1709_03802_amd/sanitize_host.sh
set -euo pipefail
pkg=$(cd "$(dirname "$0")" && pwd)
root=$(dirname "$pkg")
out="${TMPDIR:-/tmp}/libdartray_host_asan.so"
rt=$(ls /opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so | head -1)
/opt/rocm/bin/hipcc --offload-arch=gfx950 -O1 -g -std=c++17 -fPIC -shared \
    -Xclang -target-feature -Xclang -packed-fp32-ops \
    -Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined -Xarch_host -fno-omit-frame-pointer \
    -I "$root/include" -I "$pkg/csrc" -o "$out" "$pkg/csrc/dartray.hip"
cd "$root"
LD_PRELOAD="$rt" ASAN_OPTIONS=detect_leaks=0:abort_on_error=1 UBSAN_OPTIONS=print_stacktrace=1:halt_on_error=1 \
DARTRAY_LIB="$out" python -m pytest tests/test_abi.py -q -p no:cacheprovider "$@"
