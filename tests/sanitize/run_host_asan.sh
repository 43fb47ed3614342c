#!/bin/bash
# AddressSanitizer + UndefinedBehaviorSanitizer run of the host code (CPU only,
# no GPU needed; run from the repository root after building the library):
#   1. the CPU oracle, driven through every entry point by oracle_driver.c;
#   2. the library's host translation units (argument validation, pattern
#      expansion, pure-state parameters, batch schedules, the device-less error
#      paths) compiled with the sanitizers on the host side only, linked with
#      the regular kernel objects of paper_2010_15595_amd/_build, and the host
#      C-ABI tests (tests/test_abi_host.py) run against that build.
# Any sanitizer report fails the run.
set -euo pipefail
ROOT=$(cd "$(dirname "$0")/../.." && pwd)
OUT=${1:-/tmp/gbs_host_asan}
mkdir -p "$OUT"
HIPCC=/opt/rocm/bin/hipcc
CXX=/opt/rocm/llvm/bin/clang++
ASAN_RT=$(ls /opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so | head -n 1)

echo "== oracle under gcc ASan/UBSan"
gcc -O1 -g -fsanitize=address,undefined -fno-sanitize-recover=all -fno-omit-frame-pointer -fopenmp \
    -ffp-contract=off -o "$OUT/oracle_driver" "$ROOT/tests/sanitize/oracle_driver.c" "$ROOT/oracle/lhaf_oracle.c" -lm
"$OUT/oracle_driver"

echo "== host library under clang ASan/UBSan"
FLAGS=(-O1 -g -std=c++17 -fPIC --offload-arch=gfx950 -I "$ROOT/include" -fno-omit-frame-pointer
       -Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined -Xarch_host -fno-sanitize-recover=all
       -Xclang -target-feature -Xclang -packed-fp32-ops -Wno-unused-value)
for f in gbs_host gbs_batch gbs_sampler; do
    "$HIPCC" -x hip --cuda-host-only "${FLAGS[@]}" -c "$ROOT/paper_2010_15595_amd/csrc/$f.cpp" -o "$OUT/$f.o"
done
"$HIPCC" -x hip "${FLAGS[@]}" -c "$ROOT/paper_2010_15595_amd/csrc/gbs_noalloc.cpp" -o "$OUT/gbs_noalloc.o"
KOBJ=()
for f in charpoly_l88 charpoly_l84 charpoly_l44 lhaf_kernels sampler_kernels lhaf_lds; do
    KOBJ+=("$ROOT/paper_2010_15595_amd/_build/$f.hip.o")
done
"$CXX" -shared -fPIC -fsanitize=address,undefined -shared-libsan "$OUT"/gbs_*.o "${KOBJ[@]}" \
    -L/opt/rocm/lib -lamdhip64 -Wl,-rpath,/opt/rocm/lib -o "$OUT/libgbs_lhaf_asan.so"
cd "$ROOT"
LD_PRELOAD="$ASAN_RT" ASAN_OPTIONS=detect_leaks=0:halt_on_error=1 UBSAN_OPTIONS=halt_on_error=1:print_stacktrace=1 \
    GBS_LIB_PATH="$OUT/libgbs_lhaf_asan.so" python -m pytest tests/test_abi_host.py -q -p no:cacheprovider
echo "host sanitizer run clean"
