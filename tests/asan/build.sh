#!/bin/bash
# AddressSanitizer build of the library's host code (device code unchanged:
# every -fsanitize= is given to the host pass only) and of the ABI driver.
# Usage: tests/asan/build.sh OUT_DIR
set -e
HERE=$(cd "$(dirname "$0")" && pwd)
SRC="$HERE/../../paper_2606_23274_amd/csrc"
OUT=${1:?out dir}
mkdir -p "$OUT"
HIPCC=${HIPCC:-/opt/rocm/bin/hipcc}
FLAGS="-O1 -g -std=c++17 -fPIC --offload-arch=gfx950 -Xclang -target-feature -Xclang -packed-fp32-ops
       -Xarch_host -fsanitize=address -Xarch_host -fno-omit-frame-pointer -Wno-unused-command-line-argument"
pids=()
for f in gemm linalg fitkern runtime; do
  $HIPCC $FLAGS -c "$SRC/$f.hip" -o "$OUT/$f.o" 2> "$OUT/$f.err" &
  pids+=($!)
done
for p in "${pids[@]}"; do wait "$p"; done
$HIPCC --offload-arch=gfx950 -shared -fPIC -Xarch_host -fsanitize=address -shared-libasan \
  -o "$OUT/libmpofit_asan.so" "$OUT"/gemm.o "$OUT"/linalg.o "$OUT"/fitkern.o "$OUT"/runtime.o
RT=$(dirname "$(ls /opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so | head -n 1)")
/opt/rocm/llvm/bin/clang -g -fsanitize=address -shared-libasan -fno-omit-frame-pointer \
  "$HERE/abi_driver.c" -o "$OUT/abi_driver" -L"$OUT" -lmpofit_asan -Wl,-rpath,"$OUT" -Wl,-rpath,"$RT"
