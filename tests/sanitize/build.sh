#!/bin/bash
# Build tests/sanitize/host_driver.cpp against the library's sources with
# AddressSanitizer and UndefinedBehaviorSanitizer on the host code only (each
# -fsanitize is passed through -Xarch_host; the device code is built as
# usual and never launched by the driver).  Usage: build.sh OUTDIR
set -euo pipefail
here="$(cd "$(dirname "$0")" && pwd)"
root="$(cd "$here/../.." && pwd)"
out="$1"
mkdir -p "$out"
csrc="$root/paper_2008_07140_amd/csrc"
hipcc="${HIPCC:-/opt/rocm/bin/hipcc}"
flags=(-O1 -g -std=c++17 -fno-omit-frame-pointer -Xarch_host -fsanitize=address,undefined
       -Xarch_host -fno-sanitize-recover=undefined -I "$root/include" -I "$csrc")
objs=()
pids=()
for f in "$csrc"/*.hip; do
    o="$out/$(basename "$f").o"
    "$hipcc" --offload-arch=gfx950 -Xclang -target-feature -Xclang -packed-fp32-ops "${flags[@]}" -x hip \
        -c "$f" -o "$o" 2> "$o.log" & pids+=($!)
    objs+=("$o")
done
for f in "$csrc"/*.cpp "$here/host_driver.cpp"; do
    o="$out/$(basename "$f").o"
    "$hipcc" "${flags[@]}" -D__HIP_PLATFORM_AMD__ -I "${ROCM_PATH:-/opt/rocm}/include" -x c++ -c "$f" -o "$o" 2> "$o.log" & pids+=($!)
    objs+=("$o")
done
for p in "${pids[@]}"; do wait "$p"; done
"$hipcc" --offload-arch=gfx950 -Xarch_host -fsanitize=address,undefined -o "$out/host_driver" "${objs[@]}"
