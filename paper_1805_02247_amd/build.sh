#!/bin/bash
# Builds libpmr.so (gfx950) next to this script. Usage: build.sh [extra hipcc flags]
set -euo pipefail
here="$(cd "$(dirname "${BASH_SOURCE[0]}")" && pwd)"
src="$here/csrc"
out="$here/libpmr.so"
tmp="$out.tmp$$"
flags=(--offload-arch=gfx950 -O3 -std=c++17 -fPIC -shared
       -Xclang -target-feature -Xclang -packed-fp32-ops
       -I"$here/../include" -I"$src")
hipcc "${flags[@]}" "$@" "$src/fft.hip" "$src/cic.hip" "$src/halo.hip" "$src/pmr.cpp" -o "$tmp"
mv -f "$tmp" "$out"
echo "built $out"
