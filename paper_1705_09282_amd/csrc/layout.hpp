// Constants of the stencil-ELL matrix layout shared by the host setup and
// the residual kernel.
#pragma once

namespace dfmg {

// Slots of a row are stored in chunks of kEllVec consecutive values, so one
// lane reads a chunk with one vector load.
constexpr int kEllVec = 4;

// Subdomains with at most this many DOFs (the interior ones) are solved by
// one thread each in smoother variant 4; the others one entry per thread.
constexpr int kSmallPatch = 8;

}  // namespace dfmg
