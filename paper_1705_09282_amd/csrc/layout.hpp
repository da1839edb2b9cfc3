// Constants of the stencil-ELL matrix layout shared by the host setup and
// the residual kernel.
#pragma once

namespace dfmg {

// Slots of a row are stored in chunks of kEllVec consecutive values, so one
// lane reads a chunk with one vector load.
constexpr int kEllVec = 4;

}  // namespace dfmg
